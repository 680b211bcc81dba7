"""The allocation-free entry point (tpcca_track_async_noalloc) against
tpcca_track_async, through the C ABI, on two calls in a row (the second with a
smaller input, so the static scratch array still holds the first call's
contents), and its size limit."""
import numpy as np
import pytest

import synth
from gpu_util import log, tracks_equal

pytestmark = pytest.mark.gpu


def _run(fn, dc, out, torch):
    counts = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    fn(dc, out, counts, status)
    torch.cuda.synchronize()
    c = counts.cpu().numpy()
    out.n_tracks, out.n_hits = int(c[0]), int(c[1])
    return int(status.cpu().numpy()[0]), {"tracks": out.to_numpy()}


def test_noalloc_equals_async_on_two_calls():
    import torch
    from paper_1811_11481_amd import DeviceClusters, Tracker
    trk = Tracker()
    big = synth.generate("C2").subset([0, 1, 2])
    small = synth.generate("C1")
    assert small.n_clusters < big.n_clusters <= 131072
    for name, cs in (("three C2 sectors", big), ("one sector", small)):
        log("allocation-free form on %s (%d clusters)" % (name, cs.n_clusters))
        dc = DeviceClusters.from_host(cs)
        st_a, ref = _run(trk.track_async, dc, trk.alloc_tracks(dc), torch)
        st_n, got = _run(trk.track_async_noalloc, dc, trk.alloc_tracks(dc), torch)
        assert st_a == 0 and st_n == 0
        assert len(got["tracks"]["inst"]) == len(ref["tracks"]["inst"]) > 0
        assert tracks_equal(got, ref)


def test_noalloc_rejects_inputs_above_its_limit():
    import torch
    from paper_1811_11481_amd import DeviceClusters, Tracker, TpccaError
    trk = Tracker()
    cs = synth.generate("C2").subset(list(range(6)))
    assert cs.n_clusters > 131072
    log("allocation-free form above its limit (%d clusters)" % cs.n_clusters)
    dc = DeviceClusters.from_host(cs)
    counts = torch.zeros(2, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(TpccaError) as e:
        trk.track_async_noalloc(dc, trk.alloc_tracks(dc), counts, status)
    assert e.value.status == 2
