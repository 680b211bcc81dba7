"""The batched form without host synchronisation (tpcca_track_async): the CSR
check runs on the device, counts and status stay on the device, and the
output buffers equal those of the synchronising batched form bit for bit."""
import numpy as np
import pytest

import synth
from gpu_util import log, run_gpu, tracks_equal
from util import with_dense_rows

pytestmark = pytest.mark.gpu


def _async(trk, dc, out, torch):
    counts = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    trk.track_async(dc, out, counts, status)
    torch.cuda.synchronize()
    c = counts.cpu().numpy()
    out.n_tracks, out.n_hits = int(c[0]), int(c[1])
    return int(status.cpu().numpy()[0]), out


def test_async_equals_batched_and_reports_on_device():
    import torch
    from paper_1811_11481_amd import DeviceClusters, Tracker
    trk = Tracker()
    for name, cs in (("C1", synth.generate("C1")), ("C2 sectors 0-5", synth.generate("C2").subset(range(6)))):
        log("async form on %s (%d clusters)" % (name, cs.n_clusters))
        ref = run_gpu(cs, exports=False)
        dc = DeviceClusters.from_host(cs)
        out = trk.alloc_tracks(dc)
        st, out = _async(trk, dc, out, torch)
        assert st == 0
        assert out.n_tracks == ref["n_tracks"] and out.n_hits == ref["n_hits"]
        assert tracks_equal({"tracks": out.to_numpy()}, ref)


def test_async_errors_stay_on_device():
    import torch
    from paper_1811_11481_amd import DeviceClusters, Tracker, Tracks
    cs = synth.generate("C1")
    trk = Tracker()
    dc = DeviceClusters.from_host(cs)
    ref = run_gpu(cs, exports=False)
    log("async: malformed CSR")
    bad = dc.row_start.clone()
    bad[10] = bad[11] + 1
    st, _ = _async(trk, DeviceClusters(dc.n_inst, dc.inst_sector, bad, dc.y, dc.z), trk.alloc_tracks(dc), torch)
    assert st == 1
    last = dc.row_start.clone()
    last[-1] = last[-1] - 1
    st, _ = _async(trk, DeviceClusters(dc.n_inst, dc.inst_sector, last, dc.y, dc.z), trk.alloc_tracks(dc), torch)
    assert st == 1
    log("async: output capacity")
    st, small = _async(trk, dc, Tracks(3, 100), torch)
    assert st == 2 and small.n_tracks == ref["n_tracks"] and small.n_hits == ref["n_hits"]
    log("async: a row above the per-row limit")
    dense = with_dense_rows(cs, {60: 16400})
    dd = DeviceClusters.from_host(dense)
    st, _ = _async(trk, dd, trk.alloc_tracks(dd), torch)
    assert st == 2
    log("async: a good call after the failures")
    st, out = _async(trk, dc, trk.alloc_tracks(dc), torch)
    assert st == 0 and tracks_equal({"tracks": out.to_numpy()}, ref)
