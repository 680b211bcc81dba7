"""Cross-sector merge on the GPU (tpcca_merge) against the oracle's merge of
the same sector tracks: pair links, merged cluster lists, segment counts and
the binary32 merged refit, bit for bit."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import f32_equal, first_diff, log

pytestmark = pytest.mark.gpu


def _compare(cs, inst_event, label):
    import torch
    from paper_1811_11481_amd import FLAG_MERGE, DeviceClusters, Tracker, default_params
    log("%s: merge of %d clusters in %d instances" % (label, cs.n_clusters, cs.n_inst))
    o = oracle.run(cs, 32, threads=16, inst_event=inst_event)
    trk = Tracker(params=default_params(flags=FLAG_MERGE))
    dc = DeviceClusters.from_host(cs)
    T = trk.track(dc, batched=True)
    assert T.n_tracks == o.n_tracks
    ev = torch.as_tensor(np.asarray(inst_event, np.int32), device="cuda")
    M, nseg, nxt = trk.merge(ev)
    g = M.to_numpy()
    m = o.merged
    assert np.array_equal(nxt.cpu().numpy(), m["next"]), "links: " + first_diff(nxt.cpu().numpy(), m["next"])
    assert M.n_tracks == len(m["src"]), (M.n_tracks, len(m["src"]))
    assert np.array_equal(nseg.cpu().numpy(), m["nseg"])
    assert np.array_equal(g["inst"], m["inst"])
    assert np.array_equal(g["hit_start"], m["hit_start"]) and np.array_equal(g["hit_id"], m["hit_id"])
    assert np.array_equal(g["ndf"], m["ndf"])
    assert f32_equal(g["x_ref"], m["x_ref"]) and f32_equal(g["alpha"], m["alpha"])
    assert f32_equal(g["param"], m["param"]), "params: " + first_diff(g["param"], m["param"].astype(np.float32))
    assert f32_equal(g["cov"], m["cov"]) and f32_equal(g["chi2"], m["chi2"])
    log("%s: %d sector tracks -> %d tracks, %d with 2+ segments" % (label, T.n_tracks, M.n_tracks,
                                                                   int((nseg.cpu().numpy() > 1).sum())))
    # the merge flag changes no sector track
    ref = Tracker().track(dc, batched=True).to_numpy()
    got = T.to_numpy()
    for k in ("hit_start", "hit_id", "param", "cov"):
        assert np.array_equal(got[k], ref[k])
    return M


def test_merge_central_event_bit_exact():
    cs = synth.generate("C2")
    M = _compare(cs, np.zeros(cs.n_inst, np.int32), "C2")
    assert M.n_tracks < 0.7 * 18887


def test_merge_two_events_bit_exact():
    a = synth.generate("C2").subset(list(range(0, 9)) + list(range(18, 27)))
    b = synth.generate("C2", event=1).subset(list(range(0, 9)) + list(range(18, 27)))
    cs = synth.ClusterSet(a.n_inst + b.n_inst, np.concatenate([a.inst_sector, b.inst_sector]),
                          np.concatenate([a.row_start, b.row_start[1:] + a.row_start[-1]]),
                          np.concatenate([a.x, b.x]), np.concatenate([a.y, b.y]), np.concatenate([a.z, b.z]),
                          np.concatenate([a.row, b.row]), np.concatenate([a.label, b.label]), a.truth)
    ev = np.repeat([3, 7], [a.n_inst, b.n_inst]).astype(np.int32)
    _compare(cs, ev, "two half events")
