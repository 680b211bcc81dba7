"""GPU-side helpers of the parity tests: run the HIP library through its C ABI
and compare every stage export with the oracle."""
from __future__ import annotations

import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_gpu(cs, batched=True, tuning=None, params=None, tracker=None, exports=True):
    from paper_1811_11481_amd import DeviceClusters, Tracker

    trk = tracker if tracker is not None else Tracker(params=params, tuning=tuning)
    if tuning is not None and tracker is not None:
        trk.set_tuning(tuning)
    dc = DeviceClusters.from_host(cs)
    out = trk.track(dc, batched=batched)
    res = {"tracks": out.to_numpy(), "n_tracks": out.n_tracks, "n_hits": out.n_hits,
           "row_start": np.asarray(cs.row_start)}
    if exports:
        res["grid"] = trk.export_grid()
        res["links"] = trk.export_links()
        res["tracklets"] = trk.export_tracklets()
        res["selected"] = trk.export_selected()
        res["sizes"] = trk.sizes()
    res["tracker"] = trk
    return res


def f32_equal(gpu_f32, orc_f64):
    """Bit equality of binary32 GPU values with the oracle's binary32 values
    (exported as doubles, which hold them exactly)."""
    a = np.asarray(gpu_f32, dtype=np.float32)
    b = np.asarray(orc_f64, dtype=np.float64).astype(np.float32)
    assert np.array_equal(np.asarray(orc_f64, np.float64), b.astype(np.float64)), "oracle value is not binary32"
    return np.array_equal(a.view(np.uint32), b.view(np.uint32))


def first_diff(a, b):
    a, b = np.asarray(a), np.asarray(b)
    if a.shape != b.shape:
        return "shape %s vs %s" % (a.shape, b.shape)
    idx = np.nonzero(a.reshape(-1) != b.reshape(-1))[0]
    return "%d differ, first at %s: %s vs %s" % (len(idx), idx[:5], a.reshape(-1)[idx[:5]], b.reshape(-1)[idx[:5]])


def used_bin_slots(row_start, nbins):
    """Indices of the bin_start entries a grid owns: segment s holds nbins[s] + 1
    entries from row_start[s] + s (the rest of its n + 1 slots is unused)."""
    rs = np.asarray(row_start, np.int64)
    starts = rs[:-1] + np.arange(len(rs) - 1)
    return np.concatenate([np.arange(a, a + nb + 1) for a, nb in zip(starts, nbins)]) if len(nbins) else \
        np.zeros(0, np.int64)


def compare_with_oracle(g, o, stages=("grid", "links", "tracklets", "selected", "tracks")):
    """Bit-exact comparison of every stage; raises AssertionError naming the first mismatch."""
    if "grid" in stages:
        gr = g["grid"]
        assert np.array_equal(gr["sorted_id"], o.sorted_id), "grid sorted_id: " + first_diff(gr["sorted_id"], o.sorted_id)
        assert np.array_equal(gr["ny"], o.g_ny) and np.array_equal(gr["nz"], o.g_nz), "grid shape"
        used = used_bin_slots(g["row_start"], o.g_ny * o.g_nz)
        assert np.array_equal(gr["bin_start"][used], o.bin_start[used]), "grid bin_start: " + first_diff(
            gr["bin_start"][used], o.bin_start[used])
        assert f32_equal(gr["meta"], o.g_meta), "grid meta"
    if "links" in stages:
        L = g["links"]
        for k, v in (("up", o.up), ("dn", o.dn), ("upc", o.upc), ("dnc", o.dnc)):
            assert np.array_equal(L[k], v), "links %s: %s" % (k, first_diff(L[k], v))
    if "tracklets" in stages:
        t = g["tracklets"]
        assert np.array_equal(t["start_hit"], o.start_hit), "starts: " + first_diff(t["start_hit"], o.start_hit)
        assert np.array_equal(t["start_inst"], o.start_inst) and np.array_equal(t["start_tid"], o.start_tid)
        assert np.array_equal(t["nhits"], o.tl_nhits), "tracklet nhits: " + first_diff(t["nhits"], o.tl_nhits)
        assert np.array_equal(t["rowhit"], o.tl_rowhit), "tracklet rows: " + first_diff(t["rowhit"], o.tl_rowhit)
        assert np.array_equal(t["state_row"], o.tl_row), "tracklet state row"
        assert f32_equal(t["state"], o.tl_state), "tracklet state: " + first_diff(
            t["state"], o.tl_state.astype(np.float32))
        assert np.array_equal(t["weight"], o.weight), "weights: " + first_diff(t["weight"], o.weight)
    if "selected" in stages:
        s = g["selected"]
        assert np.array_equal(s["sel_tl"], o.sel_tl), "selected: " + first_diff(s["sel_tl"], o.sel_tl)
        assert np.array_equal(s["hit_start"], o.sel_hit_start), "selected hit_start"
        assert np.array_equal(s["hit_id"], o.sel_hit), "selected hits"
        assert np.array_equal(s["mask"], o.sel_mask), "refit masks: " + first_diff(s["mask"], o.sel_mask)
        assert np.array_equal(s["status"], o.sel_status), "refit status"
    if "tracks" in stages:
        T = g["tracks"]
        assert g["n_tracks"] == o.n_tracks, "n_tracks %d vs %d" % (g["n_tracks"], o.n_tracks)
        assert np.array_equal(T["inst"], o.trk_inst)
        assert np.array_equal(T["hit_start"], o.trk_hit_start), "track hit_start"
        assert np.array_equal(T["hit_id"], o.trk_hit), "track hits"
        assert np.array_equal(T["ndf"], o.trk_ndf)
        assert f32_equal(T["x_ref"], o.trk_x) and f32_equal(T["alpha"], o.trk_alpha)
        assert f32_equal(T["param"], o.trk_param), "params: " + first_diff(T["param"], o.trk_param.astype(np.float32))
        assert f32_equal(T["cov"], o.trk_cov), "cov"
        assert f32_equal(T["chi2"], o.trk_chi2), "chi2"
        tot = T["chi2_total"]
        assert abs(tot[0] - o.chi2_total) <= 1e-12 * max(1.0, abs(o.chi2_total)), (tot[0], o.chi2_total)
        assert tot[1] == o.ndf_total


def tracks_equal(a, b):
    """Bit equality of two GPU track outputs (numpy dicts)."""
    ta, tb = a["tracks"], b["tracks"]
    for k in ta:
        x, y = np.asarray(ta[k]), np.asarray(tb[k])
        if x.dtype.kind == "f":
            if not np.array_equal(x.view(np.uint32 if x.dtype == np.float32 else np.uint64),
                                  y.view(np.uint32 if y.dtype == np.float32 else np.uint64)):
                return False
        elif not np.array_equal(x, y):
            return False
    return True
