"""Precision and batching forms on the GPU.

Precision: every output of the binary32 GPU path against binary64 (the FP64
replay on the same hit lists and accept masks, and the independent FP64
tracker for the decisions). Batching: the autotuner's choice gives output
bit-identical to the default tiling, and the batched form equals per-sector
launches.
"""
import json

import numpy as np
import pytest

import oracle
import synth
from gpu_util import log, run_gpu, tracks_equal
from util import row_of_ids

pytestmark = pytest.mark.gpu


def test_precision_report_central_event():
    cs = synth.generate("C2")
    log("precision report on C2 (%d clusters)" % cs.n_clusters)
    g = run_gpu(cs)
    T, S, tl = g["tracks"], g["selected"], g["tracklets"]
    rows = row_of_ids(cs)
    sel_idx = np.nonzero(S["status"].astype(bool))[0]
    hs = S["hit_start"]
    idx = np.concatenate([np.arange(hs[i], hs[i + 1]) for i in sel_idx])
    hit_start = np.concatenate([[0], np.cumsum(np.diff(hs)[sel_idx])])
    hits = S["hit_id"][idx]
    ok, out, chi2 = oracle.replay_f64(tl["state"][S["sel_tl"][sel_idx]].astype(np.float64),
                                      tl["state_row"][S["sel_tl"][sel_idx]], hit_start, rows[hits], cs.y[hits],
                                      cs.z[hits], S["mask"][idx])
    assert ok.all()
    p32, c32 = T["param"].astype(np.float64), T["cov"].astype(np.float64)
    p64, c64 = out[:, :5], out[:, 5:]
    floors = np.array([1.0, 1.0, 0.01, 0.01, 0.1])
    sig = np.sqrt(c64[:, [0, 2, 5, 9, 14]])
    names = ["y", "z", "sin_phi", "tan_lambda", "q_over_pt"]
    rep = {"n_tracks": int(len(p32))}
    rel = np.abs(p32 - p64) / np.maximum(np.abs(p64), floors)
    rel_s = np.abs(p32 - p64) / np.maximum(np.maximum(np.abs(p64), floors), sig)
    for k, nm in enumerate(names):
        rep["param_" + nm] = {"max_rel": float(rel[:, k].max()), "p99_9_rel": float(np.percentile(rel[:, k], 99.9)),
                              "max_rel_sigma_scale": float(rel_s[:, k].max()),
                              "max_in_sigma": float((np.abs(p32 - p64)[:, k] / sig[:, k]).max())}
    ii, jj = np.tril_indices(5)
    scale = np.sqrt(np.abs(c64[:, [0, 2, 5, 9, 14]][:, ii] * c64[:, [0, 2, 5, 9, 14]][:, jj]))
    crel = np.abs(c32 - c64) / scale
    rep["cov"] = {"max_rel_to_sqrt_cii_cjj": float(crel.max()), "p99_9": float(np.percentile(crel, 99.9))}
    rep["chi2"] = {"max_rel": float((np.abs(T["chi2"] - chi2) / np.maximum(chi2, 1.0)).max())}
    rep["ndf"] = "identical (same accept masks)"
    tot = g["tracks"]["chi2_total"]
    rep["chi2_total_fp64_sum_vs_sum_of_fp64"] = float(abs(tot[0] - chi2.sum()) / chi2.sum())
    # decisions: binary32 path against the independent binary64 tracker
    o64 = oracle.run(cs, 64, threads=16)
    same_tracks = np.array_equal(T["hit_start"], o64.trk_hit_start) and np.array_equal(T["hit_id"], o64.trk_hit)
    a = {tuple(T["hit_id"][T["hit_start"][t]:T["hit_start"][t + 1]]) for t in range(g["n_tracks"])}
    b = {tuple(o64.trk_hit[o64.trk_hit_start[t]:o64.trk_hit_start[t + 1]]) for t in range(o64.n_tracks)}
    rep["hit_lists_vs_fp64_tracker"] = {"identical": bool(same_tracks), "tracks_fp32": len(a), "tracks_fp64": len(b),
                                        "common_identical_lists": len(a & b)}
    log("PRECISION_REPORT " + json.dumps(rep))
    for nm in names:  # the stated bound, |dp| <= 1e-4 max(|p|, floor), on every track
        assert rep["param_" + nm]["max_rel"] <= 1e-4, (nm, rep["param_" + nm])
    assert rep["cov"]["max_rel_to_sqrt_cii_cjj"] <= 1e-3
    assert len(a & b) >= 0.995 * len(b)


def test_autotuned_tiling_is_bit_identical():
    from paper_1811_11481_amd import DeviceClusters, Tracker, default_tuning
    cs = synth.generate("C4").subset(list(range(0, 256, 4)))
    log("autotune on 64 C4 instances (%d clusters)" % cs.n_clusters)
    trk = Tracker()
    dc = DeviceClusters.from_host(cs)
    ref = run_gpu(cs, tuning=default_tuning(), exports=False)
    t = trk.autotune(dc, repeats=2)
    log("autotuned: %s" % t.as_dict())
    got = run_gpu(cs, tracker=trk, exports=False)
    assert tracks_equal(ref, got)
    plain = run_gpu(cs, tracker=trk, batched=False, exports=False)
    assert tracks_equal(ref, plain)
