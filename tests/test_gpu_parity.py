"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Integer and index results (grid order, links, starts, tracklet rows, weights,
ownership, masks, track cluster lists) must be identical; binary32 values
(states, parameters, covariances, chi2) must be bit-identical to the binary32
oracle, which runs the same operation order; FP64 totals agree to 1e-12
(different summation order). Parameters are also checked against the FP64
replay of the same hit lists and masks: |dp| <= 1e-4 max(|p|, floor, sigma_p)
with floors (1 cm, 1 cm, 0.01, 0.01, 0.1 c/GeV) and sigma_p the parameter's
own statistical error, and at least 99.9 % of tracks within 1e-4 max(|p|, floor).
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import compare_with_oracle, log, run_gpu, tracks_equal
from util import make_clusterset, row_of_ids

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def c1():
    return synth.generate("C1")


@pytest.fixture(scope="module")
def c1_oracle(c1):
    return oracle.run(c1, 32)


@pytest.fixture(scope="module")
def c2():
    return synth.generate("C2")


@pytest.fixture(scope="module")
def c2_oracle(c2):
    return oracle.run(c2, 32, threads=16)


def test_fp32_division_and_sqrt_are_correctly_rounded():
    from paper_1811_11481_amd import fp32_selfcheck
    rng = np.random.default_rng(0)
    n = 1 << 20
    a = (rng.standard_normal(n) * np.exp(rng.uniform(-30, 30, n))).astype(np.float32)
    b = (rng.standard_normal(n) * np.exp(rng.uniform(-30, 30, n))).astype(np.float32)
    special = np.array([1e-40, -3e-39, 1.0, 2.0, 1e38, 7.0, 0.1, 3.0, 1.0000001], np.float32)
    a[:9], b[:9] = special, special[::-1]
    log("fp32 self-check on %d values" % n)
    d, s = fp32_selfcheck(a, b)
    with np.errstate(all="ignore"):
        assert np.array_equal(d.view(np.uint32), (a / b).view(np.uint32))
        assert np.array_equal(s.view(np.uint32), np.sqrt(np.abs(a)).view(np.uint32))


def test_helix_step_sqrt_equals_sqrtf_over_its_domain():
    """Every binary32 argument from 2^-96 to +inf (1.9 G bit patterns), the
    zeros, a run of negatives and of NaNs: the helix step's root is bit-equal
    to sqrtf (itself checked against numpy above)."""
    from paper_1811_11481_amd import sqrt_step_check
    ranges = [(0x0F800000, 0x7F800000), (0x00000000, 0x00000000), (0x80000000, 0x80000000),
              (0xBF800000, 0xBF8FFFFF), (0x7F800001, 0x7F80FFFF), (0x7FC00000, 0x7FC0FFFF), (0xFFC00000, 0xFFC0FFFF)]
    for lo, hi in ranges:
        log("sqrt step check %08x..%08x" % (lo, hi))
        assert sqrt_step_check(lo, hi) == 0, (hex(lo), hex(hi))


def test_golden_neighbour_cases_on_gpu():
    cases = json.load(open(os.path.join(GOLDEN, "neighbour_cases.json")))["cases"]
    for case in cases:
        log("golden case: " + case["name"])
        cs = make_clusterset([(0, r, y, z) for r, y, z in case["hits"]])
        g = run_gpu(cs)
        m = case["middle"]
        assert (g["links"]["up"][m], g["links"]["dn"][m]) == (case["expect"]["up"], case["expect"]["dn"]), case["name"]
        compare_with_oracle(g, oracle.run(cs, 32))


def test_empty_and_degenerate_inputs():
    log("empty input")
    empty = make_clusterset([], n_inst=3)
    for batched in (True, False):
        g = run_gpu(empty, batched=batched)
        assert g["n_tracks"] == 0 and g["tracks"]["hit_start"][0] == 0
    log("hits on edge rows only, single hits, one dense row")
    hits = [(0, 0, 0.0, 1.0), (0, 151, 0.0, 1.0), (1, 5, 3.0, 4.0)]
    hits += [(1, 70, 0.001 * k, 2.0) for k in range(300)]  # one dense row, identical z
    cs = make_clusterset(hits, n_inst=2, sectors=[0, 19])
    g = run_gpu(cs)
    compare_with_oracle(g, oracle.run(cs, 32))


def test_c1_bit_exact_against_oracle(c1, c1_oracle):
    log("C1: %d clusters" % c1.n_clusters)
    g = run_gpu(c1)
    compare_with_oracle(g, c1_oracle)
    assert g["n_tracks"] > 50


def test_plain_equals_batched_and_is_deterministic(c1):
    log("C1 plain vs batched")
    a = run_gpu(c1, batched=True)
    b = run_gpu(c1, batched=False)
    c = run_gpu(c1, batched=True, tracker=a["tracker"])  # graph replay
    assert tracks_equal(a, b) and tracks_equal(a, c)


def test_batched_graph_follows_new_output_buffers(c1):
    """The batched form replays its captured graph only while every buffer it
    captured is the same: new alpha/ndf buffers, or x_ref and chi2 exchanged,
    must give a new capture that writes into the buffers of this call."""
    from paper_1811_11481_amd import DeviceClusters, Tracks
    log("C1 batched with new output buffers")
    ref = run_gpu(c1, batched=False, exports=False)
    trk = ref["tracker"]
    dc = DeviceClusters.from_host(c1)
    first = trk.track(dc, batched=True)
    assert tracks_equal({"tracks": first.to_numpy()}, ref)
    fresh = Tracks(first.cap_tracks, first.cap_hits)
    trk.track(dc, out=fresh, batched=True)
    assert tracks_equal({"tracks": fresh.to_numpy()}, ref)
    swapped = Tracks(first.cap_tracks, first.cap_hits)
    for k in ("inst", "param", "cov", "hit_start", "hit_id", "chi2_total"):
        setattr(swapped, k, getattr(first, k))
    swapped.x_ref, swapped.chi2 = first.chi2, first.x_ref
    trk.track(dc, out=swapped, batched=True)
    assert tracks_equal({"tracks": swapped.to_numpy()}, ref)


@pytest.mark.parametrize("tune", [dict(hits_per_bin=2), dict(hits_per_bin=3, block_tracklet=64, xcd_remap=0),
                                  dict(hits_per_bin=8, block_links=64, block_refit=256, block_scan=512, sort_seeds=1),
                                  dict(inward_wgs=1024), dict(inward_wgs=3, block_tracklet=64, xcd_remap=0),
                                  dict(inward_sort=0, block_tracklet=256), dict(inward_sort=0, block_tracklet=64, xcd_remap=0),
                                  dict(inward_sort=1, block_tracklet=256, xcd_remap=0), dict(sort_seeds=2),
                                  dict(sort_seeds=2, block_refit=64, xcd_remap=0), dict(sort_seeds=0),
                                  dict(sort_seeds=0, block_refit=256)])
def test_results_independent_of_tuning(c1, c1_oracle, tune):
    from paper_1811_11481_amd import default_tuning
    log("C1 tuning %s" % tune)
    g = run_gpu(c1, tuning=default_tuning(**tune))
    compare_with_oracle(g, c1_oracle, stages=("links", "tracklets", "selected", "tracks"))


def test_c2_full_event_bit_exact(c2, c2_oracle):
    log("C2: %d clusters, batched" % c2.n_clusters)
    g = run_gpu(c2)
    compare_with_oracle(g, c2_oracle)
    log("C2 plain (per-instance launches)")
    p = run_gpu(c2, batched=False, exports=False)
    assert tracks_equal(g, p)


def test_c2_split_inward_pass_bit_exact(c2, c2_oracle):
    # the single tracklet kernel, and the inward pass in its own kernel: ordered
    # by the row the outward pass reached (the default at 64 threads, here at
    # 256), and persistent with a full grid and with a grid of a few waves that
    # drains all eight queues; same stages bit for bit
    from paper_1811_11481_amd import default_tuning
    for tune in (dict(inward_sort=0), dict(inward_sort=1, block_tracklet=256), dict(inward_wgs=1024),
                 dict(inward_wgs=5)):
        log("C2 batched, split inward pass %s" % tune)
        g = run_gpu(c2, tuning=default_tuning(**tune))
        compare_with_oracle(g, c2_oracle)


def test_c2_refit_in_work_order_bit_exact(c2, c2_oracle):
    # the refit's tracks counting-sorted by estimated work per chunk of 1024
    # (sort_seeds = 2): batched against the oracle, and the plain form (one
    # launch per instance, selection ranges that start past zero) against it;
    # the consecutive order (sort_seeds = 0) against the oracle too
    from paper_1811_11481_amd import default_tuning
    log("C2 batched, refit in chunk order")
    compare_with_oracle(run_gpu(c2, tuning=default_tuning(sort_seeds=0)), c2_oracle)
    log("C2 batched, refit in work order")
    g = run_gpu(c2, tuning=default_tuning(sort_seeds=2))
    compare_with_oracle(g, c2_oracle)
    log("C2 plain, refit in work order")
    p = run_gpu(c2, batched=False, exports=False, tuning=default_tuning(sort_seeds=2, block_refit=64))
    assert tracks_equal(g, p)


def test_c2_parameters_against_fp64_replay(c2, c2_oracle):
    log("C2 FP64 replay")
    g = run_gpu(c2)
    T, S, tl = g["tracks"], g["selected"], g["tracklets"]
    rows = row_of_ids(c2)
    status = S["status"].astype(bool)
    sel_idx = np.nonzero(status)[0]
    assert len(sel_idx) == g["n_tracks"]
    hs = S["hit_start"]
    lens = np.diff(hs)[sel_idx]
    idx = np.concatenate([np.arange(hs[i], hs[i + 1]) for i in sel_idx])
    hit_start = np.concatenate([[0], np.cumsum(lens)])
    hits = S["hit_id"][idx]
    st0 = tl["state"][S["sel_tl"][sel_idx]].astype(np.float64)
    row0 = tl["state_row"][S["sel_tl"][sel_idx]]
    ok, out, chi2 = oracle.replay_f64(st0, row0, hit_start, rows[hits], c2.y[hits], c2.z[hits], S["mask"][idx])
    assert ok.all()
    p32 = T["param"].astype(np.float64)
    floors = np.array([1.0, 1.0, 0.01, 0.01, 0.1])
    sigma = np.sqrt(out[:, 5 + np.array([0, 2, 5, 9, 14])])
    err_p = np.abs(p32 - out[:, :5]) / np.maximum(np.abs(out[:, :5]), floors)
    log("max |p|-relative parameter error vs FP64: %s; above 1e-4: %s" % (err_p.max(axis=0), (err_p > 1e-4).sum(0)))
    # the stated bound on every track and parameter: |dp| <= 1e-4 max(|p|, floor)
    assert np.all(err_p <= 1e-4), err_p.max(axis=0)
    # report only: the error in units of each parameter's own statistical error
    log("max error in sigma units: %s" % (np.abs(p32 - out[:, :5]) / sigma).max(axis=0))
    rel_chi2 = np.abs(T["chi2"] - chi2) / np.maximum(chi2, 1.0)
    assert np.all(rel_chi2 <= 1e-3)


def test_output_capacity_error_reports_required_sizes(c1):
    from paper_1811_11481_amd import DeviceClusters, Tracker, Tracks, TpccaError
    log("C1 capacity error path")
    trk = Tracker()
    dc = DeviceClusters.from_host(c1)
    small = Tracks(3, 100)
    with pytest.raises(TpccaError) as e:
        trk.track(dc, out=small)
    assert e.value.status == 2
    assert small.n_tracks > 3 and small.n_hits > 100
    ok = trk.track(dc, out=Tracks(small.n_tracks, small.n_hits))
    assert ok.n_tracks == small.n_tracks


def test_malformed_csr_is_rejected_on_host(c1):
    import torch

    from paper_1811_11481_amd import DeviceClusters, Tracker, TpccaError
    log("malformed row_start")
    trk = Tracker()
    dc = DeviceClusters.from_host(c1)
    bad = dc.row_start.clone()
    bad[10] = bad[11] + 1  # decreasing
    with pytest.raises(TpccaError) as e:
        trk.track(DeviceClusters(dc.n_inst, dc.inst_sector, bad, dc.y, dc.z))
    assert e.value.status == 1
    short = DeviceClusters(dc.n_inst, dc.inst_sector, dc.row_start, dc.y[:-5], dc.z[:-5])
    with pytest.raises(TpccaError):
        trk.track(short)
    torch.cuda.synchronize()


def _sampled_instance_parity(cs, instances, gpu):
    """GPU output restricted to instance k == oracle run on instance k alone."""
    T = gpu["tracks"]
    for k in instances:
        sub = cs.subset([k])
        o = oracle.run(sub, 32, threads=4)
        parent = sub.meta["parent_index"]
        sel = np.nonzero(T["inst"] == k)[0]
        assert len(sel) == o.n_tracks, (k, len(sel), o.n_tracks)
        hs = T["hit_start"]
        g_hits = np.concatenate([T["hit_id"][hs[t]:hs[t + 1]] for t in sel]) if len(sel) else np.zeros(0, int)
        assert np.array_equal(g_hits, parent[o.trk_hit])
        assert np.array_equal(T["param"][sel].view(np.uint32), o.trk_param.astype(np.float32).view(np.uint32))
        assert np.array_equal(T["cov"][sel].view(np.uint32), o.trk_cov.astype(np.float32).view(np.uint32))


def test_c3_time_frame_sampled_parity():
    cs = synth.generate("C3")
    log("C3: %d clusters (full size on GPU, 2 sampled instances on the oracle)" % cs.n_clusters)
    g = run_gpu(cs, exports=False)
    _sampled_instance_parity(cs, [5, 30], g)


def test_c4_uneven_instances_sampled_parity():
    cs = synth.generate("C4")
    log("C4: %d clusters in %d instances" % (cs.n_clusters, cs.n_inst))
    g = run_gpu(cs, exports=False)
    sizes = np.diff(cs.row_start[::152])
    pick = [int(np.argmax(sizes)), int(np.argmin(sizes)), 100]
    _sampled_instance_parity(cs, pick, g)
    log("C4 plain vs batched")
    p = run_gpu(cs, batched=False, exports=False)
    assert tracks_equal(g, p)
    from paper_1811_11481_amd import default_tuning
    for order in (0, 2):
        log("C4 batched, refit order %d" % order)
        w = run_gpu(cs, exports=False, tuning=default_tuning(sort_seeds=order))
        assert tracks_equal(g, w)


def test_vertex_z_of_every_track(c2):
    """Each output track's closest-approach z (FP64 on the GPU from its binary32
    final state) against the oracle's FP64 formula on the same state."""
    log("C2 vertex z")
    g = run_gpu(c2, exports=False)
    T = g["tracks"]
    ref = oracle.vertex_z(T["x_ref"].astype(np.float64), T["param"].astype(np.float64))
    assert np.isfinite(T["z0"]).all()
    err = np.abs(T["z0"].astype(np.float64) - ref) / np.maximum(np.abs(ref), 1.0)
    assert err.max() <= 1e-6, err.max()
