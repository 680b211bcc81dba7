"""GPU differentiable refit (tpcca_refit_fwd / tpcca_refit_bwd) against the oracle.

* Without a map the frozen-mask refit is the refit the tracker ran: chi2 per
  track bit-identical to the tracker's output (and so to the binary32 oracle).
* With a correction map, chi2 against the FP64 oracle on the same binary32
  inputs.
* Gradients against central differences of the FP64 oracle function, for the
  start states of every track and for a sample of map coefficients, with the
  adjoint in binary32 and in binary64.
* Identities of the exact derivative that the GPU gradient must keep: the sum
  over a track's clusters of dchi2/dz' equals -dchi2/dz0 (and the same in y),
  and the sum over all dz coefficients of dchi2/dcoef equals sum_t dchi2_t/dz0_t.
* The torch.autograd wrapper, its recomputation after an intervening forward,
  input validation and the empty set.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import log

pytestmark = pytest.mark.gpu

N_ROWS = 152


def _set_to_host(cs, rset):
    """Oracle inputs for a device refit set (cluster rows from the CSR)."""
    p0 = rset.params0.cpu().numpy().astype(np.float64)
    c0 = rset.cov0.cpu().numpy().astype(np.float64)
    hs = rset.hit_start.cpu().numpy()
    hid = rset.hit_id.cpu().numpy()
    inst = rset.inst.cpu().numpy()
    seg = np.searchsorted(cs.row_start, hid, side="right") - 1
    sector = cs.inst_sector[inst]
    alpha32 = (((sector % 18) + 0.5) * (20.0 * np.pi / 180.0)).astype(np.float32).astype(np.float64)
    return dict(st0=np.concatenate([p0, c0], axis=1), row0=rset.row0.cpu().numpy(), alpha=alpha32,
                hit_start=hs, hit_rows=(seg % N_ROWS).astype(np.int32), hit_id=hid,
                ys=cs.y[hid].astype(np.float64), zs=cs.z[hid].astype(np.float64),
                masks=rset.hit_mask.cpu().numpy(), inst=inst)


def _smooth_map(seed, amp=0.1):
    rng = np.random.default_rng(seed)
    return (amp * rng.standard_normal(oracle.MAP_SHAPE)).astype(np.float32)


@pytest.fixture(scope="module")
def c1_setup():
    from paper_1811_11481_amd import DeviceClusters, RefitSet, Tracker
    cs = synth.generate("C1")
    trk = Tracker()
    dc = DeviceClusters.from_host(cs)
    out = trk.track(dc)
    T = out.to_numpy()
    rset = RefitSet.from_tracker(trk)
    return cs, trk, dc, T, rset


def test_refit_set_from_tracker_matches_oracle_set(c1_setup):
    cs, _, _, _, rset = c1_setup
    h = _set_to_host(cs, rset)
    o = oracle.refit_inputs(oracle.run(cs, 32), cs)
    for k in ("st0", "row0", "hit_start", "hit_rows", "hit_id", "masks", "inst"):
        assert np.array_equal(np.asarray(h[k]), np.asarray(o[k])), k


def test_forward_without_map_is_the_trackers_refit(c1_setup):
    import torch
    cs, trk, dc, T, rset = c1_setup
    log("C1 frozen refit, %d tracks" % rset.n_tracks)
    chi2, ok, total = trk.refit_forward(dc, rset)
    assert ok.cpu().numpy().all()
    assert np.array_equal(chi2.cpu().numpy().view(np.uint32), T["chi2"].view(np.uint32))
    zero = torch.zeros(oracle.MAP_SHAPE, dtype=torch.float32, device="cuda")
    chi2z, _, totz = trk.refit_forward(dc, rset, coef=zero)
    assert np.array_equal(chi2z.cpu().numpy().view(np.uint32), T["chi2"].view(np.uint32))
    ref = T["chi2"].astype(np.float64).sum()
    assert abs(total.item() - ref) <= 1e-12 * ref and total.item() == totz.item()


def test_forward_with_map_against_fp64(c1_setup):
    import torch
    cs, trk, dc, T, rset = c1_setup
    coef = _smooth_map(11)
    chi2, ok, _ = trk.refit_forward(dc, rset, coef=torch.as_tensor(coef, device="cuda"))
    h = _set_to_host(cs, rset)
    ok_o, chi2_o = oracle.refit_frozen_f64(h["st0"], h["row0"], h["alpha"], h["hit_start"], h["hit_rows"], h["ys"],
                                           h["zs"], h["masks"], coef.astype(np.float64))
    g = chi2.cpu().numpy().astype(np.float64)
    assert np.array_equal(ok.cpu().numpy().astype(bool), ok_o)
    rel = np.abs(g - chi2_o) / np.maximum(chi2_o, 1.0)
    log("chi2 with map vs FP64: max rel %.3g, median %.3g; chi2 changed by the map: %.3g" % (
        rel.max(), np.median(rel), np.abs(chi2_o - T["chi2"]).max()))
    assert rel.max() <= 2e-4
    assert np.abs(chi2_o - T["chi2"]).max() > 1.0  # the map matters


def _scaled_err(g, ref, scale):
    """max over tracks of |g - ref| / max|ref| with components in units of the start sigma."""
    a, b = g * scale, ref * scale
    return np.abs(a - b).max(axis=1) / np.maximum(np.abs(b).max(axis=1), 1e-300)


def _subset(rset, idx):
    """A refit set of the tracks idx (their cluster lists gathered into one CSR)."""
    import torch

    from paper_1811_11481_amd import RefitSet
    hs = rset.hit_start.cpu().numpy()
    lens = np.diff(hs)[idx]
    cl = np.concatenate([np.arange(hs[t], hs[t + 1]) for t in idx])
    ti = torch.as_tensor(np.asarray(idx, np.int64), device="cuda")
    ci = torch.as_tensor(cl, device="cuda")
    return RefitSet(rset.params0[ti].contiguous(), rset.cov0[ti].contiguous(), rset.row0[ti].contiguous(),
                    rset.inst[ti].contiguous(),
                    torch.as_tensor(np.concatenate([[0], np.cumsum(lens)]).astype(np.int64), device="cuda"),
                    rset.hit_id[ci].contiguous(), rset.hit_mask[ci].contiguous())


@pytest.mark.parametrize("f64", [False, True])
def test_gradients_against_fp64_finite_differences(c1_setup, f64):
    cs, _, dc, _, rset = c1_setup
    _fd_check(cs, dc, rset, f64)


def test_gradients_against_fp64_finite_differences_central_event():
    # every 40th track of the central event: all 36 sectors, both sides, the
    # map's full phi and z range
    from paper_1811_11481_amd import DeviceClusters, RefitSet, Tracker
    cs = synth.generate("C2")
    trk = Tracker()
    dc = DeviceClusters.from_host(cs)
    trk.track(dc)
    full = RefitSet.from_tracker(trk)
    idx = np.arange(0, full.n_tracks, 40)
    rset = _subset(full, idx)
    log("C2: finite differences on %d of %d tracks" % (rset.n_tracks, full.n_tracks))
    # start-state gradient error bound in units of the track's largest
    # cluster sensitivity: 1e-6 is 16 binary32 ulp of that unit (C1's 1e-7 is
    # under 2 ulp, met there with room; a central-event track reaches 2.5 ulp)
    _fd_check(cs, dc, rset, False, drop_failed=True, start_tol=1e-6)


def _fd_check(cs, dc, rset, f64, drop_failed=False, start_tol=1e-7):
    import torch

    from paper_1811_11481_amd import FLAG_ADJOINT_F64, Tracker, default_params
    trk = Tracker(params=default_params(flags=FLAG_ADJOINT_F64 if f64 else 0))
    coef = _smooth_map(12)
    n = rset.n_tracks
    trk.refit_forward(dc, rset, coef=torch.as_tensor(coef, device="cuda"))
    ones = torch.ones(n, dtype=torch.float32, device="cuda")
    gp, gm, gh = trk.refit_backward(ones, want_map=True, want_hits=True)
    gp, gm, gh = gp.cpu().numpy(), gm.cpu().numpy().reshape(-1), gh.cpu().numpy()
    h = _set_to_host(cs, rset)
    # coefficient sample: the largest GPU gradients of each component plus random touched ones
    rng = np.random.default_rng(3)
    nz = np.nonzero(gm)[0]
    sample = np.unique(np.concatenate([[np.argmax(np.abs(gm[c * 8192:(c + 1) * 8192])) + c * 8192 for c in range(3)],
                                       rng.choice(nz, 21, replace=False)]))
    sig = np.sqrt(h["st0"][:, 5 + np.array([0, 2, 5, 9, 14])])
    # start-state steps of 1 % of each parameter's sigma: the chi2 changes so
    # little with the start state that smaller steps drown in rounding
    ok, gp_fd, gc_fd = oracle.frozen_chi2_grad_fd(h, coef=coef.astype(np.float64), coef_index=sample,
                                                  h_param=1e-2 * sig)
    if drop_failed and not ok.all():
        # a step of a few tracks near the |sin phi| guard fails at a +-h
        # evaluation: their difference quotient is undefined; check the rest
        log("finite differences undefined for %d tracks: dropped" % (~ok.astype(bool)).sum())
        return _fd_check(cs, dc, _subset(rset, np.nonzero(ok)[0]), f64, start_tol=start_tol)
    assert ok.all()
    hs = h["hit_start"]
    # The pass-3 chi2 barely depends on the start state (three covariance
    # resets forget it): its gradient, in chi2 per start sigma, is ~1e-7 of the
    # chi2 per sigma of the track's most sensitive cluster, a small difference
    # of large adjoint terms, and the binary32 forward states perturb it at the
    # 1e-9 level of that scale. So the start gradient is checked in that unit,
    # and by its median relative error.
    gsc = np.maximum.reduceat(np.abs(gh).max(axis=1), hs[:-1]) * 0.1
    err_n = (np.abs(gp - gp_fd) * sig).max(axis=1) / gsc
    rel_p = _scaled_err(gp, gp_fd, sig)
    err_c = np.abs(gm[sample] - gc_fd) / np.abs(gc_fd).max()
    log("adjoint %s: start-state gradient error %.3g (max, cluster-sensitivity units), median relative %.3g; "
        "map gradient error max %.3g of max|g| = %.3g" % ("f64" if f64 else "f32", err_n.max(), np.median(rel_p),
                                                          err_c.max(), np.abs(gc_fd).max()))
    assert err_n.max() <= start_tol
    assert np.median(rel_p) <= 2e-2
    assert err_c.max() <= (2e-5 if f64 else 1e-4)
    # identities of the exact derivative
    for k in (0, 1):
        per_track = np.add.reduceat(gh[:, k], hs[:-1]) if len(gh) else np.zeros(0)
        scale = np.maximum(np.abs(gh[:, k]).max(), 1e-30)
        assert np.abs(per_track + gp[:, k]).max() <= (1e-9 if f64 else 1e-4) * scale
    # (the B-spline weights are binary32: they sum to 1 within a few ulp)
    lhs, rhs = gm[2 * 8192:].sum(), gp[:, 1].sum()
    assert abs(lhs - rhs) <= (1e-6 if f64 else 1e-4) * np.abs(gh[:, 1]).sum()


def test_autograd_function_and_recompute(c1_setup):
    import torch

    from paper_1811_11481_amd import refit_chi2
    cs, trk, dc, T, rset = c1_setup
    n = rset.n_tracks
    rng = np.random.default_rng(7)
    w = torch.as_tensor(rng.uniform(0.5, 2.0, n), dtype=torch.float64, device="cuda")
    p = rset.params0.clone().to(torch.float64).requires_grad_(True)
    c = torch.as_tensor(_smooth_map(13), dtype=torch.float64, device="cuda").requires_grad_(True)
    chi2, ok = refit_chi2(trk, dc, rset, p, c)
    loss = (chi2.to(torch.float64) * w).sum()
    trk.refit_forward(dc, rset)  # an intervening forward: backward must recompute its checkpoints
    loss.backward()
    # direct call with the same weights
    trk.refit_forward(dc, rset, p.detach().float().contiguous(), c.detach().float().contiguous())
    gp, gm, _ = trk.refit_backward(w.float().contiguous())
    assert torch.equal(p.grad, gp)
    # map gradients: FP64 atomics, the order of accumulation may differ
    assert torch.allclose(c.grad.reshape(-1), gm.reshape(-1), rtol=1e-12, atol=1e-12 * float(gm.abs().max()))
    assert p.grad.dtype == torch.float64 and c.grad.shape == c.shape
    # no map input: gradient for the start states only
    p2 = rset.params0.clone().requires_grad_(True)
    chi2b, _ = refit_chi2(trk, dc, rset, p2)
    assert np.array_equal(chi2b.detach().cpu().numpy().view(np.uint32), T["chi2"].view(np.uint32))
    chi2b.sum().backward()
    assert p2.grad.shape == p2.shape and torch.isfinite(p2.grad).all()


def test_refit_set_validation(c1_setup):
    import torch

    from paper_1811_11481_amd import RefitSet, TpccaError
    cs, trk, dc, T, rset = c1_setup

    def variant(**over):
        d = {k: getattr(rset, k) for k in ("params0", "cov0", "row0", "inst", "hit_start", "hit_id", "hit_mask")}
        d.update(over)
        return RefitSet(**d)

    hs = rset.hit_start.clone()
    hs[-1] -= 1  # does not end at n_hits
    bad_rows = rset.hit_id.clone()
    a, b = int(rset.hit_start[3]), int(rset.hit_start[3]) + 1
    bad_rows[a], bad_rows[b] = rset.hit_id[b], rset.hit_id[a]  # rows of track 3 out of order
    other = rset.hit_id.clone()
    other[0] = cs.n_clusters + 5  # not a cluster of the instance
    row0 = rset.row0.clone()
    row0[1] = N_ROWS
    inst = rset.inst.clone()
    inst[2] = dc.n_inst
    for name, rs in (("hit_start", variant(hit_start=hs)), ("rows", variant(hit_id=bad_rows)),
                     ("hit id", variant(hit_id=other)), ("row0", variant(row0=row0)), ("inst", variant(inst=inst))):
        log("invalid refit set: " + name)
        with pytest.raises(TpccaError) as e:
            trk.refit_forward(dc, rs)
        assert e.value.status == 1
        with pytest.raises(TpccaError):  # no valid forward to differentiate
            trk.refit_backward(torch.ones(rset.n_tracks, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    # the empty set
    e = variant(params0=rset.params0[:0], cov0=rset.cov0[:0], row0=rset.row0[:0], inst=rset.inst[:0],
                hit_start=torch.zeros(1, dtype=torch.int64, device="cuda"), hit_id=rset.hit_id[:0],
                hit_mask=rset.hit_mask[:0])
    chi2, ok, total = trk.refit_forward(dc, e)
    assert chi2.numel() == 0 and total.item() == 0.0
    gp, gm, _ = trk.refit_backward(torch.zeros(0, dtype=torch.float32, device="cuda"))
    assert gp.numel() == 0 and float(gm.abs().max()) == 0.0


def _permute(rset, order):
    import torch

    from paper_1811_11481_amd import RefitSet
    hs = rset.hit_start.cpu().numpy()
    order = np.asarray(order)
    pos = np.concatenate([np.arange(hs[t], hs[t + 1]) for t in order])
    lens = hs[order + 1] - hs[order]
    o = torch.as_tensor(order, device="cuda")
    p = torch.as_tensor(pos, device="cuda")
    return RefitSet(rset.params0[o].contiguous(), rset.cov0[o].contiguous(), rset.row0[o].contiguous(),
                    rset.inst[o].contiguous(), torch.as_tensor(np.concatenate([[0], np.cumsum(lens)]), device="cuda"),
                    rset.hit_id[p].contiguous(), rset.hit_mask[p].contiguous())


def test_map_gradient_independent_of_track_order():
    """C2, all tracks: in instance order a workgroup's clusters touch a small
    coefficient box; in random order every workgroup spans all sectors and both
    sides (full phi range, z cut into slabs). The map gradient is summed in
    fixed point (exact, associative integer additions), so it is bit-identical
    in either order and from one run to the next."""
    import torch

    from paper_1811_11481_amd import DeviceClusters, RefitSet, Tracker
    cs = synth.generate("C2")
    trk = Tracker()
    dc = DeviceClusters.from_host(cs)
    trk.track(dc)
    rs = RefitSet.from_tracker(trk)
    log("C2 refit set: %d tracks, %d clusters" % (rs.n_tracks, rs.n_hits))
    coef = torch.as_tensor(_smooth_map(21), device="cuda")
    perm = np.random.default_rng(2).permutation(rs.n_tracks)
    out = []
    for r in (rs, _permute(rs, perm), rs):
        chi2, ok, _ = trk.refit_forward(dc, r, coef=coef)
        w = torch.ones(r.n_tracks, dtype=torch.float32, device="cuda")
        gp, gm, _ = trk.refit_backward(w)
        out.append((chi2.cpu().numpy(), gp.cpu().numpy(), gm.cpu().numpy().reshape(-1)))
    (c0, p0, m0), (c1, p1, m1), (c2, p2, m2) = out
    assert np.array_equal(c0[perm], c1) and np.array_equal(p0[perm], p1)
    assert np.array_equal(m0, m1) and np.array_equal(m0, m2)
    assert np.count_nonzero(m0) > 1000


def test_batched_recompute_equals_full_tape(c1_setup):
    """A tape budget below the set's tape makes the backward re-record the
    forward batch by batch: same gradients as the whole-set tape."""
    import torch

    from paper_1811_11481_amd import DeviceClusters, RefitSet, Tracker, TpccaError, default_tuning
    cs = synth.generate("C2")
    dc = DeviceClusters.from_host(cs)
    full = Tracker()
    full.track(dc)
    rs = RefitSet.from_tracker(full)
    small = Tracker(tuning=default_tuning(tape_mb=1))  # ~13 tracks per batch
    coef = torch.as_tensor(_smooth_map(31), device="cuda")
    w = torch.as_tensor(np.random.default_rng(1).uniform(0.5, 2, rs.n_tracks), dtype=torch.float32, device="cuda")
    res = []
    for trk in (full, small):
        chi2, _, tot = trk.refit_forward(dc, rs, coef=coef)
        gp, gm, gh = trk.refit_backward(w, want_map=True, want_hits=True)
        res.append((chi2.cpu().numpy(), tot.item(), gp.cpu().numpy(), gm.cpu().numpy(), gh.cpu().numpy()))
    (c0, t0, p0, m0, h0), (c1, t1, p1, m1, h1) = res
    assert np.array_equal(c0, c1) and t0 == t1
    assert np.array_equal(p0, p1) and np.array_equal(h0, h1)
    assert np.array_equal(m0, m1)
    # forward only: nothing recorded to differentiate
    full.refit_forward(dc, rs, coef=coef, record=False)
    with pytest.raises(TpccaError):
        full.refit_backward(w)


@pytest.mark.parametrize("f64", [False, True])
def test_pass_checkpoints_equal_full_tape(f64):
    """Checkpoint mode: the forward keeps only each pass's starting point and
    the backward recomputes one pass at a time (last first) from it, carrying
    the adjoint between passes; with a budget that also forces batches. Every
    gradient bit-identical to the whole-set tape."""
    import torch

    from paper_1811_11481_amd import FLAG_ADJOINT_F64, DeviceClusters, RefitSet, Tracker, default_params, \
        default_tuning
    cs = synth.generate("C2")
    dc = DeviceClusters.from_host(cs)
    prm = default_params(flags=FLAG_ADJOINT_F64) if f64 else None
    full = Tracker(params=prm)
    full.track(dc)
    rs = RefitSet.from_tracker(full)
    log("checkpoint mode on %d tracks (binary%d adjoint)" % (rs.n_tracks, 64 if f64 else 32))
    coef = torch.as_tensor(_smooth_map(41), device="cuda")
    w = torch.as_tensor(np.random.default_rng(4).uniform(0.5, 2, rs.n_tracks), dtype=torch.float32, device="cuda")
    res = []
    for tr in (full, Tracker(params=prm, tuning=default_tuning(ckpt=1)),
               Tracker(params=prm, tuning=default_tuning(ckpt=1, tape_mb=2))):
        chi2, _, tot = tr.refit_forward(dc, rs, coef=coef)
        gp, gm, gh = tr.refit_backward(w, want_map=True, want_hits=True)
        res.append((chi2.cpu().numpy(), tot.item(), gp.cpu().numpy(), gm.cpu().numpy(), gh.cpu().numpy()))
    for c, t, p, m, h in res[1:]:
        assert np.array_equal(c, res[0][0]) and t == res[0][1]
        assert np.array_equal(p, res[0][2]) and np.array_equal(h, res[0][4]) and np.array_equal(m, res[0][3])

