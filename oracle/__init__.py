"""CPU oracle of the TPC track-finding hot path — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product path (the HIP library and its
binding) never loads it; the two share no code.

The arithmetic lives in ``tpc_oracle.cpp`` (plain, slow, brute force), built
with ``g++ -O2 -ffp-contract=off -fno-fast-math`` so that the binary32 mode
runs in IEEE single precision in the written operation order. This module
only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libtpcoracle.so")
_SRC = os.path.join(_HERE, "tpc_oracle.cpp")
CFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC", "-pthread"]


class Params(ctypes.Structure):
    _fields_ = [
        ("n_rows", ctypes.c_int32),
        ("bz", ctypes.c_double),
        ("sigma_y", ctypes.c_double),
        ("sigma_z", ctypes.c_double),
        ("win_ty", ctypes.c_double),
        ("win_tz", ctypes.c_double),
        ("win_ny", ctypes.c_double),
        ("win_nz", ctypes.c_double),
        ("nbr_score_max", ctypes.c_double),
        ("nsig", ctypes.c_double),
        ("chi2_pick", ctypes.c_double),
        ("chi2_rej", ctypes.c_double),
        ("sinphi_max", ctypes.c_double),
        ("cov_reset", ctypes.c_double),
        ("q_max", ctypes.c_double),
        ("u_max", ctypes.c_double),
        ("c0", ctypes.c_double * 5),
        ("n_min", ctypes.c_int32),
        ("max_miss", ctypes.c_int32),
        ("hits_per_bin", ctypes.c_int32),
        ("n_threads", ctypes.c_int32),
        ("planes_f32", ctypes.c_int32),
        ("chi2_merge", ctypes.c_double),
        ("merge_max_gap", ctypes.c_int32),
    ]


_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++"] + CFLAGS + [_SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.orc_default_params.argtypes = [ctypes.POINTER(Params)]
        L.orc_run.restype = vp
        L.orc_run.argtypes = [ctypes.POINTER(Params), i32, i32, vp, vp, vp, vp]
        L.orc_free.argtypes = [vp]
        L.orc_sizes.argtypes = [vp, vp]
        L.orc_get_grid.argtypes = [vp] + [vp] * 8
        L.orc_get_links.argtypes = [vp] + [vp] * 4
        L.orc_get_tracklets.argtypes = [vp] + [vp] * 8
        L.orc_get_selected.argtypes = [vp] + [vp] * 5
        L.orc_get_tracks.argtypes = [vp] + [vp] * 11
        L.orc_merge.restype = i64
        L.orc_merge.argtypes = [vp, ctypes.POINTER(Params), i32, vp, vp, vp, vp, vp]
        L.orc_merged_hits.restype = i64
        L.orc_merged_hits.argtypes = [vp]
        L.orc_get_merged.argtypes = [vp] + [vp] * 13
        L.orc_propagate.restype = i32
        L.orc_propagate.argtypes = [ctypes.POINTER(Params), i32, vp, dbl, dbl]
        L.orc_rotate.restype = i32
        L.orc_rotate.argtypes = [ctypes.POINTER(Params), i32, vp, vp, dbl]
        L.orc_update.restype = dbl
        L.orc_update.argtypes = [ctypes.POINTER(Params), i32, vp, dbl, dbl]
        L.orc_asin_over.restype = dbl
        L.orc_asin_over.argtypes = [i32, dbl]
        L.orc_seed.restype = i32
        L.orc_seed.argtypes = [ctypes.POINTER(Params), i32, vp, vp]
        L.orc_pick.restype = i64
        L.orc_pick.argtypes = [ctypes.POINTER(Params), i32, vp, i64, vp, vp, vp]
        L.orc_refit.restype = i32
        L.orc_refit.argtypes = [ctypes.POINTER(Params), i32, vp, i32, i32, vp, vp, vp, vp, vp, vp, vp]
        L.orc_replay_f64.argtypes = [ctypes.POINTER(Params), i64] + [vp] * 10
        L.orc_map_eval.argtypes = [vp, i64, vp, vp, vp, vp]
        L.orc_correct.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
        L.orc_refit_frozen_f64.argtypes = [ctypes.POINTER(Params), i64] + [vp] * 11
        L.orc_track_residuals.restype = i32
        L.orc_track_residuals.argtypes = [ctypes.POINTER(Params), vp, i32, i32, vp, vp, vp, i32, vp]
        L.orc_track_decode.restype = None
        L.orc_track_decode.argtypes = [ctypes.POINTER(Params), vp, i32, i32, vp, vp, i32, vp, vp]
        L.orc_vertex_z.restype = dbl
        L.orc_vertex_z.argtypes = [ctypes.POINTER(Params), dbl, vp]
        L.orc_fit_corrected.restype = None
        L.orc_fit_corrected.argtypes = [ctypes.POINTER(Params), i64] + [vp] * 16
        L.orc_native_to_local.restype = None
        L.orc_native_to_local.argtypes = [i32, i32, vp, vp, vp, vp, ctypes.c_float, ctypes.c_float, vp, vp, vp, vp]
        _lib = L
    return _lib


def default_params(**over) -> Params:
    p = Params()
    lib().orc_default_params(ctypes.byref(p))
    for k, v in over.items():
        if k == "c0":
            for i in range(5):
                p.c0[i] = v[i]
        else:
            setattr(p, k, v)
    return p


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


@dataclass
class OracleResult:
    precision: int
    n_rows: int
    # grid
    sorted_id: np.ndarray
    bin_start: np.ndarray
    g_ny: np.ndarray
    g_nz: np.ndarray
    g_meta: np.ndarray  # [n_seg, 4]: ymin zmin invy invz
    # CA links (input-id space)
    up: np.ndarray
    dn: np.ndarray
    upc: np.ndarray
    dnc: np.ndarray
    # starts / tracklets
    start_hit: np.ndarray
    start_inst: np.ndarray
    start_tid: np.ndarray
    tl_nhits: np.ndarray
    tl_rowhit: np.ndarray  # [N_s, n_rows]
    tl_state: np.ndarray  # [N_s, 20]
    tl_row: np.ndarray
    weight: np.ndarray
    # selected (pre-refit) tracks
    sel_tl: np.ndarray
    sel_hit_start: np.ndarray
    sel_hit: np.ndarray
    sel_mask: np.ndarray
    sel_status: np.ndarray
    # output tracks
    trk_inst: np.ndarray
    trk_sel: np.ndarray
    trk_x: np.ndarray
    trk_alpha: np.ndarray
    trk_param: np.ndarray  # [n_t, 5]
    trk_cov: np.ndarray  # [n_t, 15]
    trk_chi2: np.ndarray
    trk_ndf: np.ndarray
    trk_hit_start: np.ndarray
    trk_hit: np.ndarray
    chi2_total: float
    ndf_total: int

    @property
    def n_tracks(self) -> int:
        return int(self.trk_inst.shape[0])


def run(cs, precision: int = 32, params: Params | None = None, threads: int = 1, inst_event=None) -> OracleResult:
    """Track a ClusterSet (instances x rows CSR) with the oracle. With
    inst_event (the event of each instance) the sector tracks are also merged
    across sectors; the result then carries a `merged` dict."""
    L = lib()
    p = params if params is not None else default_params()
    p.n_threads = threads
    nr = p.n_rows
    inst_sector = np.ascontiguousarray(cs.inst_sector, dtype=np.int32)
    row_start = np.ascontiguousarray(cs.row_start, dtype=np.int64)
    y = np.ascontiguousarray(cs.y, dtype=np.float32)
    z = np.ascontiguousarray(cs.z, dtype=np.float32)
    h = L.orc_run(ctypes.byref(p), precision, int(cs.n_inst), inst_sector.ctypes.data, row_start.ctypes.data,
                  _ptr(y), _ptr(z))
    try:
        sz = np.zeros(6, np.int64)
        L.orc_sizes(h, sz.ctypes.data)
        N, ns, nsel, nselh, nt, nth = (int(v) for v in sz)
        nseg = int(cs.n_inst) * nr
        sorted_id = np.zeros(N, np.int32)
        bin_start = np.zeros(N + nseg + 1, np.int32)
        g_ny, g_nz = np.zeros(nseg, np.int32), np.zeros(nseg, np.int32)
        meta = [np.zeros(nseg, np.float64) for _ in range(4)]
        L.orc_get_grid(h, _ptr(sorted_id), _ptr(bin_start), _ptr(g_ny), _ptr(g_nz), *[_ptr(m) for m in meta])
        up, dn, upc, dnc = (np.zeros(N, np.int32) for _ in range(4))
        L.orc_get_links(h, _ptr(up), _ptr(dn), _ptr(upc), _ptr(dnc))
        start_hit, start_inst, start_tid, nhits = (np.zeros(ns, np.int32) for _ in range(4))
        rowhit = np.zeros(ns * nr, np.int32)
        state = np.zeros(ns * 20, np.float64)
        srow = np.zeros(ns, np.int32)
        weight = np.zeros(N, np.uint32)
        L.orc_get_tracklets(h, _ptr(start_hit), _ptr(start_inst), _ptr(start_tid), _ptr(nhits), _ptr(rowhit),
                            _ptr(state), _ptr(srow), _ptr(weight))
        sel_tl = np.zeros(nsel, np.int32)
        sel_hs = np.zeros(nsel + 1, np.int64)
        sel_hit = np.zeros(nselh, np.int32)
        sel_mask = np.zeros(nselh, np.uint8)
        sel_status = np.zeros(nsel, np.int32)
        L.orc_get_selected(h, _ptr(sel_tl), _ptr(sel_hs), _ptr(sel_hit), _ptr(sel_mask), _ptr(sel_status))
        ti, tsel, tndf = (np.zeros(nt, np.int32) for _ in range(3))
        tx, ta, tchi2 = (np.zeros(nt, np.float64) for _ in range(3))
        tpar = np.zeros(nt * 5, np.float64)
        tcov = np.zeros(nt * 15, np.float64)
        ths = np.zeros(nt + 1, np.int64)
        thit = np.zeros(nth, np.int32)
        tot = np.zeros(2, np.float64)
        L.orc_get_tracks(h, _ptr(ti), _ptr(tsel), _ptr(tx), _ptr(ta), _ptr(tpar), _ptr(tcov), _ptr(tchi2), _ptr(tndf),
                         _ptr(ths), _ptr(thit), _ptr(tot))
        merged = None
        if inst_event is not None:
            ev = np.ascontiguousarray(np.asarray(inst_event, dtype=np.int32))
            nm = int(L.orc_merge(h, ctypes.byref(p), int(cs.n_inst), inst_sector.ctypes.data, ev.ctypes.data,
                                 row_start.ctypes.data, _ptr(y), _ptr(z)))
            nmh = int(L.orc_merged_hits(h))
            m = {"next": np.zeros(nt, np.int32), "src": np.zeros(nm, np.int32), "nseg": np.zeros(nm, np.int32),
                 "inst": np.zeros(nm, np.int32), "x_ref": np.zeros(nm), "alpha": np.zeros(nm),
                 "param": np.zeros(nm * 5), "cov": np.zeros(nm * 15), "chi2": np.zeros(nm),
                 "ndf": np.zeros(nm, np.int32), "hit_start": np.zeros(nm + 1, np.int64),
                 "hit_id": np.zeros(nmh, np.int32), "state2": np.zeros(nt * 20)}
            L.orc_get_merged(h, *[_ptr(m[k]) for k in ("next", "src", "nseg", "inst", "x_ref", "alpha", "param",
                                                            "cov", "chi2", "ndf", "hit_start", "hit_id", "state2")])
            m["param"] = m["param"].reshape(nm, 5)
            m["cov"] = m["cov"].reshape(nm, 15)
            m["state2"] = m["state2"].reshape(nt, 20)
            merged = m
    finally:
        L.orc_free(h)
    res = OracleResult(
        precision, nr, sorted_id, bin_start, g_ny, g_nz, np.stack(meta, axis=1), up, dn, upc, dnc,
        start_hit, start_inst, start_tid, nhits, rowhit.reshape(ns, nr), state.reshape(ns, 20), srow, weight,
        sel_tl, sel_hs, sel_hit, sel_mask, sel_status, ti, tsel, tx, ta, tpar.reshape(nt, 5),
        tcov.reshape(nt, 15), tchi2, tndf, ths, thit, float(tot[0]), int(tot[1]))
    res.merged = merged
    return res


# ---------------------------------------------------------------- primitives
def propagate(state20, x1, x2, precision=64, params=None):
    p = params if params is not None else default_params()
    st = np.ascontiguousarray(np.array(state20, dtype=np.float64))
    if st.shape != (20,):
        raise ValueError("state must hold 5 parameters and 15 covariance terms")
    ok = lib().orc_propagate(ctypes.byref(p), precision, st.ctypes.data, float(x1), float(x2))
    return bool(ok), st


def rotate(state20, x, d, precision=64, params=None):
    """Rotate a state at local x into the frame turned by d; returns (ok, state20, new x)."""
    p = params if params is not None else default_params()
    st = np.ascontiguousarray(np.array(state20, dtype=np.float64))
    xx = np.array([x], np.float64)
    ok = lib().orc_rotate(ctypes.byref(p), precision, st.ctypes.data, xx.ctypes.data, float(d))
    return bool(ok), st, float(xx[0])


def update(state20, my, mz, precision=64, params=None):
    p = params if params is not None else default_params()
    st = np.ascontiguousarray(np.array(state20, dtype=np.float64))
    if st.shape != (20,):
        raise ValueError("state must hold 5 parameters and 15 covariance terms")
    chi2 = lib().orc_update(ctypes.byref(p), precision, st.ctypes.data, float(my), float(mz))
    return chi2, st


def asin_over(u, precision=64):
    return lib().orc_asin_over(precision, float(u))


def seed(points8, precision=64, params=None):
    p = params if params is not None else default_params()
    pts = np.ascontiguousarray(np.array(points8, dtype=np.float64))
    st = np.zeros(20, np.float64)
    ok = lib().orc_seed(ctypes.byref(p), precision, pts.ctypes.data, st.ctypes.data)
    return bool(ok), st


def pick(state20, ys, zs, precision=64, params=None):
    """The track-following pick rule on one row: index of the chosen candidate
    (input order) or -1, and its predicted chi2 (None if nothing is picked)."""
    p = params if params is not None else default_params()
    st = np.ascontiguousarray(np.array(state20, dtype=np.float64))
    if st.shape != (20,):
        raise ValueError("state must hold 5 parameters and 15 covariance terms")
    ys = np.ascontiguousarray(np.asarray(ys, dtype=np.float32))
    zs = np.ascontiguousarray(np.asarray(zs, dtype=np.float32))
    if ys.shape != zs.shape:
        raise ValueError("ys and zs must have equal length")
    chi2 = ctypes.c_double(0.0)
    c = lib().orc_pick(ctypes.byref(p), precision, st.ctypes.data, len(ys), _ptr(ys), _ptr(zs), ctypes.byref(chi2))
    return int(c), (chi2.value if c >= 0 else None)


def refit(state20, row, rows, ys, zs, precision=64, params=None, replay=None):
    """Three-pass refit of one hit list; returns (ok, state20, chi2, nacc, row, masks)."""
    p = params if params is not None else default_params()
    st0 = np.ascontiguousarray(np.array(state20, dtype=np.float64))
    if st0.shape != (20,):
        raise ValueError("state must hold 5 parameters and 15 covariance terms")
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int32))
    if len(ys) != len(rows) or len(zs) != len(rows):
        raise ValueError("rows, ys and zs must have equal length")
    ys = np.ascontiguousarray(np.asarray(ys, dtype=np.float64))
    zs = np.ascontiguousarray(np.asarray(zs, dtype=np.float64))
    n = len(rows)
    masks = np.zeros(max(n, 1), np.uint8)
    rp = None if replay is None else np.ascontiguousarray(np.asarray(replay, dtype=np.uint8))
    out = np.zeros(20, np.float64)
    sc = np.zeros(3, np.float64)
    ok = lib().orc_refit(ctypes.byref(p), precision, st0.ctypes.data, int(row), n, _ptr(rows), _ptr(ys), _ptr(zs),
                         _ptr(rp), masks.ctypes.data, out.ctypes.data, sc.ctypes.data)
    return bool(ok), out, sc[0], int(sc[1]), int(sc[2]), masks[:n]


def replay_f64(st0, row0, hit_start, hit_rows, ys, zs, masks, params=None, planes_f32=True):
    """FP64 replay of refits with given start states and accept masks.

    The comparison of the binary32 tracker with binary64 arithmetic is made on
    the same hits, masks and detector: by default the pad-row planes are the
    binary32 positions the tracker is given (its row_x parameters), not their
    exact decimal values, which differ by up to 7.6e-6 cm. That difference
    alone moves the q/pT of a short track by ~1e-4 of its scale, and it is a
    difference of geometry, not of arithmetic precision."""
    p = Params.from_buffer_copy(params if params is not None else default_params())
    p.planes_f32 = 1 if planes_f32 else 0
    n = len(row0)
    st0 = np.ascontiguousarray(np.asarray(st0, dtype=np.float64).reshape(n, 20))
    row0 = np.ascontiguousarray(np.asarray(row0, dtype=np.int32))
    hit_start = np.ascontiguousarray(np.asarray(hit_start, dtype=np.int64))
    hit_rows = np.ascontiguousarray(np.asarray(hit_rows, dtype=np.int32))
    ys = np.ascontiguousarray(np.asarray(ys, dtype=np.float64))
    zs = np.ascontiguousarray(np.asarray(zs, dtype=np.float64))
    masks = np.ascontiguousarray(np.asarray(masks, dtype=np.uint8))
    out = np.zeros((n, 20), np.float64)
    chi2 = np.zeros(n, np.float64)
    ok = np.zeros(n, np.int32)
    lib().orc_replay_f64(ctypes.byref(p), n, _ptr(st0), _ptr(row0), _ptr(hit_start), _ptr(hit_rows), _ptr(ys),
                         _ptr(zs), _ptr(masks), _ptr(out), _ptr(chi2), _ptr(ok))
    return ok.astype(bool), out, chi2


# ------------------------------------------------------- differentiable refit
MAP_SHAPE = (3, 16, 16, 32)  # components (delta r, delta r*phi, delta z) x r x phi x z
MAP_SIZE = 3 * 16 * 16 * 32


def map_eval(coef, r, phi, z):
    """Map components (n, 3) at global (r, phi, z)."""
    coef = np.ascontiguousarray(np.asarray(coef, np.float64).reshape(-1))
    r, phi, z = (np.ascontiguousarray(np.asarray(v, np.float64).reshape(-1)) for v in (r, phi, z))
    out = np.zeros((len(r), 3), np.float64)
    lib().orc_map_eval(_ptr(coef), len(r), _ptr(r), _ptr(phi), _ptr(z), _ptr(out))
    return out


def correct(coef, alpha, x, y, z):
    coef = np.ascontiguousarray(np.asarray(coef, np.float64).reshape(-1))
    a, x, y, z = (np.ascontiguousarray(np.asarray(v, np.float64).reshape(-1)) for v in (alpha, x, y, z))
    yc, zc = np.zeros(len(y)), np.zeros(len(y))
    lib().orc_correct(_ptr(coef), len(y), _ptr(a), _ptr(x), _ptr(y), _ptr(z), _ptr(yc), _ptr(zc))
    return yc, zc


def refit_frozen_f64(st0, row0, alpha, hit_start, hit_rows, ys, zs, masks, coef=None, params=None):
    """Per-track pass-3 chi2 (FP64) of the refit with frozen masks on corrected clusters."""
    p = params if params is not None else default_params()
    n = len(row0)
    st0 = np.ascontiguousarray(np.asarray(st0, np.float64).reshape(n, 20))
    row0 = np.ascontiguousarray(np.asarray(row0, np.int32))
    alpha = np.ascontiguousarray(np.asarray(alpha, np.float64))
    hit_start = np.ascontiguousarray(np.asarray(hit_start, np.int64))
    hit_rows = np.ascontiguousarray(np.asarray(hit_rows, np.int32))
    ys = np.ascontiguousarray(np.asarray(ys, np.float64))
    zs = np.ascontiguousarray(np.asarray(zs, np.float64))
    masks = np.ascontiguousarray(np.asarray(masks, np.uint8))
    cf = None if coef is None else np.ascontiguousarray(np.asarray(coef, np.float64).reshape(-1))
    chi2 = np.zeros(n)
    ok = np.zeros(n, np.int32)
    lib().orc_refit_frozen_f64(ctypes.byref(p), n, _ptr(st0), _ptr(row0), _ptr(alpha), _ptr(hit_start),
                               _ptr(hit_rows), _ptr(ys), _ptr(zs), _ptr(masks), _ptr(cf), _ptr(chi2), _ptr(ok))
    return ok.astype(bool), chi2


def refit_inputs(res: OracleResult, cs, only_ok: bool = True):
    """Inputs of the frozen-mask refit for the selected tracks of an oracle run:
    start state (tracklet state), its row, sector angle, hit rows/coordinates and
    the accept masks the refit took (pass p in bit p)."""
    status = res.sel_status.astype(bool) if only_ok else np.ones(len(res.sel_tl), bool)
    idx = np.nonzero(status)[0]
    hs = res.sel_hit_start
    lens = (hs[idx + 1] - hs[idx]).astype(np.int64)
    hit_start = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    pos = np.concatenate([np.arange(hs[i], hs[i + 1]) for i in idx]) if len(idx) else np.zeros(0, np.int64)
    hits = res.sel_hit[pos]
    seg = np.searchsorted(cs.row_start, hits, side="right") - 1
    rows = (seg % res.n_rows).astype(np.int32)
    inst = res.start_inst[res.sel_tl[idx]]
    sector = cs.inst_sector[inst]
    alpha = ((sector % 18) + 0.5) * (20.0 * np.pi / 180.0)
    return dict(st0=res.tl_state[res.sel_tl[idx]].astype(np.float64), row0=res.tl_row[res.sel_tl[idx]],
                alpha=alpha, hit_start=hit_start, hit_rows=rows, hit_id=hits.astype(np.int32),
                ys=cs.y[hits].astype(np.float64), zs=cs.z[hits].astype(np.float64), masks=res.sel_mask[pos],
                inst=inst.astype(np.int32), sel=idx)


def frozen_chi2_grad_fd(inp, coef=None, coef_index=(), h_param=(1e-4, 1e-4, 1e-6, 1e-6, 1e-5), h_coef=1e-4,
                        params=None):
    """Reference gradient of the frozen-mask refit chi2 by central differences of
    the FP64 function: d chi2_t / d params0_t (n x 5, each track's chi2 depends
    only on its own start state, so one perturbation serves all tracks) and
    d (sum_t chi2_t) / d coef[k] for the flat coefficient indices in coef_index.
    h_param: steps for the five start parameters, a 5-vector or per track (n x 5)."""
    base = np.zeros(MAP_SIZE) if coef is None else np.asarray(coef, np.float64).reshape(-1).copy()
    use_map = coef is not None or len(coef_index) > 0

    def f(st0, cf):
        ok, chi2 = refit_frozen_f64(st0, inp["row0"], inp["alpha"], inp["hit_start"], inp["hit_rows"], inp["ys"],
                                    inp["zs"], inp["masks"], cf if use_map else None, params)
        return ok, chi2

    st0 = np.asarray(inp["st0"], np.float64)
    gp = np.zeros((len(st0), 5))
    hp = np.broadcast_to(np.asarray(h_param, np.float64), (len(st0), 5))
    ok_all = f(st0, base)[0]
    for k in range(5):
        sp, sm = st0.copy(), st0.copy()
        sp[:, k] += hp[:, k]
        sm[:, k] -= hp[:, k]
        okp, cp = f(sp, base)
        okm, cm = f(sm, base)
        ok_all &= okp & okm
        gp[:, k] = (cp - cm) / (2.0 * hp[:, k])
    gc = np.zeros(len(coef_index))
    for j, k in enumerate(coef_index):
        cpl, cmi = base.copy(), base.copy()
        cpl[k] += h_coef
        cmi[k] -= h_coef
        okp, cp = f(st0, cpl)
        okm, cm = f(st0, cmi)
        ok_all &= okp & okm
        gc[j] = (cp[okp & okm].sum() - cm[okp & okm].sum()) / (2.0 * h_coef)
    return ok_all, gp, gc


def vertex_z(x, states, params=None):
    """z of the point of closest approach to the beam line (FP64) of each track
    state (y, z, sin phi, tan lambda, q/pT) at local x."""
    p = params if params is not None else default_params()
    x = np.broadcast_to(np.asarray(x, np.float64), (len(states),))
    st = np.ascontiguousarray(np.asarray(states, np.float64).reshape(-1, 5))
    L = lib()
    return np.array([L.orc_vertex_z(ctypes.byref(p), float(x[i]), st[i].ctypes.data) for i in range(len(st))])


RES_ESCAPE = -32768


def track_residuals(params5, rows, ys, zs, step_log2=-7, params=None, row0=None):
    """Quantised residuals (int16 [n, 2]) of a track's clusters (rows
    ascending) to the binary32 track model started from params5 at row0 (the
    first cluster's row by default); returns (residuals, number of escaped
    values)."""
    p = params if params is not None else default_params()
    pr = np.ascontiguousarray(np.asarray(params5, np.float64))
    rows = np.ascontiguousarray(np.asarray(rows, np.int32))
    ys = np.ascontiguousarray(np.asarray(ys, np.float64))
    zs = np.ascontiguousarray(np.asarray(zs, np.float64))
    q = np.zeros((max(len(rows), 1), 2), np.int16)
    r0 = int(rows[0]) if row0 is None else int(row0)
    n_esc = lib().orc_track_residuals(ctypes.byref(p), pr.ctypes.data, r0, len(rows), _ptr(rows), _ptr(ys),
                                      _ptr(zs), int(step_log2), q.ctypes.data)
    return q[:len(rows)], int(n_esc)


def track_decode(params5, rows, q, step_log2=-7, params=None, row0=None):
    """Clusters (ys, zs) decoded from the parameters, rows and residuals."""
    p = params if params is not None else default_params()
    pr = np.ascontiguousarray(np.asarray(params5, np.float64))
    rows = np.ascontiguousarray(np.asarray(rows, np.int32))
    q = np.ascontiguousarray(np.asarray(q, np.int16).reshape(-1, 2))
    ys, zs = np.zeros(max(len(rows), 1)), np.zeros(max(len(rows), 1))
    r0 = int(rows[0]) if row0 is None else int(row0)
    lib().orc_track_decode(ctypes.byref(p), pr.ctypes.data, r0, len(rows), _ptr(rows), q.ctypes.data,
                           int(step_log2), ys.ctypes.data, zs.ctypes.data)
    return ys[:len(rows)], zs[:len(rows)]


# ---------------------------------------------------------------- native coordinates
def native_geometry(row_x=None) -> dict:
    """Pad geometry and drift constants of native cluster coordinates (the
    readings for Sections 4 and 6): pad pitch 0.416 cm on rows 0-62, 0.42 cm on
    63-126 and 0.46 cm on 127-151 (the four readout regions of 63, 34, 30 and 25
    rows); each row has the even number of pads that covers its full width
    2 x tan(10 deg) at its plane, and pad coordinate (n_pads - 1) / 2 is local
    y = 0; drift 2.58 cm/us sampled every 200 ns (0.516 cm per time bin);
    readout planes at |z| = 250 cm. Values as binary32, as the tracker uses them."""
    import math
    if row_x is None:
        row_x = [float(np.float32(85.0 + i * 162.0 / 151.0)) for i in range(152)]
    t10 = math.tan(10.0 * math.pi / 180.0)
    width = np.array([0.416 if i < 63 else 0.42 if i < 127 else 0.46 for i in range(len(row_x))])
    n_pads = np.array([2.0 * math.ceil(float(x) * t10 / w) for x, w in zip(row_x, width)])
    return dict(pad_width=width.astype(np.float32), pad_center=((n_pads - 1.0) * 0.5).astype(np.float32),
                n_pads=n_pads.astype(np.int64), z_per_bin=np.float32(2.58 * 0.2), z_readout=np.float32(250.0))


def native_to_local(n_rows, inst_sector, row_start, pad, time, geo=None):
    """Local (y, z) binary32 of clusters given in native (pad, time) (orc_native_to_local)."""
    geo = geo or native_geometry()
    sec = np.ascontiguousarray(inst_sector, np.int32)
    rs = np.ascontiguousarray(row_start, np.int64)
    pad = np.ascontiguousarray(pad, np.float32)
    time = np.ascontiguousarray(time, np.float32)
    pw = np.ascontiguousarray(geo["pad_width"], np.float32)
    pc = np.ascontiguousarray(geo["pad_center"], np.float32)
    y = np.zeros(len(pad), np.float32)
    z = np.zeros(len(pad), np.float32)
    lib().orc_native_to_local(int(n_rows), len(sec), _ptr(sec), _ptr(rs), _ptr(pw), _ptr(pc),
                              float(geo["z_per_bin"]), float(geo["z_readout"]), _ptr(pad), _ptr(time), _ptr(y), _ptr(z))
    return y, z


def fit_corrected(st0, row0, z0, alpha, hit_start, hit_rows, ys, zs, coef=None, params=None):
    """FP64 corrected final fit (orc_fit_corrected): per track, clusters and
    start state moved to the absolute frame by the track's vertex z, clusters
    corrected by the map (coef [3*16*16*32] or None), three passes with chi2
    rejection. Returns dict(ok, state [n,20], chi2, nacc, row, z0, masks)."""
    p = params if params is not None else default_params(planes_f32=1)
    st0 = np.ascontiguousarray(st0, np.float64)
    n = len(st0)
    row0 = np.ascontiguousarray(row0, np.int32)
    z0 = np.ascontiguousarray(z0, np.float64)
    alpha = np.ascontiguousarray(alpha, np.float64)
    hs = np.ascontiguousarray(hit_start, np.int64)
    rows = np.ascontiguousarray(hit_rows, np.int32)
    ys = np.ascontiguousarray(ys, np.float64)
    zs = np.ascontiguousarray(zs, np.float64)
    cf = None if coef is None else np.ascontiguousarray(coef, np.float64)
    out = dict(state=np.zeros((n, 20)), chi2=np.zeros(n), nacc=np.zeros(n, np.int32), row=np.zeros(n, np.int32),
               z0=np.zeros(n), ok=np.zeros(n, np.int32), masks=np.zeros(max(len(rows), 1), np.uint8))
    lib().orc_fit_corrected(ctypes.byref(p), n, _ptr(st0), _ptr(row0), _ptr(z0), _ptr(alpha), _ptr(hs), _ptr(rows),
                            _ptr(ys), _ptr(zs), _ptr(cf), _ptr(out["state"]), _ptr(out["chi2"]), _ptr(out["nacc"]),
                            _ptr(out["row"]), _ptr(out["z0"]), _ptr(out["ok"]), _ptr(out["masks"]))
    out["masks"] = out["masks"][:len(rows)]
    return out
