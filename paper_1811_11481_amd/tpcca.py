"""ctypes binding of libtpcca.so (include/tpcca.h).

Argument marshalling only: torch allocates device memory and supplies the
HIP stream; every step of the tracking runs in the HIP library. Importing
works without a GPU (the CPU tests check the exported symbols); any compute
call needs the built library and a HIP device and fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtpcca.so")

OK, E_ARG, E_CAPACITY, E_DEVICE, E_OOM, E_INTERNAL = range(6)
FLAG_STATS = 1
FLAG_TIMING = 2
FLAG_ADJOINT_F64 = 4
FLAG_MERGE = 8
MAP_SHAPE = (3, 16, 16, 32)  # (delta r, delta r*phi, delta z) x r x phi x z
MAP_SIZE = 3 * 16 * 16 * 32
MAX_ROW_CLUSTERS = 16384
STATUS_NAMES = {0: "OK", 1: "E_ARG", 2: "E_CAPACITY", 3: "E_DEVICE", 4: "E_OOM", 5: "E_INTERNAL"}

# every extern "C" symbol of include/tpcca.h
EXPORTED = [
    "tpcca_default_params", "tpcca_default_tuning", "tpcca_create", "tpcca_destroy", "tpcca_last_error",
    "tpcca_set_tuning", "tpcca_get_tuning", "tpcca_track", "tpcca_track_batched", "tpcca_track_async",
    "tpcca_track_async_noalloc", "tpcca_merge", "tpcca_track_native", "tpcca_native_to_local", "tpcca_autotune",
    "tpcca_export_sizes", "tpcca_export_grid", "tpcca_export_links", "tpcca_export_tracklets",
    "tpcca_export_selected", "tpcca_get_stats", "tpcca_get_stage_times", "tpcca_fp32_selfcheck",
    "tpcca_refit_fwd", "tpcca_refit_bwd", "tpcca_fit_corrected", "tpcca_sqrt_step_check",
]


class TpccaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("n_rows", ctypes.c_int32),
        ("row_x", ctypes.c_float * 256),
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
        ("flags", ctypes.c_uint32),
        ("chi2_merge", ctypes.c_double),
        ("merge_max_gap", ctypes.c_int32),
        ("pad_width", ctypes.c_float * 256),
        ("pad_center", ctypes.c_float * 256),
        ("z_per_bin", ctypes.c_double),
        ("z_readout", ctypes.c_double),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [
        ("hits_per_bin", ctypes.c_int32),
        ("block_links", ctypes.c_int32),
        ("block_tracklet", ctypes.c_int32),
        ("block_refit", ctypes.c_int32),
        ("block_scan", ctypes.c_int32),
        ("sort_seeds", ctypes.c_int32),
        ("tape_mb", ctypes.c_int32),
        ("xcd_remap", ctypes.c_int32),
        ("ckpt", ctypes.c_int32),
        ("inward_wgs", ctypes.c_int32),
        ("inward_sort", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Clusters(ctypes.Structure):
    _fields_ = [
        ("n_inst", ctypes.c_int32),
        ("inst_sector", ctypes.c_void_p),
        ("row_start", ctypes.c_void_p),
        ("y", ctypes.c_void_p),
        ("z", ctypes.c_void_p),
        ("n_clusters", ctypes.c_int64),
    ]


class NativeClustersC(ctypes.Structure):
    _fields_ = [
        ("n_inst", ctypes.c_int32),
        ("inst_sector", ctypes.c_void_p),
        ("row_start", ctypes.c_void_p),
        ("pad", ctypes.c_void_p),
        ("time", ctypes.c_void_p),
        ("n_clusters", ctypes.c_int64),
    ]


class TracksC(ctypes.Structure):
    _fields_ = [
        ("cap_tracks", ctypes.c_int64),
        ("cap_hits", ctypes.c_int64),
        ("inst", ctypes.c_void_p),
        ("x_ref", ctypes.c_void_p),
        ("alpha", ctypes.c_void_p),
        ("param", ctypes.c_void_p),
        ("cov", ctypes.c_void_p),
        ("chi2", ctypes.c_void_p),
        ("ndf", ctypes.c_void_p),
        ("hit_start", ctypes.c_void_p),
        ("hit_id", ctypes.c_void_p),
        ("chi2_total", ctypes.c_void_p),
        ("z0", ctypes.c_void_p),
        ("residuals", ctypes.c_void_p),
        ("residual_step_log2", ctypes.c_int32),
        ("n_tracks", ctypes.c_int64),
        ("n_hits", ctypes.c_int64),
    ]


class RefitSetC(ctypes.Structure):
    _fields_ = [
        ("n_tracks", ctypes.c_int64),
        ("n_hits", ctypes.c_int64),
        ("params0", ctypes.c_void_p),
        ("cov0", ctypes.c_void_p),
        ("row0", ctypes.c_void_p),
        ("inst", ctypes.c_void_p),
        ("hit_start", ctypes.c_void_p),
        ("hit_id", ctypes.c_void_p),
        ("hit_mask", ctypes.c_void_p),
    ]


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "n_clusters", "n_segments", "n_links", "n_starts", "n_chain_hits", "tl_rows_visited", "tl_candidates",
        "tl_picks", "n_selected", "n_selected_hits", "n_tracks", "n_track_hits", "rf_rows_visited",
        "rf_hit_visits", "nb_candidates_u", "nb_pairs")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def load():
    """Load libtpcca.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libtpcca.so is not built: run __graft_entry__.build() (hipcc, gfx950)")
        # torch first: its HIP runtime then satisfies the library's runtime
        # dependency, so both share one runtime (streams, synchronisation,
        # device memory). Loaded the other way round the process would hold
        # two runtimes and the second could not open the device.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        st = ctypes.c_int
        L.tpcca_default_params.restype = st
        L.tpcca_default_params.argtypes = [ctypes.POINTER(Params)]
        L.tpcca_default_tuning.restype = st
        L.tpcca_default_tuning.argtypes = [ctypes.POINTER(Tuning)]
        L.tpcca_create.restype = st
        L.tpcca_create.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Tuning), ctypes.c_int,
                                   ctypes.POINTER(vp)]
        L.tpcca_destroy.restype = None
        L.tpcca_destroy.argtypes = [vp]
        L.tpcca_last_error.restype = ctypes.c_char_p
        L.tpcca_last_error.argtypes = [vp]
        L.tpcca_set_tuning.restype = st
        L.tpcca_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.tpcca_get_tuning.restype = st
        L.tpcca_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        for fn in ("tpcca_track", "tpcca_track_batched"):
            getattr(L, fn).restype = st
            getattr(L, fn).argtypes = [vp, ctypes.POINTER(Clusters), ctypes.POINTER(TracksC), vp]
        for fn in ("tpcca_track_async", "tpcca_track_async_noalloc"):
            getattr(L, fn).restype = st
            getattr(L, fn).argtypes = [vp, ctypes.POINTER(Clusters), ctypes.POINTER(TracksC), vp, vp, vp]
        L.tpcca_track_native.restype = st
        L.tpcca_track_native.argtypes = [vp, ctypes.POINTER(NativeClustersC), ctypes.POINTER(TracksC), vp]
        L.tpcca_native_to_local.restype = st
        L.tpcca_native_to_local.argtypes = [vp, ctypes.POINTER(NativeClustersC), vp, vp, vp]
        L.tpcca_merge.restype = st
        L.tpcca_merge.argtypes = [vp, vp, ctypes.POINTER(TracksC), vp, vp, vp]
        L.tpcca_autotune.restype = st
        L.tpcca_autotune.argtypes = [vp, ctypes.POINTER(Clusters), i32, ctypes.POINTER(Tuning), vp]
        L.tpcca_export_sizes.restype = st
        L.tpcca_export_sizes.argtypes = [vp, vp, vp]
        L.tpcca_export_grid.restype = st
        L.tpcca_export_grid.argtypes = [vp] * 7
        L.tpcca_export_links.restype = st
        L.tpcca_export_links.argtypes = [vp] * 6
        L.tpcca_export_tracklets.restype = st
        L.tpcca_export_tracklets.argtypes = [vp] * 10
        L.tpcca_export_selected.restype = st
        L.tpcca_export_selected.argtypes = [vp] * 7
        L.tpcca_get_stats.restype = st
        L.tpcca_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.tpcca_get_stage_times.restype = st
        L.tpcca_get_stage_times.argtypes = [vp, vp]
        L.tpcca_fp32_selfcheck.restype = st
        L.tpcca_fp32_selfcheck.argtypes = [vp, vp, vp, vp, i64, vp]
        L.tpcca_sqrt_step_check.restype = st
        L.tpcca_sqrt_step_check.argtypes = [ctypes.c_uint32, ctypes.c_uint32, vp, vp]
        L.tpcca_refit_fwd.restype = st
        L.tpcca_refit_fwd.argtypes = [vp, ctypes.POINTER(Clusters), ctypes.POINTER(RefitSetC), vp, vp, vp, vp,
                                      i32, vp]
        L.tpcca_fit_corrected.restype = st
        L.tpcca_fit_corrected.argtypes = [vp] * 11
        L.tpcca_refit_bwd.restype = st
        L.tpcca_refit_bwd.argtypes = [vp] * 6
        _lib = L
    return _lib


def default_params(**over) -> Params:
    p = Params()
    load().tpcca_default_params(ctypes.byref(p))
    for k, v in over.items():
        if k == "c0":
            for i in range(5):
                p.c0[i] = v[i]
        else:
            setattr(p, k, v)
    return p


def default_tuning(**over) -> Tuning:
    t = Tuning()
    load().tpcca_default_tuning(ctypes.byref(t))
    for k, v in over.items():
        setattr(t, k, v)
    return t


def _torch():
    import torch

    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else None


@dataclass
class DeviceClusters:
    """Clusters resident in device memory (torch tensors)."""

    n_inst: int
    inst_sector: "object"  # int32 [n_inst]
    row_start: "object"  # int64 [n_inst * n_rows + 1]
    y: "object"  # float32 [N]
    z: "object"  # float32 [N]

    @property
    def n_clusters(self) -> int:
        return int(self.y.shape[0])

    @classmethod
    def from_host(cls, cs, device="cuda"):
        torch = _torch()
        return cls(int(cs.n_inst),
                   torch.as_tensor(np.asarray(cs.inst_sector, np.int32), device=device),
                   torch.as_tensor(np.asarray(cs.row_start, np.int64), device=device),
                   torch.as_tensor(np.asarray(cs.y, np.float32), device=device),
                   torch.as_tensor(np.asarray(cs.z, np.float32), device=device))

    def c_struct(self) -> Clusters:
        c = Clusters()
        c.n_inst = self.n_inst
        c.inst_sector = self.inst_sector.data_ptr() if self.n_inst else None
        c.row_start = self.row_start.data_ptr()
        c.y = self.y.data_ptr() if self.n_clusters else None
        c.z = self.z.data_ptr() if self.n_clusters else None
        c.n_clusters = self.n_clusters
        return c


@dataclass
class DeviceNativeClusters:
    """Clusters in native coordinates (pad, time per cluster) in device memory."""

    n_inst: int
    inst_sector: "object"  # int32 [n_inst]
    row_start: "object"  # int64 [n_inst * n_rows + 1]
    pad: "object"  # float32 [N]
    time: "object"  # float32 [N]

    @property
    def n_clusters(self) -> int:
        return int(self.pad.shape[0])

    @property
    def y(self):  # for capacity sizing and the device of outputs
        return self.pad

    @classmethod
    def from_host(cls, n_inst, inst_sector, row_start, pad, time, device="cuda"):
        torch = _torch()
        return cls(int(n_inst),
                   torch.as_tensor(np.asarray(inst_sector, np.int32), device=device),
                   torch.as_tensor(np.asarray(row_start, np.int64), device=device),
                   torch.as_tensor(np.asarray(pad, np.float32), device=device),
                   torch.as_tensor(np.asarray(time, np.float32), device=device))

    def c_struct(self) -> NativeClustersC:
        c = NativeClustersC()
        c.n_inst = self.n_inst
        c.inst_sector = self.inst_sector.data_ptr() if self.n_inst else None
        c.row_start = self.row_start.data_ptr()
        c.pad = self.pad.data_ptr() if self.n_clusters else None
        c.time = self.time.data_ptr() if self.n_clusters else None
        c.n_clusters = self.n_clusters
        return c


class Tracks:
    """Output track arrays (device tensors) with capacities."""

    def __init__(self, cap_tracks, cap_hits, device="cuda"):
        torch = _torch()
        self.cap_tracks, self.cap_hits = int(cap_tracks), int(cap_hits)
        ct = max(self.cap_tracks, 1)
        self.inst = torch.empty(ct, dtype=torch.int32, device=device)
        self.x_ref = torch.empty(ct, dtype=torch.float32, device=device)
        self.alpha = torch.empty(ct, dtype=torch.float32, device=device)
        self.param = torch.empty(ct * 5, dtype=torch.float32, device=device)
        self.cov = torch.empty(ct * 15, dtype=torch.float32, device=device)
        self.chi2 = torch.empty(ct, dtype=torch.float32, device=device)
        self.ndf = torch.empty(ct, dtype=torch.int32, device=device)
        self.hit_start = torch.empty(ct + 1, dtype=torch.int64, device=device)
        self.hit_id = torch.empty(max(self.cap_hits, 1), dtype=torch.int32, device=device)
        self.chi2_total = torch.empty(2, dtype=torch.float64, device=device)
        self.z0 = torch.empty(ct, dtype=torch.float32, device=device)
        self.residuals = None  # int16 [cap_hits * 2] when compression residuals are wanted
        self.residual_step_log2 = -7
        self.n_tracks = 0
        self.n_hits = 0

    def c_struct(self) -> TracksC:
        t = TracksC()
        t.cap_tracks, t.cap_hits = self.cap_tracks, self.cap_hits
        for k in ("inst", "x_ref", "alpha", "param", "cov", "chi2", "ndf", "hit_start", "hit_id", "chi2_total", "z0"):
            setattr(t, k, getattr(self, k).data_ptr())
        t.residuals = self.residuals.data_ptr() if self.residuals is not None else None
        t.residual_step_log2 = self.residual_step_log2
        return t

    def want_residuals(self, step_log2: int = -7):
        """Ask the track calls for track-model compression residuals (step 2^k cm)."""
        torch = _torch()
        self.residuals = torch.empty(max(self.cap_hits, 1) * 2, dtype=torch.int16, device=self.hit_id.device)
        self.residual_step_log2 = int(step_log2)
        return self

    def to_numpy(self) -> dict:
        n, h = self.n_tracks, self.n_hits
        return {
            "inst": self.inst[:n].cpu().numpy(), "x_ref": self.x_ref[:n].cpu().numpy(),
            "alpha": self.alpha[:n].cpu().numpy(), "param": self.param[:n * 5].cpu().numpy().reshape(n, 5),
            "cov": self.cov[:n * 15].cpu().numpy().reshape(n, 15), "chi2": self.chi2[:n].cpu().numpy(),
            "ndf": self.ndf[:n].cpu().numpy(), "hit_start": self.hit_start[:n + 1].cpu().numpy(),
            "hit_id": self.hit_id[:h].cpu().numpy(), "chi2_total": self.chi2_total.cpu().numpy(),
            "z0": self.z0[:n].cpu().numpy(),
            **({"residuals": self.residuals[:2 * h].cpu().numpy().reshape(h, 2)} if self.residuals is not None
               else {}),
        }


class Tracker:
    """One library context on one device."""

    def __init__(self, params: Params | None = None, tuning: Tuning | None = None, device: int = 0):
        self.lib = load()
        self.params = params if params is not None else default_params()
        self.h = ctypes.c_void_p()
        st = self.lib.tpcca_create(ctypes.byref(self.params), ctypes.byref(tuning) if tuning else None, device,
                                   ctypes.byref(self.h))
        if st != OK:
            raise TpccaError(st, "tpcca_create failed")

    def close(self):
        if self.h:
            self.lib.tpcca_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != OK:
            raise TpccaError(st, self.lib.tpcca_last_error(self.h).decode())

    @property
    def tuning(self) -> Tuning:
        t = Tuning()
        self._check(self.lib.tpcca_get_tuning(self.h, ctypes.byref(t)))
        return t

    def set_tuning(self, t: Tuning):
        self._check(self.lib.tpcca_set_tuning(self.h, ctypes.byref(t)))

    def alloc_tracks(self, clusters: DeviceClusters) -> Tracks:
        n = clusters.n_clusters
        return Tracks(n // self.params.n_min + clusters.n_inst + 1, max(n, 1), device=clusters.y.device)

    def track(self, clusters: DeviceClusters, out: Tracks | None = None, batched: bool = True, stream=None,
              check: bool = True) -> Tracks:
        out = out if out is not None else self.alloc_tracks(clusters)
        cin, cout = clusters.c_struct(), out.c_struct()
        fn = self.lib.tpcca_track_batched if batched else self.lib.tpcca_track
        st = fn(self.h, ctypes.byref(cin), ctypes.byref(cout), _stream(stream))
        out.n_tracks, out.n_hits = int(cout.n_tracks), int(cout.n_hits)
        if check:
            self._check(st)
        out.status = st
        return out

    def track_native(self, clusters: DeviceNativeClusters, out: Tracks | None = None, stream=None,
                     check: bool = True) -> Tracks:
        """Batched track call on native (pad, time) clusters, transformed by the grid kernel."""
        out = out if out is not None else self.alloc_tracks(clusters)
        cin, cout = clusters.c_struct(), out.c_struct()
        st = self.lib.tpcca_track_native(self.h, ctypes.byref(cin), ctypes.byref(cout), _stream(stream))
        out.n_tracks, out.n_hits = int(cout.n_tracks), int(cout.n_hits)
        if check:
            self._check(st)
        out.status = st
        return out

    def native_to_local(self, clusters: DeviceNativeClusters, stream=None):
        """Local (y, z) float32 device tensors of native clusters (the library's transform)."""
        torch = _torch()
        n = clusters.n_clusters
        y = torch.empty(max(n, 1), dtype=torch.float32, device=clusters.pad.device)
        z = torch.empty(max(n, 1), dtype=torch.float32, device=clusters.pad.device)
        c = clusters.c_struct()
        self._check(self.lib.tpcca_native_to_local(self.h, ctypes.byref(c), _ptr(y), _ptr(z), _stream(stream)))
        return y[:n], z[:n]

    def track_async(self, clusters: DeviceClusters, out: Tracks, counts, status, stream=None) -> Tracks:
        """Batched form with nothing read back: `counts` (int64[2] device tensor)
        receives (n_tracks, n_hits) and `status` (int32[1]) the status code when
        the stream reaches the end of the call; out.n_tracks / n_hits are not set."""
        cin, cout = clusters.c_struct(), out.c_struct()
        self._check(self.lib.tpcca_track_async(self.h, ctypes.byref(cin), ctypes.byref(cout), _ptr(counts),
                                               _ptr(status), _stream(stream)))
        return out

    def track_async_noalloc(self, clusters: DeviceClusters, out: Tracks, counts, status, stream=None) -> Tracks:
        """track_async on the library's static scratch array (no allocation)."""
        cin, cout = clusters.c_struct(), out.c_struct()
        self._check(self.lib.tpcca_track_async_noalloc(self.h, ctypes.byref(cin), ctypes.byref(cout), _ptr(counts),
                                                       _ptr(status), _stream(stream)))
        return out

    def merge(self, inst_event, stream=None):
        """Cross-sector merge of the last synchronous track call's tracks (the
        context needs FLAG_MERGE). inst_event: int32 device tensor [n_inst].
        Returns (merged Tracks, nseg per merged track, seg_next per sector track)."""
        torch = _torch()
        sz = self.sizes()
        nt, nh = sz["n_tracks"], sz["n_track_hits"]
        out = Tracks(max(nt, 1), max(nh, 1), device=inst_event.device)
        nseg = torch.empty(max(nt, 1), dtype=torch.int32, device=inst_event.device)
        nxt = torch.empty(max(nt, 1), dtype=torch.int32, device=inst_event.device)
        c = out.c_struct()
        self._check(self.lib.tpcca_merge(self.h, _ptr(inst_event), ctypes.byref(c), _ptr(nseg), _ptr(nxt),
                                         _stream(stream)))
        out.n_tracks, out.n_hits = int(c.n_tracks), int(c.n_hits)
        return out, nseg[:out.n_tracks], nxt[:nt]

    def fit_corrected(self, coef=None, want_masks: bool = False, want_yz: bool = False, stream=None) -> dict:
        """Corrected final fit of the last synchronous track call's tracks (their
        output, z0 included, must still be alive): clusters and states moved to
        the absolute frame by each track's z0 and corrected by the map coef
        (float32 device tensor [3*16*16*32] or None). Returns device tensors
        param [n,5], cov [n,15], chi2, ndf (-1: failed), x_ref, z0 and, with
        want_masks / want_yz, the accept masks and the corrected (y, z) per
        output cluster."""
        torch = _torch()
        sz = self.sizes()
        nt, nh = sz["n_tracks"], sz["n_track_hits"]
        dev = "cuda"
        o = {"param": torch.empty(max(nt, 1) * 5, dtype=torch.float32, device=dev),
             "cov": torch.empty(max(nt, 1) * 15, dtype=torch.float32, device=dev),
             "chi2": torch.empty(max(nt, 1), dtype=torch.float32, device=dev),
             "ndf": torch.empty(max(nt, 1), dtype=torch.int32, device=dev),
             "x_ref": torch.empty(max(nt, 1), dtype=torch.float32, device=dev),
             "z0": torch.empty(max(nt, 1), dtype=torch.float32, device=dev)}
        masks = torch.empty(max(nh, 1), dtype=torch.uint8, device=dev) if want_masks else None
        yz = torch.empty(max(nh, 1) * 2, dtype=torch.float32, device=dev) if want_yz else None
        self._check(self.lib.tpcca_fit_corrected(self.h, _ptr(coef), _ptr(o["param"]), _ptr(o["cov"]), _ptr(o["chi2"]),
                                                 _ptr(o["ndf"]), _ptr(o["x_ref"]), _ptr(o["z0"]), _ptr(masks), _ptr(yz),
                                                 _stream(stream)))
        out = {"param": o["param"][:nt * 5].view(nt, 5), "cov": o["cov"][:nt * 15].view(nt, 15),
               "chi2": o["chi2"][:nt], "ndf": o["ndf"][:nt], "x_ref": o["x_ref"][:nt], "z0": o["z0"][:nt]}
        if want_masks:
            out["masks"] = masks[:nh]
        if want_yz:
            out["hit_yz"] = yz[:2 * nh].view(nh, 2)
        return out

    def autotune(self, clusters: DeviceClusters, repeats: int = 3, stream=None) -> Tuning:
        t = Tuning()
        cin = clusters.c_struct()
        self._check(self.lib.tpcca_autotune(self.h, ctypes.byref(cin), repeats, ctypes.byref(t), _stream(stream)))
        return t

    # ---- exports (numpy, cluster-id space) -----------------------------
    def sizes(self):
        s = np.zeros(8, np.int64)
        self._check(self.lib.tpcca_export_sizes(self.h, ctypes.c_void_p(s.ctypes.data), None))
        keys = ("n_clusters", "n_segments", "n_starts", "n_selected", "n_selected_hits", "n_tracks",
                "n_track_hits", "n_rows")
        return dict(zip(keys, (int(v) for v in s)))

    def export_grid(self, stream=None):
        torch = _torch()
        sz = self.sizes()
        N, nseg = sz["n_clusters"], sz["n_segments"]
        sid = torch.empty(max(N, 1), dtype=torch.int32, device="cuda")
        bs = torch.empty(N + nseg + 1, dtype=torch.int32, device="cuda")
        ny = torch.empty(max(nseg, 1), dtype=torch.int32, device="cuda")
        nz = torch.empty(max(nseg, 1), dtype=torch.int32, device="cuda")
        meta = torch.empty(max(nseg, 1) * 4, dtype=torch.float32, device="cuda")
        self._check(self.lib.tpcca_export_grid(self.h, _ptr(sid), _ptr(bs), _ptr(ny), _ptr(nz), _ptr(meta),
                                               _stream(stream)))
        torch.cuda.synchronize()
        return {"sorted_id": sid[:N].cpu().numpy(), "bin_start": bs.cpu().numpy(), "ny": ny[:nseg].cpu().numpy(),
                "nz": nz[:nseg].cpu().numpy(), "meta": meta[:nseg * 4].cpu().numpy().reshape(nseg, 4)}

    def export_links(self, stream=None):
        torch = _torch()
        N = max(self.sizes()["n_clusters"], 1)
        arrs = [torch.empty(N, dtype=torch.int32, device="cuda") for _ in range(4)]
        self._check(self.lib.tpcca_export_links(self.h, *[_ptr(a) for a in arrs], _stream(stream)))
        torch.cuda.synchronize()
        n = self.sizes()["n_clusters"]
        return dict(zip(("up", "dn", "upc", "dnc"), (a[:n].cpu().numpy() for a in arrs)))

    def export_tracklets(self, stream=None):
        torch = _torch()
        sz = self.sizes()
        ns, N, nr = sz["n_starts"], sz["n_clusters"], sz["n_rows"]
        d = "cuda"
        sh, si, stid, nh = (torch.empty(max(ns, 1), dtype=torch.int32, device=d) for _ in range(4))
        rowhit = torch.empty(max(ns, 1) * nr, dtype=torch.int32, device=d)
        state = torch.empty(max(ns, 1) * 20, dtype=torch.float32, device=d)
        srow = torch.empty(max(ns, 1), dtype=torch.int32, device=d)
        w = torch.empty(max(N, 1), dtype=torch.int32, device=d)
        self._check(self.lib.tpcca_export_tracklets(self.h, _ptr(sh), _ptr(si), _ptr(stid), _ptr(nh), _ptr(rowhit),
                                                    _ptr(state), _ptr(srow), _ptr(w), _stream(stream)))
        torch.cuda.synchronize()
        return {"start_hit": sh[:ns].cpu().numpy(), "start_inst": si[:ns].cpu().numpy(),
                "start_tid": stid[:ns].cpu().numpy(), "nhits": nh[:ns].cpu().numpy(),
                "rowhit": rowhit[:ns * nr].cpu().numpy().reshape(ns, nr),
                "state": state[:ns * 20].cpu().numpy().reshape(ns, 20), "state_row": srow[:ns].cpu().numpy(),
                "weight": w[:N].cpu().numpy().view(np.uint32)}

    def export_selected(self, stream=None):
        torch = _torch()
        sz = self.sizes()
        nsel, nh = sz["n_selected"], sz["n_selected_hits"]
        d = "cuda"
        tl = torch.empty(max(nsel, 1), dtype=torch.int32, device=d)
        hs = torch.empty(nsel + 1, dtype=torch.int64, device=d)
        hid = torch.empty(max(nh, 1), dtype=torch.int32, device=d)
        mask = torch.empty(max(nh, 1), dtype=torch.uint8, device=d)
        status = torch.empty(max(nsel, 1), dtype=torch.int32, device=d)
        if nsel == 0:
            hs.zero_()
        self._check(self.lib.tpcca_export_selected(self.h, _ptr(tl), _ptr(hs), _ptr(hid), _ptr(mask), _ptr(status),
                                                   _stream(stream)))
        torch.cuda.synchronize()
        return {"sel_tl": tl[:nsel].cpu().numpy(), "hit_start": hs.cpu().numpy(), "hit_id": hid[:nh].cpu().numpy(),
                "mask": mask[:nh].cpu().numpy(), "status": status[:nsel].cpu().numpy()}

    def stats(self) -> dict:
        s = Stats()
        self._check(self.lib.tpcca_get_stats(self.h, ctypes.byref(s)))
        return s.as_dict()

    def stage_times(self):
        a = np.zeros(8, np.float32)
        self._check(self.lib.tpcca_get_stage_times(self.h, ctypes.c_void_p(a.ctypes.data)))
        return dict(zip(("grid", "links", "clean_starts", "tracklets", "select", "refit", "write", "finish"),
                        a.tolist()))

    # ---- differentiable refit ---------------------------------------------
    def refit_forward(self, clusters: DeviceClusters, rset: "RefitSet", params0=None, coef=None, record=True,
                      stream=None):
        """chi2 per track (float32), track ok flags, FP64 total of the refit with
        frozen masks; params0 (n, 5) float32 overrides rset.params0, coef is
        the (3, 16, 16, 32) float32 correction map or None; record keeps what
        refit_backward needs."""
        torch = _torch()
        n = rset.n_tracks
        dev = clusters.y.device
        p0 = rset.params0 if params0 is None else params0
        for name, t, dt in (("params0", p0, torch.float32), ("coef", coef, torch.float32)):
            if t is not None and (t.dtype != dt or not t.is_contiguous()):
                raise TypeError("%s must be a contiguous float32 tensor" % name)
        if coef is not None and coef.numel() != MAP_SIZE:
            raise ValueError("coef must hold %d coefficients" % MAP_SIZE)
        chi2 = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
        ok = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        total = torch.empty(1, dtype=torch.float64, device=dev)
        cin, cset = clusters.c_struct(), rset.c_struct(p0)
        self._check(self.lib.tpcca_refit_fwd(self.h, ctypes.byref(cin), ctypes.byref(cset), _ptr(coef), _ptr(chi2),
                                             _ptr(ok), _ptr(total), 1 if record else 0, _stream(stream)))
        self._adj_gen = getattr(self, "_adj_gen", 0) + 1
        self._adj_hits = rset.n_hits
        return chi2[:n], ok[:n], total

    def refit_backward(self, grad_chi2, want_map=True, want_hits=False, stream=None):
        """Gradients (FP64) of sum_t grad_chi2[t] * chi2[t] of the last refit_forward:
        d/dparams0 (n, 5), d/dcoef (3, 16, 16, 32) or None, d/d(y', z') per cluster slot or None."""
        torch = _torch()
        n = int(grad_chi2.numel())
        dev = grad_chi2.device
        if grad_chi2.dtype != torch.float32 or not grad_chi2.is_contiguous():
            raise TypeError("grad_chi2 must be a contiguous float32 tensor")
        gp = torch.empty((max(n, 1), 5), dtype=torch.float64, device=dev)
        gm = torch.empty(MAP_SHAPE, dtype=torch.float64, device=dev) if want_map else None
        nh = getattr(self, "_adj_hits", 0)
        gh = torch.empty((max(nh, 1), 2), dtype=torch.float64, device=dev) if want_hits else None
        self._check(self.lib.tpcca_refit_bwd(self.h, _ptr(grad_chi2), _ptr(gp), _ptr(gm), _ptr(gh),
                                             _stream(stream)))
        return gp[:n], gm, (gh[:nh] if gh is not None else None)


@dataclass
class RefitSet:
    """Tracks to refit (device tensors): start state and covariance at row0,
    instance, CSR of cluster ids (rows strictly increasing) and accept masks."""

    params0: "object"  # float32 [n, 5]
    cov0: "object"  # float32 [n, 15]
    row0: "object"  # int32 [n]
    inst: "object"  # int32 [n]
    hit_start: "object"  # int64 [n + 1]
    hit_id: "object"  # int32 [n_hits]
    hit_mask: "object"  # uint8 [n_hits]

    @property
    def n_tracks(self) -> int:
        return int(self.row0.shape[0])

    @property
    def n_hits(self) -> int:
        return int(self.hit_id.shape[0])

    def c_struct(self, params0=None) -> RefitSetC:
        c = RefitSetC()
        c.n_tracks, c.n_hits = self.n_tracks, self.n_hits
        c.params0 = _ptr(self.params0 if params0 is None else params0)
        c.cov0, c.row0, c.inst = _ptr(self.cov0), _ptr(self.row0), _ptr(self.inst)
        c.hit_start, c.hit_id, c.hit_mask = _ptr(self.hit_start), _ptr(self.hit_id), _ptr(self.hit_mask)
        return c

    def head(self, n: int) -> "RefitSet":
        """The first n tracks (views)."""
        n = min(int(n), self.n_tracks)
        nh = int(self.hit_start[n])
        return RefitSet(self.params0[:n], self.cov0[:n], self.row0[:n], self.inst[:n], self.hit_start[:n + 1],
                        self.hit_id[:nh], self.hit_mask[:nh])

    @classmethod
    def from_arrays(cls, st0, row0, inst, hit_start, hit_id, hit_mask, device="cuda"):
        torch = _torch()
        st0 = np.asarray(st0, np.float32).reshape(-1, 20)
        return cls(torch.as_tensor(np.ascontiguousarray(st0[:, :5]), device=device),
                   torch.as_tensor(np.ascontiguousarray(st0[:, 5:]), device=device),
                   torch.as_tensor(np.asarray(row0, np.int32), device=device),
                   torch.as_tensor(np.asarray(inst, np.int32), device=device),
                   torch.as_tensor(np.asarray(hit_start, np.int64), device=device),
                   torch.as_tensor(np.asarray(hit_id, np.int32), device=device),
                   torch.as_tensor(np.asarray(hit_mask, np.uint8), device=device))

    @classmethod
    def from_tracker(cls, tracker: Tracker, device="cuda"):
        """The output tracks of the tracker's last call: tracklet state at its
        row as the start, the owned clusters and the masks the refit took."""
        tl, sel = tracker.export_tracklets(), tracker.export_selected()
        idx = np.nonzero(sel["status"])[0]
        hs = sel["hit_start"]
        lens = hs[idx + 1] - hs[idx]
        pos = np.concatenate([np.arange(hs[i], hs[i + 1]) for i in idx]) if len(idx) else np.zeros(0, np.int64)
        tli = sel["sel_tl"][idx]
        return cls.from_arrays(tl["state"][tli], tl["state_row"][tli], tl["start_inst"][tli],
                               np.concatenate([[0], np.cumsum(lens)]), sel["hit_id"][pos], sel["mask"][pos],
                               device=device)


def refit_chi2(tracker: Tracker, clusters: DeviceClusters, rset: RefitSet, params0, coef=None):
    """chi2 per track of the frozen-mask refit as a differentiable torch function
    of params0 (n, 5) and of the correction map coef (3, 16, 16, 32) or None."""
    torch = _torch()
    # (inside Function.forward gradients are always disabled: decide here)
    record = torch.is_grad_enabled() and (params0.requires_grad or (coef is not None and coef.requires_grad))

    class _RefitChi2(torch.autograd.Function):
        @staticmethod
        def forward(fctx, p, c):
            p32 = p.detach().to(torch.float32).contiguous()
            c32 = None if c is None else c.detach().to(torch.float32).contiguous()
            chi2, ok, _ = tracker.refit_forward(clusters, rset, p32, c32, record=record)
            fctx.p32, fctx.c32, fctx.gen = p32, c32, tracker._adj_gen
            fctx.p_shape, fctx.c_shape = p.shape, None if c is None else c.shape
            fctx.mark_non_differentiable(ok)
            return chi2.clone(), ok

        @staticmethod
        def backward(fctx, g, _gok):
            if tracker._adj_gen != fctx.gen:  # another forward ran since: recompute the checkpoints
                tracker.refit_forward(clusters, rset, fctx.p32, fctx.c32)
                fctx.gen = tracker._adj_gen
            gp, gm, _ = tracker.refit_backward(g.to(torch.float32).contiguous(), want_map=fctx.needs_input_grad[1])
            return gp.reshape(fctx.p_shape), None if gm is None else gm.reshape(fctx.c_shape)

    return _RefitChi2.apply(params0, coef)


def sqrt_step_check(first, last, stream=None):
    """Number of binary32 bit patterns in [first, last] for which the helix
    step's square root differs from sqrtf on the device."""
    torch = _torch()
    lib = load()
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = lib.tpcca_sqrt_step_check(int(first), int(last), _ptr(cnt), _stream(stream))
    if st != OK:
        raise TpccaError(st, "sqrt self-check failed")
    return int(cnt.item())


def fp32_selfcheck(a, b, stream=None):
    """Device a/b and sqrt(|a|) with the library's binary32 operations."""
    torch = _torch()
    lib = load()
    ta = torch.as_tensor(np.asarray(a, np.float32), device="cuda")
    tb = torch.as_tensor(np.asarray(b, np.float32), device="cuda")
    od = torch.empty_like(ta)
    os_ = torch.empty_like(ta)
    st = lib.tpcca_fp32_selfcheck(_ptr(ta), _ptr(tb), _ptr(od), _ptr(os_), ta.numel(), _stream(stream))
    if st != OK:
        raise TpccaError(st, "fp32 self-check failed")
    return od.cpu().numpy(), os_.cpu().numpy()
