"""Seeded synthetic TPC inputs (helices in a uniform 0.5 T field).

Input generator only: no track-finding arithmetic lives here. Both the CPU
oracle tests and the GPU path consume these arrays.

Named workloads (seed = 1000 * config + event):

* ``C1``  one A-side sector (sector 0), 200 helices from the origin with
  0 < eta < 0.9 and phi0 uniform inside the sector, 1 % noise (~10 k clusters).
* ``C2``  a full central event: 36 sectors, 8000 primaries with |eta| < 0.9
  over the full azimuth plus 10 % secondaries with vertex radius U(0, 50) cm,
  2 % noise (~1.3 M clusters).
* ``C3``  continuous-readout slice: 100 collisions with Exp(800) tracks each,
  pT truncated to [0.05, 10] GeV, drift shift U(0, 250) cm per collision,
  2 % noise (~9.9 M clusters).
* ``C4``  256 sector instances of uneven occupancy: instance j is sector
  j mod 36 with round(exp(U(ln 50, ln 2000))) helices, 1 % noise (~6.6 M clusters).
* ``C2x8`` eight central events (seeds 2000..2007 law, one generator call) in
  288 instances (~10.9 M clusters).
* ``C5``  twelve central events whose clusters are displaced by a smooth
  synthetic space-charge map (amplitude 0.5 cm) before the smear: the input
  of the differentiable refit.

Common law: pT exponential with mean 0.5 GeV truncated (resampled) to
[0.1, 10] GeV, random charge, Gaussian smear sigma_y = sigma_z = 0.1 cm, one
cluster per pad-row plane crossing, x exactly on the row plane.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libtpcsynth.so")
N_ROWS = 152


class _Config(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32),
        ("n_units", ctypes.c_int32),
        ("unit_sector", ctypes.c_void_p),
        ("unit_ntracks", ctypes.c_void_p),
        ("bz", ctypes.c_double),
        ("pt_mean", ctypes.c_double),
        ("pt_min", ctypes.c_double),
        ("pt_max", ctypes.c_double),
        ("eta_max", ctypes.c_double),
        ("sec_frac", ctypes.c_double),
        ("sec_rmax", ctypes.c_double),
        ("noise_frac", ctypes.c_double),
        ("sigma_y", ctypes.c_double),
        ("sigma_z", ctypes.c_double),
        ("zshift_max", ctypes.c_double),
        ("shuffle", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("n_explicit", ctypes.c_int32),
        ("ex_vx", ctypes.c_void_p),
        ("ex_vy", ctypes.c_void_p),
        ("ex_vz", ctypes.c_void_p),
        ("ex_pt", ctypes.c_void_p),
        ("ex_tanl", ctypes.c_void_p),
        ("ex_phi0", ctypes.c_void_p),
        ("ex_q", ctypes.c_void_p),
        ("distort", ctypes.c_int32),
    ]


_lib = None


def build(force: bool = False) -> str:
    """Compile the generator library with g++ (host code only)."""
    import subprocess

    src = os.path.join(_HERE, "helix_gen.cpp")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", src, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.syn_generate.restype = ctypes.c_void_p
        lib.syn_generate.argtypes = [ctypes.POINTER(_Config)]
        lib.syn_sizes.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int64)] * 3
        lib.syn_copy.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 8
        lib.syn_free.argtypes = [ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclass
class ClusterSet:
    """Clusters sorted by (instance, row) in CSR form, plus Monte-Carlo truth."""

    n_inst: int
    inst_sector: np.ndarray  # int32 [n_inst]
    row_start: np.ndarray  # int64 [n_inst * 152 + 1]
    x: np.ndarray  # float32 [N] (row-plane position)
    y: np.ndarray  # float32 [N] (local y)
    z: np.ndarray  # float32 [N]
    row: np.ndarray  # int32 [N]
    label: np.ndarray  # int32 [N] (track index, -1 = noise)
    truth: np.ndarray  # float64 [n_tracks, 8]: vx vy vz pt tanl phi0 q dz
    bz: float = 0.5
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_clusters(self) -> int:
        return int(self.y.shape[0])

    def instance_of(self) -> np.ndarray:
        """Instance index of every cluster (int32 [N])."""
        seg = np.repeat(np.arange(self.n_inst * N_ROWS, dtype=np.int64), np.diff(self.row_start))
        return (seg // N_ROWS).astype(np.int32)

    def subset(self, instances) -> "ClusterSet":
        """The clusters of the given instances, re-packed (instance order kept)."""
        instances = np.asarray(instances, dtype=np.int64)
        parts, rs = [], [0]
        for j in instances:
            a, b = self.row_start[j * N_ROWS], self.row_start[(j + 1) * N_ROWS]
            parts.append((a, b))
            rs.extend((self.row_start[j * N_ROWS + 1:(j + 1) * N_ROWS + 1] - a + rs[-1]).tolist())
        idx = np.concatenate([np.arange(a, b) for a, b in parts]) if parts else np.zeros(0, np.int64)
        return ClusterSet(
            n_inst=len(instances), inst_sector=self.inst_sector[instances].copy(),
            row_start=np.asarray(rs, dtype=np.int64), x=self.x[idx], y=self.y[idx], z=self.z[idx],
            row=self.row[idx], label=self.label[idx], truth=self.truth, bz=self.bz,
            name=self.name + "[sub]", meta=dict(self.meta, parent_index=idx))


def generate_raw(mode, n_units, unit_ntracks, unit_sector=None, *, bz=0.5, pt_mean=0.5, pt_min=0.1,
                 pt_max=10.0, eta_max=0.9, sec_frac=0.0, sec_rmax=50.0, noise_frac=0.0,
                 sigma=0.1, zshift_max=0.0, shuffle=True, seed=0, explicit=None, distort=False,
                 name="") -> ClusterSet:
    lib = _load()
    cfg = _Config()
    cfg.mode, cfg.n_units = mode, n_units
    nt = np.ascontiguousarray(np.asarray(unit_ntracks, dtype=np.int32))
    sec = np.ascontiguousarray(np.asarray(unit_sector if unit_sector is not None else np.zeros(max(n_units, 1)),
                                          dtype=np.int32))
    cfg.unit_ntracks = nt.ctypes.data
    cfg.unit_sector = sec.ctypes.data
    cfg.bz, cfg.pt_mean, cfg.pt_min, cfg.pt_max = bz, pt_mean, pt_min, pt_max
    cfg.eta_max, cfg.sec_frac, cfg.sec_rmax = eta_max, sec_frac, sec_rmax
    cfg.noise_frac, cfg.sigma_y, cfg.sigma_z = noise_frac, sigma, sigma
    cfg.zshift_max, cfg.shuffle, cfg.seed = zshift_max, int(shuffle), seed
    cfg.distort = int(bool(distort))
    keep = [nt, sec]
    if explicit is not None:
        cols = [np.ascontiguousarray(np.asarray(explicit[k], dtype=np.float64))
                for k in ("vx", "vy", "vz", "pt", "tanl", "phi0")]
        q = np.ascontiguousarray(np.asarray(explicit["q"], dtype=np.int32))
        keep += cols + [q]
        cfg.n_explicit = len(q)
        cfg.ex_vx, cfg.ex_vy, cfg.ex_vz, cfg.ex_pt, cfg.ex_tanl, cfg.ex_phi0 = [c.ctypes.data for c in cols]
        cfg.ex_q = q.ctypes.data
    h = lib.syn_generate(ctypes.byref(cfg))
    if not h:
        raise ValueError("generator rejected the configuration")
    try:
        ni, nc, ntr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        lib.syn_sizes(h, ctypes.byref(ni), ctypes.byref(nc), ctypes.byref(ntr))
        ni, nc, ntr = ni.value, nc.value, ntr.value
        inst_sector = np.zeros(ni, np.int32)
        row_start = np.zeros(ni * N_ROWS + 1, np.int64)
        x, y, z = (np.zeros(nc, np.float32) for _ in range(3))
        row, label = np.zeros(nc, np.int32), np.zeros(nc, np.int32)
        truth = np.zeros((ntr, 8), np.float64)
        lib.syn_copy(h, inst_sector.ctypes.data, row_start.ctypes.data, x.ctypes.data, y.ctypes.data,
                     z.ctypes.data, row.ctypes.data, label.ctypes.data, truth.ctypes.data)
    finally:
        lib.syn_free(h)
    del keep
    return ClusterSet(ni, inst_sector, row_start, x, y, z, row, label, truth, bz=bz, name=name)


def generate(config: str, event: int = 0) -> ClusterSet:
    """One of the named workloads, seeded with 1000 * config + event."""
    cfgno = {"C1": 1, "C2": 2, "C3": 3, "C4": 4, "C2x8": 2, "C5": 5}[config]
    seed = 1000 * cfgno + event
    if config == "C1":
        return generate_raw(0, 1, [200], [0], noise_frac=0.01, seed=seed, name="C1")
    if config == "C2":
        return generate_raw(1, 1, [8000], sec_frac=0.1, noise_frac=0.02, seed=seed, name="C2")
    if config == "C2x8":
        return generate_raw(1, 8, [8000] * 8, sec_frac=0.1, noise_frac=0.02, seed=seed, name="C2x8")
    if config == "C5":
        # twelve central events with the synthetic space-charge displacement
        return generate_raw(1, 12, [8000] * 12, sec_frac=0.1, noise_frac=0.02, seed=seed, distort=True, name="C5")
    if config == "C3":
        rng = np.random.default_rng(seed)
        mult = np.rint(rng.exponential(800.0, size=100)).astype(np.int32)
        return generate_raw(2, 100, mult, pt_min=0.05, noise_frac=0.02, zshift_max=250.0, seed=seed,
                            name="C3")
    if config == "C4":
        rng = np.random.default_rng(seed)
        nt = np.rint(np.exp(rng.uniform(math.log(50.0), math.log(2000.0), size=256))).astype(np.int32)
        sec = np.arange(256, dtype=np.int32) % 36
        return generate_raw(0, 256, nt, sec, noise_frac=0.01, seed=seed, name="C4")
    raise KeyError(config)


def row_plane_x(i):
    """Pad-row plane position X_i = 85 + i * 162 / 151 cm (FP64)."""
    return 85.0 + np.asarray(i, dtype=np.float64) * 162.0 / 151.0


def to_native(cs: ClusterSet, pad_width, pad_center, z_per_bin, z_readout):
    """Native (pad, time) float32 readout coordinates of the clusters of `cs`
    for a pad geometry (pitch and centre pad per row) and drift constants: the
    readout model inverted in FP64 (pad = y / pitch + centre, time = (readout
    |z| - side * z) / drift per bin, side +1 on sectors 0..17, -1 on 18..35),
    then rounded to binary32. Input generation only."""
    pw = np.asarray(pad_width, np.float64)[cs.row]
    pc = np.asarray(pad_center, np.float64)[cs.row]
    side = np.where(cs.inst_sector[cs.instance_of()] < 18, 1.0, -1.0)
    pad = cs.y.astype(np.float64) / pw + pc
    time = (float(z_readout) - side * cs.z.astype(np.float64)) / float(z_per_bin)
    return pad.astype(np.float32), time.astype(np.float32)
