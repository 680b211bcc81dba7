"""CPU checks of the C-ABI library: it loads, exports every function that
include/tpcca.h declares, and the binding's struct layouts and defaults agree
with the header (no compute calls: there is no GPU here)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tpcca.h")
LIB = os.path.join(ROOT, "paper_1811_11481_amd", "libtpcca.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libtpcca.so not built (run __graft_entry__.build())")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tpcca_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (tpcca_[a-z0-9_]+)", out))
    assert set(names) <= exported
    from paper_1811_11481_amd.tpcca import EXPORTED
    assert sorted(EXPORTED) == names


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "tpcca.h"\nint main(){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %d %zu %zu %zu\\n",'
                   'sizeof(tpcca_params),sizeof(tpcca_tuning),sizeof(tpcca_clusters),sizeof(tpcca_tracks),'
                   'sizeof(tpcca_stats),offsetof(tpcca_params,bz),offsetof(tpcca_tracks,n_tracks),'
                   'sizeof(tpcca_refit_set),offsetof(tpcca_refit_set,hit_mask),TPCCA_MAP_SIZE,'
                   'sizeof(tpcca_native_clusters),offsetof(tpcca_params,z_readout),offsetof(tpcca_tuning,inward_wgs));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    from paper_1811_11481_amd import tpcca as T
    want = [ctypes.sizeof(T.Params), ctypes.sizeof(T.Tuning), ctypes.sizeof(T.Clusters), ctypes.sizeof(T.TracksC),
            ctypes.sizeof(T.Stats), T.Params.bz.offset, T.TracksC.n_tracks.offset, ctypes.sizeof(T.RefitSetC),
            T.RefitSetC.hit_mask.offset, T.MAP_SIZE, ctypes.sizeof(T.NativeClustersC), T.Params.z_readout.offset,
            T.Tuning.inward_wgs.offset]
    assert got == want


def test_default_params_match_the_oracle_readings():
    from paper_1811_11481_amd import default_params
    p = default_params()
    o = oracle.default_params()
    for k in ("n_rows", "bz", "sigma_y", "sigma_z", "win_ty", "win_tz", "win_ny", "win_nz", "nbr_score_max", "nsig",
              "chi2_pick", "chi2_rej", "sinphi_max", "cov_reset", "q_max", "u_max", "n_min", "max_miss"):
        assert getattr(p, k) == getattr(o, k), k
    assert list(p.c0) == list(o.c0)
    x = np.array(p.row_x[:152], dtype=np.float32)
    assert np.array_equal(x, (85.0 + np.arange(152) * 162.0 / 151.0).astype(np.float32))
    # native-coordinate geometry: the library's defaults are the oracle's readings
    g = oracle.native_geometry()
    assert np.array_equal(np.array(p.pad_width[:152], np.float32), g["pad_width"])
    assert np.array_equal(np.array(p.pad_center[:152], np.float32), g["pad_center"])
    assert np.float32(p.z_per_bin) == g["z_per_bin"] and np.float32(p.z_readout) == g["z_readout"]


def test_compute_entry_points_fail_loudly_without_a_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_1811_11481_amd import Tracker, TpccaError
    with pytest.raises(TpccaError):
        Tracker()
