"""CPU checks of bench.py's command line: one GPU is measured; asking for
more exits with a message before any device work, and the byte models
charge each stage as documented."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_tracklet_byte_model_is_the_per_unit_figures():
    sys.path.insert(0, ROOT)
    import bench
    st = {"n_chain_hits": 7, "tl_rows_visited": 11, "tl_candidates": 13, "tl_picks": 17}
    assert bench.byte_model("tracklets", st, 1000, 152, 1) == 12 * 7 + 12 * 11 + 8 * 13 + 8 * 17
    from types import SimpleNamespace
    t = SimpleNamespace(inward_wgs=0, inward_sort=1)
    assert bench.stage_kernels("tracklets", t) == ["k_tracklet<1>", "k_tl_order", "k_tracklet_inward"]
    assert bench.stage_kernels("tracklets", SimpleNamespace(inward_wgs=0, inward_sort=0)) == ["k_tracklet<0>"]
    assert bench.stage_kernels("links", t, max_row=321) == ["k_links<8>"]
    assert bench.stage_kernels("links", t, max_row=2284) == ["k_links<8>", "k_links<16>"]
