"""Native-coordinate input on the GPU: tpcca_native_to_local against the
oracle's transform (bit for bit), and tpcca_track_native, whose grid kernel
transforms each cluster as it reads it, against the oracle's tracking of the
oracle-transformed clusters (every stage, bit for bit) and against the local
track call on the continuous-readout slice; the cross-sector merge after a
native call; a non-finite native coordinate is an input error."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from gpu_util import compare_with_oracle, log, run_gpu, tracks_equal

pytestmark = pytest.mark.gpu


def _native(cs):
    g = oracle.native_geometry()
    pad, time = synth.to_native(cs, g["pad_width"], g["pad_center"], float(g["z_per_bin"]), float(g["z_readout"]))
    y, z = oracle.native_to_local(152, cs.inst_sector, cs.row_start, pad, time, g)
    return pad, time, dataclasses.replace(cs, y=y, z=z)


def _device(cs, pad, time):
    from paper_1811_11481_amd import DeviceNativeClusters
    return DeviceNativeClusters.from_host(cs.n_inst, cs.inst_sector, cs.row_start, pad, time)


@pytest.mark.parametrize("wl", ["C2", "C3"])
def test_transform_bit_exact(wl):
    from paper_1811_11481_amd import Tracker
    cs = synth.generate(wl)
    log("%s: native transform of %d clusters" % (wl, cs.n_clusters))
    pad, time, local = _native(cs)
    yg, zg = Tracker().native_to_local(_device(cs, pad, time))
    assert np.array_equal(yg.cpu().numpy().view(np.uint32), local.y.view(np.uint32))
    assert np.array_equal(zg.cpu().numpy().view(np.uint32), local.z.view(np.uint32))


def test_track_native_every_stage_bit_exact_c1():
    from paper_1811_11481_amd import Tracker
    cs = synth.generate("C1")
    pad, time, local = _native(cs)
    log("C1 native: %d clusters" % cs.n_clusters)
    o = oracle.run(local, 32)
    trk = Tracker()
    out = trk.track_native(_device(cs, pad, time))
    g = {"tracks": out.to_numpy(), "n_tracks": out.n_tracks, "n_hits": out.n_hits,
         "row_start": np.asarray(cs.row_start), "grid": trk.export_grid(), "links": trk.export_links(),
         "tracklets": trk.export_tracklets(), "selected": trk.export_selected()}
    compare_with_oracle(g, o)
    assert out.n_tracks > 50


def test_track_native_continuous_slice_equals_local_call():
    from paper_1811_11481_amd import Tracker
    cs = synth.generate("C3")
    pad, time, local = _native(cs)
    log("C3 native: %d clusters in %d instances" % (cs.n_clusters, cs.n_inst))
    trk = Tracker()
    out = trk.track_native(_device(cs, pad, time))
    a = {"tracks": out.to_numpy()}
    b = run_gpu(local, exports=False)
    assert out.n_tracks == b["n_tracks"] and out.n_tracks > 1000
    assert tracks_equal(a, b)
    # again on the captured graph, then a local call on the same context: no state leaks between the forms
    out2 = trk.track_native(_device(cs, pad, time))
    assert tracks_equal({"tracks": out2.to_numpy()}, b)
    from paper_1811_11481_amd import DeviceClusters
    assert tracks_equal({"tracks": trk.track(DeviceClusters.from_host(local)).to_numpy()}, b)


def test_merge_after_native_call():
    import torch
    from paper_1811_11481_amd import FLAG_MERGE, DeviceClusters, Tracker, default_params
    cs = synth.generate("C2")
    pad, time, local = _native(cs)
    log("C2 native + merge")
    ev = torch.zeros(cs.n_inst, dtype=torch.int32, device="cuda")
    # the merge reads the track call's inputs and outputs: both stay alive until it has run
    t1 = Tracker(params=default_params(flags=FLAG_MERGE))
    dn = _device(cs, pad, time)
    T1 = t1.track_native(dn)
    m1, n1, x1 = t1.merge(ev)
    t2 = Tracker(params=default_params(flags=FLAG_MERGE))
    dc = DeviceClusters.from_host(local)
    T2 = t2.track(dc)
    m2, n2, x2 = t2.merge(ev)
    assert T1.n_tracks == T2.n_tracks
    assert m1.n_tracks == m2.n_tracks
    a, b = m1.to_numpy(), m2.to_numpy()
    keys = ("inst", "x_ref", "alpha", "param", "cov", "chi2", "ndf", "hit_start", "hit_id")  # what the merge writes
    assert tracks_equal({"tracks": {k: a[k] for k in keys}}, {"tracks": {k: b[k] for k in keys}})
    assert np.array_equal(n1.cpu().numpy(), n2.cpu().numpy()) and np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())


def test_nonfinite_native_time_is_rejected():
    from paper_1811_11481_amd import Tracker, TpccaError
    cs = synth.generate("C1")
    pad, time, _ = _native(cs)
    time = time.copy()
    time[17] = np.nan
    with pytest.raises(TpccaError, match="E_ARG"):
        Tracker().track_native(_device(cs, pad, time))
