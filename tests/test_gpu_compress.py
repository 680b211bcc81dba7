"""Track-model compression residuals (Section 5.1) written by the GPU refit,
against the oracle's codec on the same tracks: identical int16 residuals, and
the oracle's decoder restores every cluster within half a step."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import log
from util import row_of_ids

pytestmark = pytest.mark.gpu

PLANES = np.array([np.float32(85.0 + i * 162.0 / 151.0) for i in range(152)])


@pytest.mark.parametrize("wl,step", [("C1", -7), ("C2", -7), ("C2", -10)])
def test_residuals_equal_the_oracle_codec(wl, step):
    from paper_1811_11481_amd import DeviceClusters, Tracker
    cs = synth.generate(wl)
    log("%s compression residuals, step 2^%d cm" % (wl, step))
    trk = Tracker()
    dc = DeviceClusters.from_host(cs)
    out = trk.alloc_tracks(dc).want_residuals(step)
    T = trk.track(dc, out, batched=True).to_numpy()
    rows = row_of_ids(cs)
    res = T["residuals"]
    hs = T["hit_start"]
    esc = 0
    for t in range(len(T["inst"])):
        a, b = hs[t], hs[t + 1]
        ids = T["hit_id"][a:b]
        row0 = int(np.nonzero(PLANES == T["x_ref"][t])[0][0])
        q, n_esc = oracle.track_residuals(T["param"][t].astype(np.float64), rows[ids], cs.y[ids], cs.z[ids],
                                          step_log2=step, row0=row0)
        assert np.array_equal(q, res[a:b]), t
        esc += n_esc
        if t % 7 == 0:
            yd, zd = oracle.track_decode(T["param"][t].astype(np.float64), rows[ids], q, step_log2=step, row0=row0)
            ok = q[:, 0] != oracle.RES_ESCAPE
            assert np.all(np.abs(yd[ok] - cs.y[ids][ok]) <= 2.0 ** step / 2 + 1e-5)
    # escapes: clusters beyond a step where the unrefitted model reaches the
    # |sin phi| guard (tracks that approach it near their outer end)
    assert esc <= 1e-3 * 2 * len(res), esc
    v, n = np.unique(res[:, 0], return_counts=True)
    p = n / n.sum()
    log("residual entropy (y): %.2f bits per cluster at step 2^%d cm" % (-(p * np.log2(p)).sum(), step))
    # the plain form writes the same residuals
    outp = trk.alloc_tracks(dc).want_residuals(step)
    P = trk.track(dc, outp, batched=False).to_numpy()
    assert np.array_equal(P["residuals"], res)
