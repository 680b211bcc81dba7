"""GPU parity on input shapes the central event does not reach: rows dense
enough for the large-row grid kernel and for the neighbour kernel's
global-memory path, a detector whose row count is not a multiple of four (the
tracklet kernel's scalar pick stores), sixteen instances of the continuous-
readout slice and every instance of the 256-instance workload, stage by
stage."""
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
import synth
from gpu_util import compare_with_oracle, log, run_gpu, tracks_equal
from util import first_rows, with_dense_rows

pytestmark = pytest.mark.gpu

SMALL_ROW = 4096   # rows above this go through the large-row grid kernel
LDS_ROWS = 2730    # neighbour rows above this are read from global memory


def test_dense_rows_bit_exact():
    base = synth.generate("C1")
    # rows around 3000 clusters (links from global memory, small grid kernel),
    # around 5000-9000 (large grid kernel too), beside ordinary rows
    cs = with_dense_rows(base, {40: 3000, 41: 3100, 42: 2900, 80: 5000, 81: 6000, 82: 5200, 120: 9000,
                                121: 4500})
    sizes = np.diff(cs.row_start)
    assert sizes.max() > SMALL_ROW and ((sizes > LDS_ROWS) & (sizes <= SMALL_ROW)).sum() >= 3
    log("dense rows: %d clusters, largest row %d" % (cs.n_clusters, sizes.max()))
    o = oracle.run(cs, 32)
    g = run_gpu(cs)
    compare_with_oracle(g, o)
    log("dense rows, plain form")
    p = run_gpu(cs, batched=False, exports=False)
    assert tracks_equal(g, p)


@pytest.mark.parametrize("n_rows", [151, 150])
def test_row_count_not_multiple_of_four(n_rows):
    from paper_1811_11481_amd import default_params
    base = synth.generate("C1")
    rs, y, z = first_rows(base, n_rows)
    cs = SimpleNamespace(n_inst=base.n_inst, inst_sector=base.inst_sector, row_start=rs, y=y, z=z)
    log("C1 on the first %d pad rows: %d clusters" % (n_rows, len(y)))
    o = oracle.run(cs, 32, params=oracle.default_params(n_rows=n_rows))
    g = run_gpu(cs, params=default_params(n_rows=n_rows))
    compare_with_oracle(g, o)
    assert o.n_tracks > 50


@pytest.mark.timeout(900)
def test_c3_sixteen_instances_bit_exact():
    # the oracle's brute-force searches take ~70 s per instance at this
    # occupancy: sixteen instances (one per host thread), the eight densest and
    # eight spread over the rest, all stages compared
    cs = synth.generate("C3")
    sizes = np.diff(cs.row_start[::152])
    dense = list(np.argsort(-sizes)[:8])
    rest = [i for i in range(cs.n_inst) if i not in dense]
    pick = sorted(int(i) for i in dense + rest[::max(1, len(rest) // 8)][:8])
    sub = cs.subset(pick)
    log("C3: instances %s, %d clusters, oracle on every one" % (pick, sub.n_clusters))
    o = oracle.run(sub, 32, threads=16)
    g = run_gpu(sub)
    compare_with_oracle(g, o)


@pytest.mark.timeout(900)
def test_c4_every_instance_bit_exact():
    cs = synth.generate("C4")
    log("C4: %d clusters in %d instances, oracle on every instance" % (cs.n_clusters, cs.n_inst))
    o = oracle.run(cs, 32, threads=16)
    g = run_gpu(cs)
    compare_with_oracle(g, o)
    log("C4 plain vs batched")
    p = run_gpu(cs, batched=False, exports=False)
    assert tracks_equal(g, p)
