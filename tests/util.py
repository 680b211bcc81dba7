"""Small helpers shared by the tests (input construction and structural checks)."""
from __future__ import annotations

import numpy as np

from synth import N_ROWS, ClusterSet, row_plane_x


def make_clusterset(hits, n_inst=1, sectors=None, labels=None) -> ClusterSet:
    """hits: iterable of (inst, row, y, z); kept in the given order within a row."""
    hits = list(hits)
    order = sorted(range(len(hits)), key=lambda i: (hits[i][0], hits[i][1]))
    inst = np.array([hits[i][0] for i in order], dtype=np.int64)
    row = np.array([hits[i][1] for i in order], dtype=np.int32)
    y = np.array([hits[i][2] for i in order], dtype=np.float32)
    z = np.array([hits[i][3] for i in order], dtype=np.float32)
    lab = np.full(len(hits), -1, np.int32) if labels is None else np.asarray(labels, np.int32)[order]
    seg = inst * N_ROWS + row
    counts = np.bincount(seg, minlength=n_inst * N_ROWS) if len(hits) else np.zeros(n_inst * N_ROWS, np.int64)
    rs = np.zeros(n_inst * N_ROWS + 1, np.int64)
    rs[1:] = np.cumsum(counts)
    sec = np.zeros(n_inst, np.int32) if sectors is None else np.asarray(sectors, np.int32)
    return ClusterSet(n_inst, sec, rs, row_plane_x(row).astype(np.float32), y, z, row, lab,
                      np.zeros((0, 8)), name="handmade")


def row_of_ids(cs: ClusterSet) -> np.ndarray:
    seg = np.repeat(np.arange(cs.n_inst * N_ROWS, dtype=np.int64), np.diff(cs.row_start))
    return (seg % N_ROWS).astype(np.int32)


def chains_from_links(upc: np.ndarray, dnc: np.ndarray):
    """All maximal chains (lists of ids, following up-links) of the cleaned links."""
    heads = np.nonzero((dnc < 0) & (upc >= 0))[0]
    out = []
    for h in heads:
        c = [int(h)]
        while upc[c[-1]] >= 0:
            c.append(int(upc[c[-1]]))
        out.append(c)
    return out


def with_dense_rows(cs: ClusterSet, counts: dict, inst: int = 0, seed: int = 99) -> ClusterSet:
    """`cs` with extra uniform noise clusters on some rows of one instance:
    counts = {row: number of added clusters}; y spans the row's sector width,
    z the instance's cluster range. Added clusters follow the row's own."""
    rng = np.random.default_rng(seed)
    zlo, zhi = float(cs.z.min()), float(cs.z.max())
    ys, zs, rows_out, ins, labs = [], [], [], [], []
    nseg = cs.n_inst * N_ROWS
    for seg in range(nseg):
        a, b = cs.row_start[seg], cs.row_start[seg + 1]
        ys.append(cs.y[a:b])
        zs.append(cs.z[a:b])
        labs.append(cs.label[a:b])
        r = seg % N_ROWS
        n_add = counts.get(r, 0) if seg // N_ROWS == inst else 0
        if n_add:
            half = float(row_plane_x(np.array([r]))[0]) * np.tan(np.radians(10.0))
            ys.append(rng.uniform(-half, half, n_add).astype(np.float32))
            zs.append(rng.uniform(zlo, zhi, n_add).astype(np.float32))
            labs.append(np.full(n_add, -1, np.int32))
        rows_out.append(b - a + n_add)
    rs = np.zeros(nseg + 1, np.int64)
    rs[1:] = np.cumsum(rows_out)
    row = np.repeat(np.tile(np.arange(N_ROWS, dtype=np.int32), cs.n_inst), rows_out)
    return ClusterSet(cs.n_inst, cs.inst_sector.copy(), rs, row_plane_x(row).astype(np.float32),
                      np.concatenate(ys), np.concatenate(zs), row, np.concatenate(labs), cs.truth,
                      name=cs.name + "+dense")


def first_rows(cs: ClusterSet, n_rows: int):
    """Instance-major CSR of the first n_rows pad rows of every instance (a
    detector with fewer rows): (row_start [n_inst * n_rows + 1], y, z)."""
    keep, rs = [], [0]
    for i in range(cs.n_inst):
        for r in range(n_rows):
            a, b = cs.row_start[i * N_ROWS + r], cs.row_start[i * N_ROWS + r + 1]
            keep.append(np.arange(a, b))
            rs.append(rs[-1] + (b - a))
    idx = np.concatenate(keep)
    return np.asarray(rs, np.int64), cs.y[idx].copy(), cs.z[idx].copy()
