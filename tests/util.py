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
