"""Monte-Carlo quality figures of a track set (definitions of the paper's
Section 4 footnote): efficiency, clone rate, fake rate, findable.

Sector tracking has no cross-sector merge here, so the unit of truth is a
track *segment*: the clusters of one Monte-Carlo track inside one sector
instance. A segment is findable with at least ``findable`` clusters (70 in the
paper). A reconstructed track is matched to the label holding the majority of
its clusters; it is fake when more than 10 % of its clusters carry another
label (or noise). A segment is found if at least one non-fake track matches
it; every further matching non-fake track is a clone.
"""
from __future__ import annotations

import numpy as np


def evaluate(cs, hit_start, hit, findable: int = 70, fake_frac: float = 0.10) -> dict:
    inst_of = cs.instance_of()
    lab = cs.label
    n_t = len(hit_start) - 1
    seg_key = inst_of.astype(np.int64) * (1 << 32) + (lab.astype(np.int64) & 0xFFFFFFFF)
    sig = lab >= 0
    keys, counts = np.unique(seg_key[sig], return_counts=True)
    seg_count = dict(zip(keys.tolist(), counts.tolist()))
    matched = {}
    n_fake = 0
    n_clone = 0
    for t in range(n_t):
        hs = hit[hit_start[t]:hit_start[t + 1]]
        if len(hs) == 0:
            continue
        ls = lab[hs]
        vals, cnt = np.unique(ls, return_counts=True)
        j = np.argmax(cnt)
        best, nb = int(vals[j]), int(cnt[j])
        if best < 0 or (len(hs) - nb) > fake_frac * len(hs):
            n_fake += 1
            continue
        key = int(inst_of[hs[0]]) * (1 << 32) + (best & 0xFFFFFFFF)
        if key in matched:
            n_clone += 1
        matched[key] = matched.get(key, 0) + 1
    findable_keys = [k for k, c in seg_count.items() if c >= findable]
    found = sum(1 for k in findable_keys if k in matched)
    all10 = [k for k, c in seg_count.items() if c >= 10]
    found10 = sum(1 for k in all10 if k in matched)
    return {
        "n_tracks": n_t,
        "n_findable": len(findable_keys),
        "efficiency": found / max(1, len(findable_keys)),
        "efficiency_ge10": found10 / max(1, len(all10)),
        "clone_rate": n_clone / max(1, n_t),
        "fake_rate": n_fake / max(1, n_t),
    }
