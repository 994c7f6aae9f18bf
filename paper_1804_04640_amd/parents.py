"""Exact parent-set assignment over the subset lattice (Section 4.2).

For every variable X_i the lattice of candidate parent sets
Pa in X - {X_i} is traversed level by level (|Pa| = 0, 1, ..., max_pa); the
family queries of a level are batched across all children and scored by the
fused reducers of fc_count_reduce.  The result is, per child, the parent set
with the best score: minimal MDL, or maximal BDeu.

MDL admits an exact bound: -LL >= 0, so MDL(Pa) >= penalty(Pa) =
1/2 log2(m) q(Pa) (r_i - 1), and the penalty only grows as parents are added.
A candidate whose penalty already reaches the child's best score is skipped
without counting (it, and every superset, cannot win).  BDeu is scored
exhaustively.
"""
from __future__ import annotations

import itertools
import math
from typing import Dict, List, Optional, Tuple

import numpy as np


def _combos(n: int, k: int) -> np.ndarray:
    """All k-subsets of range(n) as a [C(n,k), k] int32 array (lexicographic)."""
    if k == 0:
        return np.zeros((1, 0), np.int32)
    cnt = math.comb(n, k)
    flat = np.fromiter(itertools.chain.from_iterable(itertools.combinations(range(n), k)),
                       dtype=np.int32, count=cnt * k)
    return flat.reshape(cnt, k)


def best_parents(db, max_pa: int = 3, score: str = "mdl", ess: float = 1.0,
                 batch: int = 1 << 18, prune: bool = True, children: Optional[List[int]] = None):
    """Returns ({child: (parents tuple, score)}, stats).  Scores are the
    library's float32 values."""
    if score not in ("mdl", "bdeu"):
        raise ValueError("score must be 'mdl' or 'bdeu'")
    n, m = db.n, db.m
    ar = db.arity.astype(np.int64)
    lg = 0.5 * math.log2(m) if m > 0 else 0.0
    kids = list(range(n)) if children is None else [int(c) for c in children]
    best: Dict[int, Tuple[Tuple[int, ...], float]] = {}
    others = {c: np.array([v for v in range(n) if v != c], np.int32) for c in kids}
    stats = {"scored": 0, "pruned": 0, "levels": []}
    better = (lambda a, b: a < b) if score == "mdl" else (lambda a, b: a > b)
    for level in range(0, min(max_pa, n - 1) + 1):
        combos = _combos(n - 1, level)
        # (child, parent-index rows) of this level, pruned by the MDL bound
        fams: List[Tuple[int, np.ndarray]] = []
        for c in kids:
            pa = others[c][combos] if level else np.zeros((1, 0), np.int32)
            if score == "mdl" and prune and c in best:
                q = np.prod(ar[pa], axis=1) if level else np.ones(1, np.int64)
                pen = lg * q.astype(np.float64) * float(ar[c] - 1)
                keep = pen < best[c][1]
                stats["pruned"] += int((~keep).sum())
                pa = pa[keep]
            if len(pa):
                fams.append((c, pa))
        # submit the whole level asynchronously (host planning of a batch
        # overlaps the device work of the previous ones), then pick the bests
        scored = 0
        pending = []
        for c, pa in fams:
            for lo in range(0, len(pa), batch):
                part = pa[lo:lo + batch]
                nq = len(part)
                q = np.empty((nq, level + 1), np.int32)
                q[:, :level] = part
                q[:, level] = c
                off = np.arange(0, (nq + 1) * (level + 1), level + 1, dtype=np.int64)
                sc, _, _, _ = db.count_reduce((q.reshape(-1), off), (score,), ess=ess,
                                              with_err=False)
                pending.append((c, part, sc[score]))
                scored += nq
        for c, part, dev in pending:
            s = dev.cpu().numpy()
            i = int(np.argmin(s) if score == "mdl" else np.argmax(s))
            if c not in best or better(float(s[i]), best[c][1]):
                best[c] = (tuple(int(v) for v in part[i]), float(s[i]))
        stats["scored"] += scored
        stats["levels"].append({"level": level, "families": scored})
    return best, stats
