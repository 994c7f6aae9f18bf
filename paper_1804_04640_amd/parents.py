"""Exact parent-set assignment over the subset lattice (Section 4.2).

For every variable X_i the lattice of candidate parent sets
Pa in X - {X_i} is traversed level by level (|Pa| = 0, 1, ..., max_pa).  The
library enumerates and scores every set of a level natively
(fc_score_parent_sets: the families are counted by the batched path and
streamed into the fused reducers); the result is, per child, the parent set
with the best score: minimal MDL, or maximal BDeu.

MDL admits an exact bound: -LL >= 0, so MDL(Pa) >= penalty(Pa) =
1/2 log2(m) q(Pa) (r_i - 1), and the penalty only grows as parents are added.
A candidate whose penalty already reaches the child's best score is skipped
without counting (it, and every superset, cannot win).  BDeu is scored
exhaustively.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Tuple

import numpy as np
import torch


def _unrank(i: int, n: int, k: int) -> List[int]:
    """Positions of the i-th k-subset of range(n) in lexicographic order."""
    out, x = [], 0
    for t in range(k, 0, -1):
        while math.comb(n - x - 1, t - 1) <= i:
            i -= math.comb(n - x - 1, t - 1)
            x += 1
        out.append(x)
        x += 1
    return out


def best_parents(db, max_pa: int = 3, score: str = "mdl", ess: float = 1.0,
                 prune: bool = True, children: Optional[List[int]] = None, stream=None):
    """Returns ({child: (parents tuple, score)}, stats).  Scores are the
    library's float32 values; ties go to the lexicographically first set."""
    if score not in ("mdl", "bdeu"):
        raise ValueError("score must be 'mdl' or 'bdeu'")
    n = db.n
    kids = list(range(n)) if children is None else [int(c) for c in children]
    best: Dict[int, Tuple[Tuple[int, ...], float]] = {}
    others = {c: np.array([v for v in range(n) if v != c], np.int32) for c in kids}
    stats = {"scored": 0, "pruned": 0, "levels": []}
    better = (lambda a, b: a < b) if score == "mdl" else (lambda a, b: a > b)
    for level in range(0, min(max_pa, n - 1) + 1):
        # submit every child of the level (the device works while the host
        # enumerates the next child), then pick the bests
        pending = []
        for c in kids:
            bound = best[c][1] if (score == "mdl" and prune and c in best) else 0.0
            sc = db.score_parent_sets(c, others[c], level, (score,), ess=ess,
                                      prune_mdl=max(bound, 0.0), stream=stream)[score]
            pending.append((c, sc))
        scored = 0
        for c, sc in pending:
            i = int(torch.argmin(sc) if score == "mdl" else torch.argmax(sc))
            v = float(sc[i])
            kept = int(torch.isfinite(sc).sum())
            scored += kept
            stats["pruned"] += len(sc) - kept
            if math.isfinite(v) and (c not in best or better(v, best[c][1])):
                cand = others[c]
                best[c] = (tuple(int(cand[p]) for p in _unrank(i, len(cand), level)), v)
        stats["scored"] += scored
        stats["levels"].append({"level": level, "families": scored})
    return best, stats
