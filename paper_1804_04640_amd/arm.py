"""Bottom-up association-rule mining over binary items (Section 4.3).

Items are binary variables; an instance contains item a when X_a = 1.  The
level-wise search runs in the library (``fc_mine``): level 1 from the
database marginals, level 2 from the co-occurrence Gram (FP4 matrix cores), and
every level k >= 3 from candidates joined out of the frequent
(k-1)-itemsets that share their first k-2 items, pruned by
anti-monotonicity and counted as batched single-assignment queries
Count(X_a = 1 AND ...).

An itemset S is frequent when Count(S)/m > minsup (strict, binary64).  Every
frequent S with |S| >= 2 gives the rules S - {X} => X for each X in S, kept
when Count(S)/Count(S - {X}) > minconf.  Itemsets have at most ``max_size``
items (the paper mines rules of size less than seven).
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import _lib as L


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data if a.size else 0


def mine_arrays(db, minsup: float, minconf: float, items: Optional[Sequence[int]] = None,
                max_size: int = 6, stream=None) -> Dict[str, np.ndarray]:
    """The mining result as host arrays: itemset i is
    ``set_items[set_off[i]:set_off[i+1]]`` with count ``set_count[i]`` (level
    by level, lexicographic within a level); rule j is
    ``rule_items[rule_off[j]:rule_off[j+1]] => rule_cons[j]`` with
    ``rule_support[j]`` and ``rule_conf[j]`` (ordered by antecedent, then
    consequent)."""
    from .api import _stream
    it = np.ascontiguousarray(np.arange(db.n) if items is None else np.asarray(items), np.int32)
    h = L.fc_mine(db.handle, _ptr(it), len(it), float(minsup), float(minconf), int(max_size),
                  _stream(stream))
    try:
        ns, nsi, nr, nri = L.fc_arm_sizes(h)
        out = {"set_items": np.zeros(nsi, np.int32), "set_off": np.zeros(ns + 1, np.int64),
               "set_count": np.zeros(ns, np.int64), "rule_items": np.zeros(nri, np.int32),
               "rule_off": np.zeros(nr + 1, np.int64), "rule_cons": np.zeros(nr, np.int32),
               "rule_support": np.zeros(nr, np.float64), "rule_conf": np.zeros(nr, np.float64)}
        L.fc_arm_read(h, *(_ptr(out[k]) for k in ("set_items", "set_off", "set_count",
                                                   "rule_items", "rule_off", "rule_cons",
                                                   "rule_support", "rule_conf")))
    finally:
        L.fc_arm_free(h)
    return out


def mine(db, minsup: float, minconf: float, items: Optional[Sequence[int]] = None,
         max_size: int = 6, stream=None):
    """Returns (itemsets {tuple of variable ids: count}, rules
    [(antecedent tuple, consequent, support, confidence)], sorted)."""
    r = mine_arrays(db, minsup, minconf, items=items, max_size=max_size, stream=stream)
    si, so, sc = r["set_items"].tolist(), r["set_off"].tolist(), r["set_count"].tolist()
    freq: Dict[Tuple[int, ...], int] = {tuple(si[so[i]:so[i + 1]]): sc[i] for i in range(len(sc))}
    ri, ro, rc = r["rule_items"].tolist(), r["rule_off"].tolist(), r["rule_cons"].tolist()
    rs, rf = r["rule_support"].tolist(), r["rule_conf"].tolist()
    rules: List[tuple] = [(tuple(ri[ro[j]:ro[j + 1]]), rc[j], rs[j], rf[j]) for j in range(len(rc))]
    return freq, rules
