"""Bottom-up association-rule mining over binary items (Section 4.3).

Items are binary variables; an instance contains item a when X_a = 1.  The
search is level-wise (bottom-up, every subset of a frequent itemset is
frequent):

* level 1: item supports from the database marginals;
* level 2: all pair supports at once from the co-occurrence Gram (int8 MFMA,
  ``fc_pairs``);
* level k >= 3: candidates joined from frequent (k-1)-itemsets sharing their
  first k-2 items, kept only if every (k-1)-subset is frequent, counted in
  batches of single-assignment queries Count(X_a = 1 AND ...) with
  ``fc_count_assignments`` (|S| bitmap intersections and a popcount each).

An itemset S is frequent when Count(S)/m > minsup (strict, decided in
binary64).  Every frequent S with |S| >= 2 gives the rules S - {X} => X for
each X in S, kept when Count(S)/Count(S - {X}) > minconf.  Itemsets have at
most ``max_size`` items (the paper mines rules of size less than seven).
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


def _frequent(count: int, m: int, minsup: float) -> bool:
    return m > 0 and count / m > minsup


def _candidates(prev: Sequence[Tuple[int, ...]]) -> List[Tuple[int, ...]]:
    """Apriori join of sorted (k-1)-itemsets sharing their first k-2 items,
    pruned to those whose every (k-1)-subset is frequent."""
    prev = sorted(prev)
    have = set(prev)
    out = []
    i = 0
    while i < len(prev):
        j = i
        while j < len(prev) and prev[j][:-1] == prev[i][:-1]:
            j += 1
        block = prev[i:j]
        for a in range(len(block)):
            for b in range(a + 1, len(block)):
                cand = block[a] + (block[b][-1],)
                if all(cand[:x] + cand[x + 1:] in have for x in range(len(cand) - 2)):
                    out.append(cand)
        i = j
    return out


def mine(db, minsup: float, minconf: float, items: Optional[Sequence[int]] = None,
         max_size: int = 6, batch: int = 1 << 16):
    """Returns (itemsets {tuple of variable ids: count}, rules
    [(antecedent tuple, consequent, support, confidence)])."""
    m = db.m
    items = list(range(db.n)) if items is None else [int(i) for i in items]
    for i in items:
        if int(db.arity[i]) != 2:
            raise ValueError("item %d is not binary" % i)
    counts, _ = db.marginals()
    soff = np.concatenate([[0], np.cumsum(db.arity.astype(np.int64))])
    freq: Dict[Tuple[int, ...], int] = {}
    level1 = []
    for i in items:
        c = int(counts[soff[i] + 1])
        if _frequent(c, m, minsup):
            freq[(i,)] = c
            level1.append(i)
    level = [(i,) for i in sorted(level1)]
    if max_size >= 2 and len(level1) >= 2:
        l1 = sorted(level1)
        recs, _, total = db.pairs(minsup, items=l1)
        assert total == len(recs)
        level = []
        for r in recs:
            a, b = l1[int(r["a"])], l1[int(r["b"])]
            key = (min(a, b), max(a, b))
            freq[key] = int(r["n_ab"])
            level.append(key)
    k = 3
    while k <= max_size and level:
        cands = _candidates(level)
        level = []
        for lo in range(0, len(cands), batch):
            part = cands[lo:lo + batch]
            flat = np.array([v for c in part for v in c], np.int32)
            off = np.arange(0, (len(part) + 1) * k, k, dtype=np.int64)
            got = db.count_assignments((flat, off), np.ones(len(flat), np.uint8))
            for c, n in zip(part, got):
                if _frequent(int(n), m, minsup):
                    freq[c] = int(n)
                    level.append(c)
        k += 1
    rules = []
    for s, n in freq.items():
        if len(s) < 2:
            continue
        for x in range(len(s)):
            ante = s[:x] + s[x + 1:]
            conf = n / freq[ante]
            if conf > minconf:
                rules.append((ante, s[x], n / m, conf))
    rules.sort()
    return freq, rules
