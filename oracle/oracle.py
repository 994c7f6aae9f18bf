"""CPU oracle for exact counting queries -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The library's product path never
imports, links or calls anything under ``oracle/``; the two share no code.

Two independent routes are provided:

* ``count`` / ``ll`` / ``mdl`` / ``bdeu`` / ``mi`` / ``gram`` call the plain C
  implementation in ``fc_oracle.c`` (binary64, one pass over the instances).
* ``brute_count`` is a numpy per-cell scan for tiny inputs: for every cell it
  compares every instance with the cell's assignment (Section 2 definition of
  ``Count``), O(cells * m).  It is a pin for the C oracle, not a fast path.

Conventions: states are 0-based (the paper's state ``s+1``), a query is an
ordered list of distinct variables with the child last, and the dense table
is mixed-radix with the first variable most significant (Section 3.3 MSD
digit order, child least significant).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile fc_oracle.c with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _bind(lib):
    """Declares the C signatures on a loaded oracle library."""
    P = ctypes.c_void_p
    i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.orc_table_cells.argtypes = [P, i32, P, i32]
    lib.orc_table_cells.restype = i64
    lib.orc_count.argtypes = [P, i64, i32, P, P, i32, P, i64]
    lib.orc_count.restype = ctypes.c_int
    lib.orc_count_assignment.argtypes = [P, i64, i32, P, P, P, i32]
    lib.orc_count_assignment.restype = i64
    for name in ("orc_ll", "orc_mdl", "orc_mi"):
        f = getattr(lib, name)
        f.argtypes = [P, i64, i32]
        f.restype = f64
    lib.orc_bdeu.argtypes = [P, i64, i32, f64]
    lib.orc_bdeu.restype = f64
    lib.orc_count_sparse.argtypes = [P, i64, i32, P, P, i32, P, P]
    lib.orc_count_sparse.restype = i64
    lib.orc_gram.argtypes = [P, i64, i32, P]
    lib.orc_gram.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _cols(D):
    D = np.ascontiguousarray(D, dtype=np.uint8)
    if D.ndim != 2:
        raise ValueError("D must be [n][m] uint8 (column-major database)")
    return D


def table_cells(arity, vars_) -> int:
    arity = np.ascontiguousarray(arity, dtype=np.uint8)
    v = np.ascontiguousarray(vars_, dtype=np.int32)
    return int(_load().orc_table_cells(_ptr(arity), len(arity), _ptr(v), len(v)))


def count(D, arity, vars_) -> np.ndarray:
    """Dense int64 contingency table of ``vars_`` over column-major D [n][m]."""
    D = _cols(D)
    arity = np.ascontiguousarray(arity, dtype=np.uint8)
    v = np.ascontiguousarray(vars_, dtype=np.int32)
    n, m = D.shape
    cells = table_cells(arity, v)
    if cells < 0:
        raise ValueError("invalid query %r" % (list(v),))
    out = np.empty(cells, dtype=np.int64)
    rc = _load().orc_count(_ptr(D), m, n, _ptr(arity), _ptr(v), len(v), _ptr(out), cells)
    if rc != 0:
        raise ValueError("oracle count failed (invalid query or state >= arity)")
    return out


def count_assignment(D, arity, vars_, states) -> int:
    D = _cols(D)
    arity = np.ascontiguousarray(arity, dtype=np.uint8)
    v = np.ascontiguousarray(vars_, dtype=np.int32)
    s = np.ascontiguousarray(states, dtype=np.uint8)
    n, m = D.shape
    r = _load().orc_count_assignment(_ptr(D), m, n, _ptr(arity), _ptr(v), _ptr(s), len(v))
    if r < 0:
        raise ValueError("invalid assignment query")
    return int(r)


def count_sparse(D, arity, vars_):
    """(keys int64, counts int64) of the configurations that occur, sorted by
    mixed-radix key (first variable most significant)."""
    D = _cols(D)
    arity = np.ascontiguousarray(arity, dtype=np.uint8)
    v = np.ascontiguousarray(vars_, dtype=np.int32)
    n, m = D.shape
    keys = np.empty(max(m, 1), np.int64)
    cnt = np.empty(max(m, 1), np.int64)
    nd = _load().orc_count_sparse(_ptr(D), m, n, _ptr(arity), _ptr(v), len(v), _ptr(keys),
                                  _ptr(cnt))
    if nd < 0:
        raise ValueError("invalid sparse query")
    return keys[:nd].copy(), cnt[:nd].copy()


def _qr(table, r_child):
    T = np.ascontiguousarray(table, dtype=np.int64)
    r = int(r_child)
    if T.size % r:
        raise ValueError("table size is not a multiple of the child arity")
    return T, T.size // r, r


def ll(table, r_child) -> float:
    """Eq. (1) log-likelihood in bits (Fig. 2 uses log2)."""
    T, q, r = _qr(table, r_child)
    return float(_load().orc_ll(_ptr(T), q, r))


def mdl(table, r_child) -> float:
    T, q, r = _qr(table, r_child)
    return float(_load().orc_mdl(_ptr(T), q, r))


def bdeu(table, r_child, ess: float = 1.0) -> float:
    T, q, r = _qr(table, r_child)
    return float(_load().orc_bdeu(_ptr(T), q, r, float(ess)))


def mi(table, r_child) -> float:
    T, q, r = _qr(table, r_child)
    return float(_load().orc_mi(_ptr(T), q, r))


REDUCERS = {"ll": ll, "mdl": mdl, "bdeu": bdeu, "mi": mi}


def score(name: str, table, r_child, ess: float = 1.0) -> float:
    if name == "bdeu":
        return bdeu(table, r_child, ess)
    return REDUCERS[name](table, r_child)


def gram(D) -> np.ndarray:
    """n x n int64 co-occurrence counts of binary columns D [n][m]."""
    D = _cols(D)
    n, m = D.shape
    out = np.empty((n, n), dtype=np.int64)
    if _load().orc_gram(_ptr(D), m, n, _ptr(out)) != 0:
        raise ValueError("oracle gram failed (non-binary column?)")
    return out


def pairs(G: np.ndarray, m: int, minsup: float):
    """Association-rule pair records from a co-occurrence matrix (Section 4.3).

    Every pair a < b with support N_ab / m strictly above ``minsup`` gives
    (a, b, N_ab, support, conf(a->b) = N_ab / N_a, conf(b->a) = N_ab / N_b),
    in binary64, ordered by (a, b).
    """
    n = G.shape[0]
    recs = []
    for a in range(n):
        for b in range(a + 1, n):
            nab = int(G[a, b])
            if nab / m > minsup:
                recs.append((a, b, nab, nab / m, nab / int(G[a, a]), nab / int(G[b, b])))
    return recs


def brute_count(D, arity, vars_) -> np.ndarray:
    """Per-cell scan: for each cell, count the instances equal to its assignment.

    Independent of the one-pass C oracle; O(cells * m), tiny inputs only.
    """
    D = np.asarray(D, dtype=np.uint8)
    radices = [int(arity[v]) for v in vars_]
    cells = int(np.prod(radices))
    out = np.zeros(cells, dtype=np.int64)
    for idx in range(cells):
        # decode the mixed-radix cell index, first variable most significant
        rem, states = idx, []
        for r in reversed(radices):
            states.append(rem % r)
            rem //= r
        states.reverse()
        mask = np.ones(D.shape[1], dtype=bool)
        for v, s in zip(vars_, states):
            mask &= D[v] == s
        out[idx] = int(mask.sum())
    return out


def arm_bruteforce(D, minsup: float, minconf: float, max_size: int = 6):
    """Association rules over binary columns D [n][m] by exhaustive
    enumeration (Section 4.3): every itemset S of at most `max_size` items
    whose support Count(S)/m exceeds minsup (each support counted directly,
    no pruning), and every rule S - {X} => X with confidence
    Count(S)/Count(S - {X}) above minconf.  Small n only.
    Returns (itemsets {tuple: count}, sorted rules
    [(antecedent, consequent, support, confidence)])."""
    import itertools
    A = np.asarray(D).astype(bool)
    n, m = A.shape
    freq = {}
    for k in range(1, max_size + 1):
        for S in itertools.combinations(range(n), k):
            c = int(np.logical_and.reduce(A[list(S)], axis=0).sum())
            if m > 0 and c / m > minsup:
                freq[S] = c
    rules = []
    for S, c in freq.items():
        if len(S) < 2:
            continue
        for x in range(len(S)):
            ante = S[:x] + S[x + 1:]
            conf = c / freq[ante]
            if conf > minconf:
                rules.append((ante, S[x], c / m, conf))
    rules.sort()
    return freq, rules
