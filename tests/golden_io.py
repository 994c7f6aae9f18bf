"""Readers for the text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def fig1_database():
    """Returns (D [n][m] uint8 with 0-based states, arity uint8[n])."""
    rows, arity = [], None
    with open(os.path.join(GOLDEN, "fig1_reconstructed.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("arity"):
                arity = np.array([int(x) for x in line.split()[1:]], dtype=np.uint8)
            else:
                rows.append([int(x) for x in line.split()])
    D = (np.array(rows, dtype=np.int64).T - 1).astype(np.uint8)   # 1-based -> 0-based
    return np.ascontiguousarray(D), arity


def fig1_expected():
    out = {}
    with open(os.path.join(GOLDEN, "fig1_expected.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            if key == "table":
                out[key] = np.array([int(v) for v in vals], dtype=np.int64)
            else:
                out[key] = float(vals[0])
    return out


# ---------------------------------------------------------------- full-size
# Per-query digests of contingency tables, so that every table of a
# full-size workload can be compared with the oracle's without storing the
# tables.  A table T of C cells has the digest  sum_c T[c] * h(c)  (mod 2^64)
# with h(c) an odd 64-bit mix of the cell index c: two tables that differ in
# a single cell always differ in digest (h(c) is odd and the difference is
# below 2^63 in magnitude); several differing cells collide only through a
# linear relation between unrelated 64-bit mixes.

_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_GOLD = np.uint64(0x9E3779B97F4A7C15)


def _cell_mix(c: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser of (c + 1) * golden ratio, forced odd."""
    with np.errstate(over="ignore"):
        z = (c.astype(np.uint64) + np.uint64(1)) * _GOLD
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z | np.uint64(1)


def table_digest(T: np.ndarray) -> np.uint64:
    """Digest of one dense table (any integer dtype, non-negative counts)."""
    T = np.asarray(T)
    with np.errstate(over="ignore"):
        return np.uint64(np.sum(T.astype(np.uint64) * _cell_mix(np.arange(T.size)),
                                dtype=np.uint64))


def table_digests(T: np.ndarray, off: np.ndarray, chunk_cells: int = 1 << 26) -> np.ndarray:
    """Digests of the tables packed in T, table i being T[off[i]:off[i+1]]
    (every table has at least one cell).  Works through the tables in
    pieces of about `chunk_cells` cells."""
    off = np.asarray(off, dtype=np.int64)
    nq = len(off) - 1
    out = np.zeros(nq, dtype=np.uint64)
    i = 0
    while i < nq:
        j = int(np.searchsorted(off, off[i] + chunk_cells, side="right")) - 1
        j = min(max(j, i + 1), nq)
        lo, hi = int(off[i]), int(off[j])
        seg = np.asarray(T[lo:hi]).astype(np.uint64)
        starts = off[i:j] - lo
        local = np.arange(hi - lo, dtype=np.int64) - np.repeat(starts, np.diff(off[i:j + 1]))
        with np.errstate(over="ignore"):
            prod = seg * _cell_mix(local)
        out[i:j] = np.add.reduceat(prod, starts)
        i = j
    return out


def array_sha(*arrays) -> str:
    import hashlib
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(memoryview(a).cast("B"))
    return h.hexdigest()


def fullsize_path(name: str) -> str:
    return os.path.join(GOLDEN, "fullsize_%s.npz" % name)


def load_fullsize(name: str):
    """The stored oracle results of a full-size workload (written by
    tests/golden/make_fullsize.py), as a dict of arrays."""
    with np.load(fullsize_path(name), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}
