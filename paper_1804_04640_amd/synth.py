"""Seeded synthetic workloads shaped like the paper's benchmarks.

This module only draws random inputs (databases and query streams); it holds
none of the counting or scoring arithmetic, so both the GPU path's tests and
the CPU oracle can consume the same inputs without sharing code.

The paper's own data sets (Table 1; the association-rule data of Section 4.3)
are not available; these generators stand in for them with the shapes the
paper reports (n = 20..104 variables, arities 2 up to high values, m = 1K to
10M instances, Section 4.1).  Every generator is seeded with numpy PCG64,
seed = 180404640 + the workload's stream number (see rng_for).

Databases are column-major uint8 arrays ``D[n][m]`` with 0-based states.
Query streams are flat: ``vars_flat`` (int32) with ``var_off`` (int64, nq+1)
offsets; within a query the child (when there is one) is the last variable.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED_BASE = 180404640


@dataclasses.dataclass
class Workload:
    name: str
    D: np.ndarray                 # uint8 [n][m]
    arity: np.ndarray             # uint8 [n]
    vars_flat: np.ndarray         # int32
    var_off: np.ndarray           # int64 [nq+1]
    reducers: tuple = ()          # reducers the workload streams into
    ess: float = 1.0
    minsup: Optional[float] = None
    batches: Optional[List[np.ndarray]] = None   # serving: query ids per batch
    desc: str = ""

    @property
    def n(self) -> int:
        return int(self.D.shape[0])

    @property
    def m(self) -> int:
        return int(self.D.shape[1])

    @property
    def nq(self) -> int:
        return int(len(self.var_off) - 1)

    def query(self, i: int) -> np.ndarray:
        return self.vars_flat[self.var_off[i]:self.var_off[i + 1]]

    def queries(self) -> List[np.ndarray]:
        return [self.query(i) for i in range(self.nq)]


def rng_for(stream: int) -> np.random.Generator:
    """Generator of seed SEED_BASE + stream (plain-small 1, bn-family 2,
    batched-uneven 3, all-pairs 4, serving 5; other numbers for tests)."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + stream))


def flatten(queries) -> tuple:
    off = np.zeros(len(queries) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(q) for q in queries])
    flat = (np.concatenate([np.asarray(q, dtype=np.int32) for q in queries])
            if queries else np.zeros(0, dtype=np.int32))
    return flat.astype(np.int32), off


# ---------------------------------------------------------------- databases
def iid_uniform(rng, arity, m) -> np.ndarray:
    n = len(arity)
    D = np.empty((n, m), dtype=np.uint8)
    for v in range(n):
        D[v] = rng.integers(0, int(arity[v]), size=m, dtype=np.uint8)
    return D


def random_dag(rng, n, max_indeg):
    """Random DAG: a random topological order; the node at position t takes
    d ~ U{0..min(max_indeg, t)} parents drawn without replacement from the
    nodes before it."""
    order = rng.permutation(n)
    parents = [[] for _ in range(n)]
    for t in range(n):
        d = int(rng.integers(0, min(max_indeg, t) + 1))
        if d:
            parents[order[t]] = [int(x) for x in rng.choice(order[:t], size=d, replace=False)]
    return order, parents


def forward_sample(rng, arity, order, parents, m, alpha, chunk=1 << 20) -> np.ndarray:
    """Ancestral sampling with Dirichlet(alpha) CPT rows and an inverse CDF on
    U(0,1) (clamped to the last state)."""
    n = len(arity)
    D = np.empty((n, m), dtype=np.uint8)
    for v in order:
        v = int(v)
        r = int(arity[v])
        pa = parents[v]
        q = int(np.prod([int(arity[p]) for p in pa])) if pa else 1
        cdf = np.cumsum(rng.dirichlet(np.full(r, alpha), size=q), axis=1)
        for lo in range(0, m, chunk):
            hi = min(m, lo + chunk)
            idx = np.zeros(hi - lo, dtype=np.int64)
            for p in pa:
                idx = idx * int(arity[p]) + D[p, lo:hi]
            u = rng.random(hi - lo)
            if r <= 8:
                s = np.zeros(hi - lo, dtype=np.uint8)
                rows = cdf[idx]
                for k in range(r - 1):
                    s += (u >= rows[:, k]).astype(np.uint8)
            else:
                # the same count #{k < r-1 : cdf[k] <= u}, per parent
                # configuration: a CDF row is nondecreasing, so the count is
                # a right-sided binary search
                s = np.empty(hi - lo, dtype=np.uint8)
                order_ = np.argsort(idx, kind="stable")
                keys, starts = np.unique(idx[order_], return_index=True)
                ends = np.append(starts[1:], len(order_))
                for key, a, b in zip(keys, starts, ends):
                    sel = order_[a:b]
                    s[sel] = np.searchsorted(cdf[key, :r - 1], u[sel], side="right")
            D[v, lo:hi] = s
    return D


def random_queries(rng, n, nq, kmin, kmax) -> tuple:
    """nq queries of k ~ U{kmin..kmax} distinct variables (sampled without
    replacement); the last one plays the child."""
    qs = []
    for _ in range(nq):
        k = int(rng.integers(kmin, kmax + 1))
        qs.append(rng.choice(n, size=k, replace=False).astype(np.int32))
    return flatten(qs)


def family_queries(rng, n, nq, pmin, pmax) -> tuple:
    """Family queries: child ~ U, |Pa| ~ U{pmin..pmax}, parents without
    replacement from the other variables (Section 4.1 generator, |Pa| capped)."""
    qs = []
    for _ in range(nq):
        child = int(rng.integers(0, n))
        npa = int(rng.integers(pmin, pmax + 1))
        others = np.delete(np.arange(n), child)
        pa = rng.choice(others, size=npa, replace=False)
        qs.append(np.concatenate([pa, [child]]).astype(np.int32))
    return flatten(qs)


def _bernoulli_positions(rng, p, m) -> np.ndarray:
    """Positions of successes of m Bernoulli(p) trials via geometric gaps."""
    if p <= 0.0:
        return np.zeros(0, dtype=np.int64)
    if p >= 1.0:
        return np.arange(m, dtype=np.int64)
    est = int(p * m * 1.1 + 10 * math.sqrt(p * m + 1) + 16)
    pos = np.cumsum(rng.geometric(p, size=est)) - 1
    while pos[-1] < m:
        more = np.cumsum(rng.geometric(p, size=est)) + pos[-1]
        pos = np.concatenate([pos, more])
    return pos[pos < m]


# ---------------------------------------------------------------- workloads
def plain_small(m=10_000, nq=1000) -> Workload:
    """n=8, arities U{2,3,4}, iid uniform states, queries of 1-4 variables."""
    rng = rng_for(1)
    arity = rng.integers(2, 5, size=8).astype(np.uint8)
    D = iid_uniform(rng, arity, m)
    flat, off = random_queries(rng, 8, nq, 1, 4)
    return Workload("plain-small", D, arity, flat, off, (),
                    desc="n=8 r~U{2,3,4} m=%d iid uniform; %d queries k~U{1..4}" % (m, nq))


def bn_family(m=1_000_000, nq=50_000) -> Workload:
    """n=37, arities U{2,3,4}, random DAG (in-degree <= 4, Dirichlet(1)),
    family queries child + 0..4 parents, MDL."""
    rng = rng_for(2)
    n = 37
    arity = rng.integers(2, 5, size=n).astype(np.uint8)
    order, parents = random_dag(rng, n, 4)
    D = forward_sample(rng, arity, order, parents, m, 1.0)
    flat, off = family_queries(rng, n, nq, 0, 4)
    return Workload("bn-family", D, arity, flat, off, ("mdl",),
                    desc="n=37 r~U{2,3,4} m=%d DAG(indeg<=4, Dir(1)); %d families |Pa|~U{0..4}"
                    % (m, nq))


def batched_uneven(m=4_000_000, nq=200_000) -> Workload:
    """n=100, arities min(8, 2+Geom(0.4)), random DAG (in-degree <= 3,
    Dirichlet(0.5)), queries of 1..6 variables, BDeu(ess=1) + MI."""
    rng = rng_for(3)
    n = 100
    g = rng.geometric(0.4, size=n) - 1            # failures before success
    arity = np.minimum(8, 2 + g).astype(np.uint8)
    order, parents = random_dag(rng, n, 3)
    D = forward_sample(rng, arity, order, parents, m, 0.5)
    flat, off = random_queries(rng, n, nq, 1, 6)
    return Workload("batched-uneven", D, arity, flat, off, ("bdeu", "mi"), ess=1.0,
                    desc="n=100 r=min(8,2+Geom(0.4)) m=%d DAG(indeg<=3, Dir(0.5)); %d queries k~U{1..6}"
                    % (m, nq))


def zipf_marginals(n, s=1.1, mean=0.01):
    """f_i = min(1, c * i^-s) with c solved by bisection so the mean is `mean`."""
    i = np.arange(1, n + 1, dtype=np.float64)
    lo, hi = 0.0, 1000.0
    for _ in range(200):
        c = 0.5 * (lo + hi)
        if np.minimum(1.0, c * i ** -s).mean() < mean:
            lo = c
        else:
            hi = c
    return np.minimum(1.0, 0.5 * (lo + hi) * i ** -s)


def all_pairs(m=1 << 21, n=1024, groups=64) -> Workload:
    """Binary transactions: Zipf(1.1) item frequencies at 1% mean density,
    items independent except `groups` planted disjoint groups of 3..5 items.
    Reading of "co-occur with p=0.6": a group fires in an instance with
    probability equal to its members' mean frequency; when it fires each
    member is present with probability 0.6, OR-ed with its own draw."""
    rng = rng_for(4)
    f = zipf_marginals(n)
    perm = rng.permutation(n)                      # shuffle item ids
    freq = np.empty(n)
    freq[perm] = f
    D = np.zeros((n, m), dtype=np.uint8)
    for a in range(n):
        D[a, _bernoulli_positions(rng, float(freq[a]), m)] = 1
    members = rng.permutation(n)
    pos = 0
    for _ in range(groups):
        size = int(rng.integers(3, 6))
        grp = members[pos:pos + size]
        pos += size
        fire = _bernoulli_positions(rng, float(freq[grp].mean()), m)
        for a in grp:
            keep = fire[rng.random(len(fire)) < 0.6]
            D[a, keep] = 1
    arity = np.full(n, 2, dtype=np.uint8)
    flat = np.zeros(0, dtype=np.int32)
    off = np.zeros(1, dtype=np.int64)
    return Workload("all-pairs", D, arity, flat, off, ("suppconf",), minsup=0.001,
                    desc="n=%d binary items, m=%d, Zipf(1.1) at 1%% density, %d planted groups"
                    % (n, m, groups))


def hill_climb_batches(rng, n, nbatches, smin=10, smax=5000, max_pa=6):
    """Family batches of a simulated hill-climbing structure search: each batch
    proposes add / remove / reverse moves on the current parent sets and asks
    for the affected families (child + 1..max_pa parents); after the batch one
    proposed move is applied.  Batch sizes are log-uniform on [smin, smax].
    The search starts from a random DAG with in-degree <= max_pa - 1, so the
    families span 2..max_pa+1 variables from the first batch on."""
    _, start = random_dag(rng, n, max_pa - 1)
    par = [set(p) for p in start]
    batches = []
    for _ in range(nbatches):
        size = int(round(math.exp(rng.uniform(math.log(smin), math.log(smax)))))
        fams, moves = [], []
        while len(fams) < size:
            u, v = (int(x) for x in rng.choice(n, size=2, replace=False))
            kind = int(rng.integers(0, 3))
            if kind == 0 and u not in par[v] and len(par[v]) < max_pa:
                fams.append(sorted(par[v] | {u}) + [v])
                moves.append((0, u, v))
            elif kind == 1 and u in par[v] and len(par[v]) > 1:
                fams.append(sorted(par[v] - {u}) + [v])
                moves.append((1, u, v))
            elif kind == 2 and u in par[v] and len(par[u]) < max_pa and v not in par[u]:
                fams.append(sorted(par[u] | {v}) + [u])
                moves.append((2, u, v))
            elif not par[v]:
                # an empty parent set: propose the first edge into v
                fams.append([u, v])
                moves.append((0, u, v))
        batches.append(fams[:size])
        kind, u, v = moves[int(rng.integers(0, len(moves)))]
        if kind == 0:
            par[v].add(u)
        elif kind == 1:
            par[v].discard(u)
        else:
            par[v].discard(u)
            par[u].add(v)
    return batches


def serving(m=1 << 22, nbatches=64) -> Workload:
    """Serving: n=64, arities U{2..5}, random DAG (in-degree <= 4, Dirichlet(1))
    resident on the device; hill-climbing family batches of 10..5000 queries
    of 2..7 variables; MDL."""
    rng = rng_for(5)
    n = 64
    arity = rng.integers(2, 6, size=n).astype(np.uint8)
    order, parents = random_dag(rng, n, 4)
    D = forward_sample(rng, arity, order, parents, m, 1.0)
    fam_batches = hill_climb_batches(rng, n, nbatches)
    qs, ids, base = [], [], 0
    for b in fam_batches:
        qs.extend(b)
        ids.append(np.arange(base, base + len(b), dtype=np.int64))
        base += len(b)
    flat, off = flatten(qs)
    return Workload("serving", D, arity, flat, off, ("mdl",), batches=ids,
                    desc="n=64 r~U{2..5} m=%d DAG(indeg<=4, Dir(1)); %d hill-climbing batches"
                    % (m, nbatches))


def high_arity(m=1_000_000, nq=64) -> Workload:
    """Key spaces far beyond the data (the sparse-table path): n=30 with
    Mildew-like arities (half in 2..8, half in 9..99), a random DAG
    (in-degree <= 2, Dirichlet(0.5)); queries of 5..8 variables whose tables
    have more than 2^24 cells."""
    rng = rng_for(6)
    n = 30
    arity = np.where(rng.random(n) < 0.5, rng.integers(2, 9, size=n),
                     rng.integers(9, 100, size=n)).astype(np.uint8)
    order, parents = random_dag(rng, n, 2)
    D = forward_sample(rng, arity, order, parents, m, 0.5)
    qs = []
    while len(qs) < nq:
        k = int(rng.integers(5, 9))
        q = rng.choice(n, size=k, replace=False).astype(np.int32)
        if float(np.prod(arity[q].astype(np.float64))) > float(1 << 24):
            qs.append(q)
    flat, off = flatten(qs)
    return Workload("high-arity", D, arity, flat, off, (),
                    desc="n=30 arities half U{2..8} half U{9..99}, m=%d DAG(indeg<=2, Dir(0.5)); "
                         "%d queries k~U{5..8} with more than 2^24 cells" % (m, nq))


WORKLOADS = {"plain-small": plain_small, "bn-family": bn_family,
             "batched-uneven": batched_uneven, "all-pairs": all_pairs, "serving": serving}
