"""Pins for the CPU oracle (runs without a GPU).

Each check ties the oracle to something other than itself: the paper's worked
example (Section 2, Section 3.2), hand-derived closed forms, a brute-force
per-cell scan, table invariants, library routines (numpy bincount / matmul,
scipy entropies) and the sequential Polya-urn form of the Dirichlet marginal
likelihood.
"""
import math

import numpy as np
import pytest
from scipy.stats import entropy

from oracle import oracle as orc
from tests.golden_io import fig1_database, fig1_expected


def rand_db(seed, n=None, m=None, rmax=4):
    rng = np.random.default_rng(seed)
    n = n or int(rng.integers(1, 6))
    m = m if m is not None else int(rng.integers(0, 65))
    arity = rng.integers(1, rmax + 1, size=n).astype(np.uint8)
    D = np.stack([rng.integers(0, int(a), size=m) for a in arity]).astype(np.uint8) \
        if m else np.zeros((n, 0), np.uint8)
    return rng, D, arity


# ------------------------------------------------------------ worked example
def test_fig1_count_example():
    D, ar = fig1_database()
    # Count((X1=3) AND (X2=2) AND (X3=1)) = 2  (Section 2), 0-based states
    assert orc.count_assignment(D, ar, [0, 1, 2], [2, 1, 0]) == 2


def test_fig1_query_table_and_seven_configurations():
    D, ar = fig1_database()
    exp = fig1_expected()
    T = orc.count(D, ar, [0, 2, 1])              # Query(X2, {X1, X3})
    np.testing.assert_array_equal(T, exp["table"])
    assert int((T > 0).sum()) == 7               # Section 3.2: 7 configurations
    assert int(T.sum()) == D.shape[1]


def test_fig1_entropy_order_and_dfs_states():
    D, ar = fig1_database()
    H = [entropy(np.bincount(D[v], minlength=ar[v]), base=2) for v in range(3)]
    assert H[2] < H[0]                           # X3 has lower entropy than X1

    def considered(first, second):
        # nodes considered at the second parent level: the first variable's
        # states that occur, each expanded over all states of the second one
        nz = int((np.bincount(D[first], minlength=ar[first]) > 0).sum())
        return nz * int(ar[second])

    assert considered(2, 0) == 6 and considered(0, 2) == 9


def test_fig1_reducer_closed_forms():
    D, ar = fig1_database()
    exp = fig1_expected()
    T = orc.count(D, ar, [0, 2, 1])
    r = int(ar[1])
    assert orc.ll(T, r) == pytest.approx(exp["ll"], rel=1e-13)
    assert orc.mdl(T, r) == pytest.approx(exp["mdl"], rel=1e-13)
    assert orc.bdeu(T, r, 1.0) == pytest.approx(exp["bdeu"], rel=1e-13)
    assert orc.mi(T, r) == pytest.approx(exp["mi"], rel=1e-13)


# ------------------------------------------------------------ counting
@pytest.mark.parametrize("seed", range(40))
def test_count_matches_brute_force(seed):
    rng, D, ar = rand_db(seed)
    n = D.shape[0]
    for _ in range(4):
        k = int(rng.integers(1, n + 1))
        vs = [int(v) for v in rng.choice(n, size=k, replace=False)]
        np.testing.assert_array_equal(orc.count(D, ar, vs), orc.brute_count(D, ar, vs))


@pytest.mark.parametrize("seed", range(20))
def test_count_invariants(seed):
    rng, D, ar = rand_db(seed, n=5, m=int(np.random.default_rng(seed).integers(1, 300)))
    m = D.shape[1]
    vs = [int(v) for v in rng.permutation(5)[: int(rng.integers(2, 6))]]
    T = orc.count(D, ar, vs)
    shape = [int(ar[v]) for v in vs]
    Tn = T.reshape(shape)
    assert int(T.sum()) == m                                     # sums to m
    assert int((T > 0).sum()) <= min(T.size, m)                  # #leaves <= min(q r, m)
    for ax in range(len(vs)):                                    # marginalisation
        sub = [v for i, v in enumerate(vs) if i != ax]
        np.testing.assert_array_equal(Tn.sum(axis=ax).ravel(), orc.count(D, ar, sub))
    perm = list(rng.permutation(len(vs)))                        # axis permutation
    Tp = orc.count(D, ar, [vs[i] for i in perm]).reshape([shape[i] for i in perm])
    np.testing.assert_array_equal(Tp, np.transpose(Tn, perm))
    rows = Tn.reshape(-1, shape[-1])                             # N_ijk <= N_ij
    assert np.all(rows <= rows.sum(axis=1, keepdims=True))


@pytest.mark.parametrize("seed", range(10))
def test_single_variable_is_bincount(seed):
    _, D, ar = rand_db(seed, n=3, m=500, rmax=9)
    for v in range(3):
        np.testing.assert_array_equal(orc.count(D, ar, [v]), np.bincount(D[v], minlength=ar[v]))


@pytest.mark.parametrize("seed", range(10))
def test_count_assignment_is_table_cell(seed):
    rng, D, ar = rand_db(seed, n=4, m=200)
    vs = [0, 2, 3]
    T = orc.count(D, ar, vs).reshape([int(ar[v]) for v in vs])
    for _ in range(5):
        st = [int(rng.integers(0, int(ar[v]))) for v in vs]
        assert orc.count_assignment(D, ar, vs, st) == int(T[tuple(st)])


def test_empty_database_and_errors():
    D = np.zeros((3, 0), np.uint8)
    ar = np.array([2, 3, 4], np.uint8)
    T = orc.count(D, ar, [2, 0])
    assert T.shape == (8,) and int(T.sum()) == 0
    D2 = np.array([[0, 1], [2, 0]], np.uint8)
    with pytest.raises(ValueError):
        orc.count(D2, np.array([2, 2], np.uint8), [0, 1])        # state 2 >= arity 2
    with pytest.raises(ValueError):
        orc.count(D2, np.array([2, 3], np.uint8), [0, 0])        # duplicate variable
    with pytest.raises(ValueError):
        orc.count(D2, np.array([2, 3], np.uint8), [2])           # out of range
    with pytest.raises(ValueError):
        orc.count(D2, np.array([2, 3], np.uint8), [])            # empty query


# ------------------------------------------------------------ reducers
def family(seed, m=400, k=3, rmax=5):
    rng = np.random.default_rng(1000 + seed)
    ar = rng.integers(2, rmax + 1, size=k).astype(np.uint8)
    # a dependent child so that all terms matter
    D = np.stack([rng.integers(0, int(a), size=m) for a in ar]).astype(np.uint8)
    noise = rng.random(m) < 0.3
    D[-1] = np.where(noise, D[-1], (D[:-1].sum(axis=0) % ar[-1])).astype(np.uint8)
    return D, ar, list(range(k))


@pytest.mark.parametrize("seed", range(12))
def test_ll_is_conditional_entropy(seed):
    D, ar, vs = family(seed)
    m = D.shape[1]
    T = orc.count(D, ar, vs)
    r = int(ar[vs[-1]])
    Hj = entropy(T, base=2)                                       # H(Pa, X)
    Hp = entropy(T.reshape(-1, r).sum(axis=1), base=2)            # H(Pa)
    assert orc.ll(T, r) == pytest.approx(-m * (Hj - Hp), rel=1e-11, abs=1e-9)


@pytest.mark.parametrize("seed", range(6))
def test_mdl_deterministic_child(seed):
    rng = np.random.default_rng(seed)
    ar = np.array([3, 4, 5], np.uint8)
    m = 1000
    D = np.stack([rng.integers(0, 3, m), rng.integers(0, 4, m), np.zeros(m)]).astype(np.uint8)
    D[2] = (D[0] * 2 + D[1]) % 5                                  # child = f(parents)
    T = orc.count(D, ar, [0, 1, 2])
    assert orc.ll(T, 5) == 0.0
    assert orc.mdl(T, 5) == pytest.approx(0.5 * math.log2(m) * 12 * 4, rel=1e-14)


def polya_bdeu(D, ar, vs, ess):
    """Log marginal likelihood as the product of sequential predictive
    probabilities of a Dirichlet-multinomial urn, one instance at a time."""
    q = int(np.prod([int(ar[v]) for v in vs[:-1]])) if len(vs) > 1 else 1
    r = int(ar[vs[-1]])
    aj, ajk = ess / q, ess / (q * r)
    cj, cjk, terms = {}, {}, []
    for p in range(D.shape[1]):
        j = 0
        for v in vs[:-1]:
            j = j * int(ar[v]) + int(D[v, p])
        k = int(D[vs[-1], p])
        terms.append(math.log((ajk + cjk.get((j, k), 0)) / (aj + cj.get(j, 0))))
        cjk[(j, k)] = cjk.get((j, k), 0) + 1
        cj[j] = cj.get(j, 0) + 1
    return math.fsum(terms)


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("ess", [1.0, 0.37, 10.0])
def test_bdeu_is_polya_urn_likelihood(seed, ess):
    D, ar, vs = family(seed, m=300, k=1 + seed % 4)
    T = orc.count(D, ar, vs)
    assert orc.bdeu(T, int(ar[vs[-1]]), ess) == pytest.approx(polya_bdeu(D, ar, vs, ess), rel=1e-10)


@pytest.mark.parametrize("seed", range(12))
def test_mi_is_entropy_identity(seed):
    D, ar, vs = family(seed)
    T = orc.count(D, ar, vs)
    r = int(ar[vs[-1]])
    Tq = T.reshape(-1, r)
    expect = entropy(Tq.sum(axis=0)) + entropy(Tq.sum(axis=1)) - entropy(T)
    assert orc.mi(T, r) == pytest.approx(expect, rel=1e-10, abs=1e-12)


def test_mi_special_cases():
    rng = np.random.default_rng(5)
    x = rng.integers(0, 4, 2000).astype(np.uint8)
    D = np.stack([x, x.copy()])
    ar = np.array([4, 4], np.uint8)
    T = orc.count(D, ar, [0, 1])                                   # MI(X; X) = H(X)
    assert orc.mi(T, 4) == pytest.approx(entropy(np.bincount(x, minlength=4)), rel=1e-12)
    # exact product table: every row proportional to the child marginal
    Tp = np.outer([1, 2, 3], [2, 4, 6, 8]).ravel().astype(np.int64)
    assert abs(orc.mi(Tp, 4)) < 1e-15
    # a single variable has no parents: MI = 0, N_ij = m
    assert orc.mi(np.array([5, 7, 9], np.int64), 3) == 0.0


def decimal_mi(T, r, digits=50):
    """MI of table T (child arity r) straight from its definition,
    sum over non-zero cells of (N/m) ln(m N / (N_j N_k)), in 50-digit
    decimal arithmetic (the exact value to far below binary64 rounding)."""
    from decimal import Decimal, localcontext
    Tq = np.asarray(T, np.int64).reshape(-1, r)
    m = int(Tq.sum())
    nj = [int(x) for x in Tq.sum(axis=1)]
    nk = [int(x) for x in Tq.sum(axis=0)]
    with localcontext() as ctx:
        ctx.prec = digits
        tot = Decimal(0)
        for j in range(Tq.shape[0]):
            for k in range(r):
                n = int(Tq[j, k])
                if n:
                    tot += Decimal(n) / m * (Decimal(m * n) / (nj[j] * nk[k])).ln()
        return float(tot)


@pytest.mark.parametrize("seed", range(6))
def test_mi_of_nearly_independent_tables(seed):
    """Near independence the terms of MI cancel to a value many orders of
    magnitude below them; the oracle still matches the high-precision value
    of the definition to 1e-9 relative (an evaluation that rounds each
    ratio m N / (N_j N_k) before its logarithm is off by about 1e-6 here)."""
    rng = np.random.default_rng(100 + seed)
    q, r = int(rng.integers(2, 5)), int(rng.integers(2, 4))
    # an exact product table plus a few unit moves keeping the margins close
    rows = rng.integers(200_000, 1_200_000, size=q)
    cols = rng.integers(2, 9, size=r)
    Tq = np.outer(rows, cols).astype(np.int64)
    for _ in range(3):
        a, b = rng.integers(0, q), rng.integers(0, r)
        Tq[a, b] += int(rng.integers(1, 40))
    T = Tq.ravel()
    ref = decimal_mi(T, r)
    assert 0 < ref < 1e-7
    assert orc.mi(T, r) == pytest.approx(ref, rel=1e-9)


# ------------------------------------------------------------ pairs
@pytest.mark.parametrize("seed", range(6))
def test_gram_is_matmul(seed):
    rng = np.random.default_rng(seed)
    n, m = int(rng.integers(1, 40)), int(rng.integers(1, 9000))
    A = (rng.random((n, m)) < rng.random((n, 1)) * 0.3).astype(np.uint8)
    G = orc.gram(A)
    A64 = A.astype(np.int64)
    np.testing.assert_array_equal(G, A64 @ A64.T)
    np.testing.assert_array_equal(np.diag(G), A64.sum(axis=1))


def test_pairs_threshold_is_strict():
    G = np.array([[10, 4, 5], [4, 8, 2], [5, 2, 6]], np.int64)
    recs = orc.pairs(G, 20, 0.2)                                    # N_ab > 4 only
    assert [(a, b, n) for a, b, n, *_ in recs] == [(0, 2, 5)]
    a, b, nab, s, cab, cba = recs[0]
    assert (s, cab, cba) == (5 / 20, 5 / 10, 5 / 6)


# ------------------------------------------------------------ association rules
def test_arm_hand_example():
    # transactions over items 0..3:  {0,1,2} {0,1} {0,2} {1,2} {0,1,2,3}
    T = [[0, 1, 2], [0, 1], [0, 2], [1, 2], [0, 1, 2, 3]]
    D = np.zeros((4, 5), np.uint8)
    for p, t in enumerate(T):
        D[t, p] = 1
    freq, rules = orc.arm_bruteforce(D, 0.3, 0.6)
    assert freq == {(0,): 4, (1,): 4, (2,): 4, (0, 1): 3, (0, 2): 3, (1, 2): 3, (0, 1, 2): 2}
    # six pair rules at 3/4 and three triple rules at 2/3
    assert len(rules) == 9
    assert sorted(r[3] for r in rules) == [2 / 3] * 3 + [3 / 4] * 6
    _, rules7 = orc.arm_bruteforce(D, 0.3, 0.7)
    assert len(rules7) == 6 and all(len(r[0]) == 1 for r in rules7)


def test_arm_antimonotone_and_counts():
    rng = np.random.default_rng(4)
    D = (rng.random((9, 400)) < 0.45).astype(np.uint8)
    freq, rules = orc.arm_bruteforce(D, 0.1, 0.5, max_size=4)
    ar = np.full(9, 2, np.uint8)
    for S, c in freq.items():
        assert c == orc.count_assignment(D, ar, list(S), [1] * len(S))
        for x in range(len(S)):
            if len(S) > 1:
                assert S[:x] + S[x + 1:] in freq          # every subset is frequent
    for ante, x, sup, conf in rules:
        assert conf > 0.5 and sup > 0.1


# ------------------------------------------------------------ sparse tables
@pytest.mark.parametrize("seed", range(15))
def test_sparse_table_is_dense_nonzeros(seed):
    rng, D, ar = rand_db(seed, n=5, m=int(np.random.default_rng(seed).integers(1, 400)), rmax=7)
    vs = [int(v) for v in rng.permutation(5)[: int(rng.integers(1, 6))]]
    T = orc.count(D, ar, vs)
    keys, cnt = orc.count_sparse(D, ar, vs)
    nz = np.nonzero(T)[0]
    np.testing.assert_array_equal(keys, nz)
    np.testing.assert_array_equal(cnt, T[nz])
    assert len(keys) <= min(T.size, D.shape[1])


def test_sparse_table_huge_key_space():
    rng = np.random.default_rng(2)
    ar = np.full(8, 99, np.uint8)                      # 99^8 ~ 9.2e15 cells
    D = rng.integers(0, 99, size=(8, 3000)).astype(np.uint8)
    D[:, 1000:1010] = D[:, 0:1]                        # ten copies of instance 0
    keys, cnt = orc.count_sparse(D, ar, list(range(8)))
    assert int(cnt.sum()) == 3000 and np.all(np.diff(keys) > 0)
    key0 = 0
    for v in range(8):
        key0 = key0 * 99 + int(D[v, 0])
    assert int(cnt[np.searchsorted(keys, key0)]) >= 11
