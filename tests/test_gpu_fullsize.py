"""Parity at the full workload sizes, in the launch configuration the
benchmark times (autotuned tuning installed): oracle comparisons on sampled
queries, and properties that hold at any size checked on every query."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1804_04640_amd import synth
from paper_1804_04640_amd.api import Database

pytestmark = pytest.mark.gpu
REL = 1e-6


def autotuned(w):
    db = Database(w.D, w.arity)
    rng = np.random.default_rng(0)
    ids = np.sort(rng.choice(w.nq, size=min(w.nq, max(2000, w.nq // 20)), replace=False))
    db.autotune([w.query(int(i)) for i in ids])
    return db


def check_full(w, reducers, nsample):
    print("%s: %d queries, m=%d" % (w.name, w.nq, w.m), flush=True)
    db = autotuned(w)
    sc, er, tables, toff = db.count_reduce((w.vars_flat, w.var_off), reducers, ess=w.ess,
                                           keep_tables=True)
    torch.cuda.synchronize()
    T = tables.cpu().numpy()
    # every table sums to m (all queries)
    sums = np.add.reduceat(T.astype(np.int64), toff[:-1]) if w.nq else []
    assert np.all(sums == w.m)
    assert np.all(T >= 0)
    # marginalising every table over its child (last) variable reproduces the
    # table of the remaining variables, counted as queries of their own
    multi = [i for i in range(w.nq) if w.var_off[i + 1] - w.var_off[i] >= 2]
    subs = [w.query(i)[:-1] for i in multi]
    if subs:
        ST, soff = db.count_batch(subs)
        ST = ST.cpu().numpy()
        for j, i in enumerate(multi):
            q = w.query(i)
            r = int(w.arity[q[-1]])
            marg = T[toff[i]:toff[i + 1]].reshape(-1, r).sum(axis=1)
            assert np.array_equal(marg, ST[soff[j]:soff[j + 1]]), "query %d" % i
    rng = np.random.default_rng(1)
    sample = rng.choice(w.nq, size=min(nsample, w.nq), replace=False)
    # the largest tables are always in the sample
    cells = np.diff(toff)
    sample = np.unique(np.concatenate([sample, np.argsort(cells)[-5:]]))
    scores = {r: sc[r].cpu().numpy() for r in reducers}
    errs = {r: er[r].cpu().numpy() for r in reducers}
    worst = {r: 0.0 for r in reducers}
    for i in sample:
        q = w.query(int(i))
        ref = orc.count(w.D, w.arity, q)
        np.testing.assert_array_equal(T[toff[i]:toff[i + 1]], ref, err_msg="query %d" % i)
        r = int(w.arity[q[-1]])
        for name in reducers:
            s_ref = orc.score(name, ref, r, w.ess)
            d = abs(float(scores[name][i]) - s_ref)
            tol = REL * abs(s_ref) if s_ref != 0 else 1e-6
            assert d <= tol, (name, int(i), float(scores[name][i]), s_ref)
            assert d <= float(errs[name][i]) + 1e-30
            if s_ref:
                worst[name] = max(worst[name], d / abs(s_ref))
    print("worst relative error over %d sampled queries: %s" % (len(sample), worst), flush=True)
    db.close()


def test_bn_family_full():
    check_full(synth.bn_family(), ("mdl",), 300)


def test_batched_uneven_full():
    check_full(synth.batched_uneven(), ("bdeu", "mi"), 150)


def test_serving_database_full():
    w = synth.serving(nbatches=16)
    check_full(w, ("mdl",), 150)


def test_all_pairs_full():
    w = synth.all_pairs()
    n, m = w.D.shape
    with Database(w.D, w.arity) as db:
        recs, G, total = db.pairs(w.minsup, gram=True)
        G = G.cpu().numpy()
    ref = orc.gram(w.D)
    np.testing.assert_array_equal(G, ref)
    exp = orc.pairs(ref, m, w.minsup)
    assert total == len(exp)
    got = [(int(r["a"]), int(r["b"]), int(r["n_ab"])) for r in recs]
    assert got == [e[:3] for e in exp]
    print("pairs above minsup: %d" % total, flush=True)


def test_maximum_instances():
    """m = 2^31 - 1, the largest database int32 counts allow (the padded
    extent is exactly 2^31 rows).  The data repeats a random block of
    P = 2^20 + 7 instances, so every expected table is reps * T(block) +
    T(first rem instances of the block), both counted by the oracle."""
    m = (1 << 31) - 1
    P = (1 << 20) + 7
    reps, rem = divmod(m, P)
    rng = synth.rng_for(91)
    ar = np.array([2, 3, 16], np.uint8)
    block = np.stack([rng.integers(0, a, size=P) for a in ar]).astype(np.uint8)
    print("maximum-size database: m=%d, n=3, period %d" % (m, P), flush=True)
    D = np.empty((3, m), np.uint8)
    for v in range(3):
        D[v, :reps * P] = np.tile(block[v], reps)
        D[v, reps * P:] = block[v, :rem]

    def expect(q):
        return reps * orc.count(block, ar, q).astype(np.int64) + \
            orc.count(np.ascontiguousarray(block[:, :rem]), ar, q).astype(np.int64)

    queries = [[0, 1], [1, 0], [2, 1], [0, 1, 2], [2, 0, 1], [2]]
    with Database(D, ar) as db:
        del D
        for strategy in ("auto", "bitmap", "hist", "partition"):
            tables, off = db.count_batch(queries, strategy=strategy)
            T = tables.cpu().numpy()
            for i, q in enumerate(queries):
                np.testing.assert_array_equal(T[off[i]:off[i + 1]], expect(q), err_msg=strategy)
        sc, _, _, _ = db.count_reduce(queries, ("ll",))
        assert np.all(np.isfinite(sc["ll"].cpu().numpy()))
        assert db.count_assignment([2, 1], [5, 2]) == int(expect([2, 1])[5 * 3 + 2])
        keys, cnt, nnz = db.count_sparse([2, 1, 0], cap=4096)
        ref = expect([2, 1, 0])
        nz = np.nonzero(ref)[0]
        assert nnz == len(nz)
        np.testing.assert_array_equal(keys, nz)
        np.testing.assert_array_equal(cnt, ref[nz])
