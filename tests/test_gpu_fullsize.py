"""Parity at the full workload sizes, in the launch configuration the
benchmark times (autotuned tuning installed).

Every table of every query of the bn-family, batched-uneven and serving
workloads is compared with the CPU oracle's through per-query digests, and
every score with the oracle's binary64 score; both were written by
tests/golden/make_fullsize.py, which runs only the oracle on the seeded
inputs.  A few queries, the largest tables among them, are also counted by
the oracle here and compared cell by cell."""
import time

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1804_04640_amd import synth
from paper_1804_04640_amd.api import Database
from tests.golden_io import array_sha, load_fullsize, table_digests

pytestmark = pytest.mark.gpu
REL = 1e-6


def autotuned(w):
    db = Database(w.D, w.arity)
    rng = np.random.default_rng(0)
    ids = np.sort(rng.choice(w.nq, size=min(w.nq, max(2000, w.nq // 20)), replace=False))
    db.autotune([w.query(int(i)) for i in ids])
    return db


def check_full(w, nsample=16):
    t0 = time.time()
    print("%s: %d queries, m=%d" % (w.name, w.nq, w.m), flush=True)
    ref = load_fullsize(w.name)
    reducers = tuple(str(r) for r in ref["reducers"])
    assert int(ref["m"]) == w.m and int(ref["nq"]) == w.nq
    assert str(ref["data_sha"]) == array_sha(w.D, w.arity), \
        "the seeded generator no longer reproduces the stored database"
    assert str(ref["query_sha"]) == array_sha(w.vars_flat, w.var_off), \
        "the seeded generator no longer reproduces the stored queries"
    db = autotuned(w)
    sc, er, tables, toff = db.count_reduce((w.vars_flat, w.var_off), reducers,
                                           ess=float(ref["ess"]), keep_tables=True)
    torch.cuda.synchronize()
    T = tables.cpu().numpy()
    del tables
    print("  counted on the GPU, %.1f s" % (time.time() - t0), flush=True)
    # every table sums to m
    assert np.all(np.add.reduceat(T.astype(np.int64), toff[:-1]) == w.m)
    # every table equals the oracle's
    got = table_digests(T, toff)
    bad = np.nonzero(got != ref["digest"])[0]
    assert len(bad) == 0, "%d tables differ from the oracle's, first query %d" % (
        len(bad), int(bad[0]))
    # every score within 1e-6 relative of the oracle's binary64 score, and
    # within the GPU's own per-result error estimate
    for slot, name in enumerate(reducers):
        g = sc[name].cpu().numpy().astype(np.float64)
        e = er[name].cpu().numpy().astype(np.float64)
        s_ref = ref["scores"][slot]
        d = np.abs(g - s_ref)
        tol = np.where(s_ref != 0, REL * np.abs(s_ref), 1e-6)
        over = np.nonzero(d > tol)[0]
        assert len(over) == 0, (name, int(over[0]), float(g[over[0]]), float(s_ref[over[0]]))
        assert np.all(d <= e + 1e-30), (name, int(np.argmax(d - e)))
        nz = s_ref != 0
        print("  %s: all %d scores within 1e-6, worst relative error %.2e"
              % (name, w.nq, float(np.max(d[nz] / np.abs(s_ref[nz]))) if nz.any() else 0.0),
              flush=True)
    # a few queries counted by the oracle here, cell by cell
    rng = np.random.default_rng(1)
    cells = np.diff(toff)
    sample = np.unique(np.concatenate([rng.choice(w.nq, size=min(nsample, w.nq), replace=False),
                                       np.argsort(cells)[-4:]]))
    for i in sample:
        q = w.query(int(i))
        np.testing.assert_array_equal(T[toff[i]:toff[i + 1]], orc.count(w.D, w.arity, q),
                                      err_msg="query %d" % i)
    print("  %s: all %d tables equal the oracle's (%.1f s)" % (w.name, w.nq, time.time() - t0),
          flush=True)
    db.close()


def test_bn_family_full():
    check_full(synth.bn_family())


def test_batched_uneven_full():
    check_full(synth.batched_uneven())


def test_serving_database_full():
    check_full(synth.serving())


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
