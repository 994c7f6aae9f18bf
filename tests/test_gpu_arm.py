"""GPU association-rule mining and batched single-assignment counts."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1804_04640_amd import arm, synth
from paper_1804_04640_amd.api import Database

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("bits", [True, False])
def test_count_assignments_batch(bits):
    w = synth.batched_uneven(m=70_001, nq=10)
    rng = np.random.default_rng(3)
    qs, st = [], []
    for _ in range(300):
        k = int(rng.integers(1, 9))
        vs = rng.choice(w.n, k, replace=False)
        qs.append(vs)
        st.append([int(rng.integers(0, w.arity[v])) for v in vs])
    with Database(w.D, w.arity, bitvectors=bits) as db:
        got = db.count_assignments(qs, st)
    for q, s, g in zip(qs, st, got):
        assert g == orc.count_assignment(w.D, w.arity, q, s)


def test_mining_matches_exhaustive_definition():
    rng = np.random.default_rng(8)
    n, m = 13, 20_011
    D = (rng.random((n, m)) < rng.random((n, 1)) * 0.5).astype(np.uint8)
    grp = [2, 5, 7, 11]                       # a planted correlated group
    fire = rng.random(m) < 0.35
    for a in grp:
        D[a] |= (fire & (rng.random(m) < 0.8)).astype(np.uint8)
    with Database(D, np.full(n, 2, np.uint8)) as db:
        freq, rules = arm.mine(db, minsup=0.05, minconf=0.3, max_size=6)
    ref_freq, ref_rules = orc.arm_bruteforce(D, 0.05, 0.3, max_size=6)
    assert freq == ref_freq
    assert [(a, x) for a, x, _, _ in rules] == [(a, x) for a, x, _, _ in ref_rules]
    for (_, _, s, c), (_, _, rs, rc) in zip(rules, ref_rules):
        assert s == rs and c == rc              # same integers, same binary64 division
    assert max(len(s) for s in freq) >= 4


def test_mining_edge_cases_and_item_subsets():
    from paper_1804_04640_amd import _lib
    rng = np.random.default_rng(21)
    n, m = 12, 9_001
    D = (rng.random((n, m)) < rng.random((n, 1)) * 0.6).astype(np.uint8)
    ar = np.full(n, 2, np.uint8)
    ar[11] = 3
    D[11] = rng.integers(0, 3, size=m)
    sub = [0, 3, 4, 7, 9, 10]
    with Database(D, ar) as db:
        for max_size in (1, 2, 4):
            freq, rules = arm.mine(db, minsup=0.02, minconf=0.2, items=sub, max_size=max_size)
            ref_freq, ref_rules = orc.arm_bruteforce(D[sub], 0.02, 0.2, max_size=max_size)
            remap = lambda t: tuple(sub[i] for i in t)
            assert freq == {remap(s): c for s, c in ref_freq.items()}
            assert rules == sorted((remap(a), sub[x], sp, cf) for a, x, sp, cf in ref_rules)
        freq, rules = arm.mine(db, minsup=1.0, minconf=0.0, items=sub)
        assert freq == {} and rules == []
        freq, rules = arm.mine(db, minsup=0.0, minconf=1.0, items=[])
        assert freq == {} and rules == []
        for bad in ([0, 11], [2, 2], [0, 40]):
            with pytest.raises(_lib.FastcountError):
                arm.mine(db, minsup=0.1, minconf=0.1, items=bad)
        with pytest.raises(_lib.FastcountError):
            arm.mine(db, minsup=0.1, minconf=0.1, items=sub, max_size=9)


def test_mining_on_planted_transactions():
    w = synth.all_pairs(m=1 << 16, n=64, groups=4)
    with Database(w.D, w.arity) as db:
        freq, rules = arm.mine(db, minsup=0.002, minconf=0.3, max_size=6)
        # every reported support is the single-assignment count
        some = list(freq.items())[:: max(1, len(freq) // 40)]
        for S, c in some:
            assert c == orc.count_assignment(w.D, w.arity, list(S), [1] * len(S))
        # nothing frequent was missed among itemsets of size <= 3
        ref, _ = orc.arm_bruteforce(w.D[:, :], 0.002, 0.3, max_size=2)
        assert {s: c for s, c in freq.items() if len(s) <= 2} == ref


def test_sparse_tables():
    from paper_1804_04640_amd import synth as S
    rng = S.rng_for(77)
    n = 10
    ar = rng.integers(3, 100, size=n).astype(np.uint8)         # Mildew-like arities
    order, parents = S.random_dag(rng, n, 3)
    D = S.forward_sample(rng, ar, order, parents, 150_001, 0.5)
    with Database(D, ar) as db:
        for vs in ([0, 1, 2, 3, 4, 5, 6, 7], [9, 3, 5], [4], list(range(10))[:8][::-1]):
            keys, cnt, nnz = db.count_sparse(vs)
            rk, rc = orc.count_sparse(D, ar, vs)
            assert nnz == len(rk)
            np.testing.assert_array_equal(keys, rk)
            np.testing.assert_array_equal(cnt, rc)
        # a small table: sparse equals the dense table's non-zeros
        vs = [2, 5]
        dense = db.count(vs).cpu().numpy()
        keys, cnt, _ = db.count_sparse(vs)
        nz = np.nonzero(dense)[0]
        np.testing.assert_array_equal(keys, nz)
        np.testing.assert_array_equal(cnt, dense[nz])
        keys, cnt, nnz = db.count_sparse([0, 1, 2], cap=5)
        assert len(keys) == 5 and nnz > 5


def test_sparse_tables_skewed_keys():
    """Keys that pile up: one configuration holds 90% of the instances and a
    few hundred share most of the rest, so the partition meets buckets that
    stay large down to the last digit, and leaves of every size; plus a
    uniform column set and a table of one configuration."""
    rng = synth.rng_for(78)
    m = (1 << 20) + 333
    ar = np.array([97, 89, 83, 79, 71, 67, 2, 1], np.uint8)
    D = np.zeros((8, m), np.uint8)
    hot = rng.random(m) < 0.9
    warm = rng.integers(0, 300, size=m)
    for v in range(8):
        a = int(ar[v])
        common = rng.integers(0, a, size=300)
        D[v] = np.where(hot, a // 2, np.where(rng.random(m) < 0.8, common[warm],
                                              rng.integers(0, a, size=m))).astype(np.uint8)
    D[7] = 0
    print("skewed sparse keys: m=%d" % m, flush=True)
    with Database(D, ar, bitvectors=False) as db:
        qs = [[0, 1, 2, 3, 4, 5], [5, 4, 3, 2, 1, 0, 6], [0, 1], [7], [7, 6, 0],
              [2, 3, 4, 5, 6, 7, 0, 1]]
        keys, cnts, off = db.count_sparse_batch(qs)
        keys, cnts = keys.cpu().numpy(), cnts.cpu().numpy()
        for i, q in enumerate(qs):
            rk, rc = orc.count_sparse(D, ar, q)
            np.testing.assert_array_equal(keys[off[i]:off[i + 1]], rk, err_msg=str(q))
            np.testing.assert_array_equal(cnts[off[i]:off[i + 1]], rc, err_msg=str(q))
            k1, c1, n1 = db.count_sparse(q)
            assert n1 == len(rk)
            np.testing.assert_array_equal(k1, rk)
            np.testing.assert_array_equal(c1, rc)


@pytest.mark.parametrize("score", ["mdl", "bdeu"])
def test_parent_set_assignment_is_exact(score):
    import itertools
    from paper_1804_04640_amd import parents
    w = synth.bn_family(m=4000, nq=1)
    D, ar = w.D[:7].copy(), w.arity[:7].copy()       # 7 variables of the DAG sample
    n = 7
    with Database(D, ar) as db:
        best, stats = parents.best_parents(db, max_pa=3, score=score)
    for c in range(n):
        others = [v for v in range(n) if v != c]
        ref = {}
        for k in range(0, 4):
            for pa in itertools.combinations(others, k):
                T = orc.count(D, ar, list(pa) + [c])
                ref[pa] = orc.score(score, T, int(ar[c]), 1.0)
        opt = min(ref.values()) if score == "mdl" else max(ref.values())
        got_pa, got_s = best[c]
        # the chosen set is optimal up to the float32 tolerance of the scores
        assert abs(ref[tuple(sorted(got_pa))] - opt) <= 2e-6 * abs(opt) + 1e-9, (c, got_pa)
        assert abs(got_s - ref[tuple(sorted(got_pa))]) <= 1e-6 * abs(opt) + 1e-9
    if score == "mdl":
        assert stats["scored"] + stats["pruned"] == n * (1 + 6 + 15 + 20)


def test_score_parent_sets_matches_explicit_families():
    import ctypes
    import itertools
    import math
    from paper_1804_04640_amd import _lib
    w = synth.bn_family(m=30_011, nq=1)
    D, ar = w.D[:9].copy(), w.arity[:9].copy()
    child, cand = 4, np.array([7, 0, 2, 8, 1, 5], np.int32)
    with Database(D, ar) as db:
        for size in (0, 1, 3, 6):
            sets = [list(cand[list(p)]) for p in itertools.combinations(range(len(cand)), size)]
            ref, _, _, _ = db.count_reduce([s + [child] for s in sets], ("mdl", "bdeu"))
            got = db.score_parent_sets(child, cand, size, ("mdl", "bdeu"))
            for name in ("mdl", "bdeu"):
                assert torch.equal(got[name], ref[name]), (size, name)
            # pruning: +inf exactly where the penalty alone reaches the bound
            mdl = ref["mdl"].cpu().numpy()
            bound = float(np.median(mdl)) if size else float(mdl[0]) + 1.0
            pruned = db.score_parent_sets(child, cand, size, ("mdl",), prune_mdl=bound)["mdl"]
            pruned = pruned.cpu().numpy()
            lg = 0.5 * math.log2(D.shape[1]) * (int(ar[child]) - 1)
            for i, s in enumerate(sets):
                pen = lg * float(np.prod(ar[s].astype(np.float64))) if s else lg
                if pen < bound:
                    assert pruned[i] == mdl[i], (size, i)
                else:
                    assert np.isinf(pruned[i]) and pruned[i] > 0, (size, i)
        # host output buffer, and argument errors
        out = np.empty(math.comb(len(cand), 2), np.float32)
        params = _lib.fc_reduce_params(1.0)
        _lib.fc_score_parent_sets(db.handle, child, cand.ctypes.data, len(cand), 2,
                                  _lib.FC_RED_MDL, ctypes.addressof(params), 0.0,
                                  out.ctypes.data, len(out), 0)
        sets = [list(cand[list(p)]) + [child] for p in itertools.combinations(range(len(cand)), 2)]
        np.testing.assert_array_equal(out, db.count_reduce(sets, ("mdl",))[0]["mdl"].cpu().numpy())
        for bad_cand in (np.array([1, 1], np.int32), np.array([child, 2], np.int32)):
            with pytest.raises(_lib.FastcountError):
                db.score_parent_sets(child, bad_cand, 1, ("mdl",))
        with pytest.raises(_lib.FastcountError):
            db.score_parent_sets(child, cand, 2, ("mdl", "bdeu"), prune_mdl=10.0)


def test_sparse_tables_high_arity_full_size_device_outputs():
    """The high-arity workload at its full size (m = 1,000,000, tables of more
    than 2^24 cells): device-resident outputs equal the oracle's pairs, and a
    cap below the number of configurations keeps the smallest keys."""
    w = synth.high_arity()
    keys = torch.empty(w.m, dtype=torch.int64, device="cuda")
    cnts = torch.empty(w.m, dtype=torch.int32, device="cuda")
    with Database(w.D, w.arity, bitvectors=False) as db:
        for i in (0, 1, 17, 63):
            q = w.query(i)
            k, c, nnz = db.count_sparse(q, keys_out=keys, counts_out=cnts)
            rk, rc = orc.count_sparse(w.D, w.arity, q)
            assert nnz == len(rk) and k.is_cuda
            np.testing.assert_array_equal(k.cpu().numpy(), rk)
            np.testing.assert_array_equal(c.cpu().numpy(), rc)
        small_k, small_c = keys[:1000], cnts[:1000]
        k, c, nnz = db.count_sparse(w.query(0), keys_out=small_k, counts_out=small_c)
        rk, rc = orc.count_sparse(w.D, w.arity, w.query(0))
        assert nnz == len(rk) and len(k) == 1000
        np.testing.assert_array_equal(k.cpu().numpy(), rk[:1000])
        np.testing.assert_array_equal(c.cpu().numpy(), rc[:1000])


def test_sparse_batch_high_arity_full_size():
    """All 64 high-arity queries in one batched call (one composite-key sort
    per group) equal the oracle's sparse tables query by query."""
    w = synth.high_arity()
    with Database(w.D, w.arity, bitvectors=False) as db:
        keys, cnts, off = db.count_sparse_batch((w.vars_flat, w.var_off))
        keys, cnts = keys.cpu().numpy(), cnts.cpu().numpy()
    assert off[0] == 0 and off[-1] == len(keys)
    for i in range(w.nq):
        rk, rc = orc.count_sparse(w.D, w.arity, w.query(i))
        np.testing.assert_array_equal(keys[off[i]:off[i + 1]], rk)
        np.testing.assert_array_equal(cnts[off[i]:off[i + 1]], rc)


def _mixed_sparse_batch():
    rng = synth.rng_for(78)
    n, m = 20, 3001
    ar = rng.integers(2, 100, size=n).astype(np.uint8)
    ar[:3] = 1                                   # single-state variables: key space 1
    D = np.stack([rng.integers(0, a, size=m) for a in ar]).astype(np.uint8)
    qs = [[0], [1, 2], [5], [7, 3]]              # tiny key spaces (32-bit groups)
    for _ in range(300):
        k = int(rng.integers(1, 9))
        qs.append(rng.choice(n, size=k, replace=False).astype(np.int32))
    big = np.argsort(ar)[-8:][::-1]              # the 8 largest arities: > 2^48 keys
    qs += [big, big[::-1], [big[0]]]
    return D, ar, qs


def test_sparse_batch_mixed_groups_and_host_outputs():
    """Key spaces from 1 to beyond 2^48 in one batch (several groups, 32- and
    64-bit composite keys, groups split by the 64-bit budget), checked
    against the oracle; host-memory outputs give the same pairs."""
    from paper_1804_04640_amd import _lib as L
    from paper_1804_04640_amd.api import flatten_queries
    D, ar, qs = _mixed_sparse_batch()
    with Database(D, ar, bitvectors=False) as db:
        keys, cnts, off = db.count_sparse_batch(qs)
        keys, cnts = keys.cpu().numpy(), cnts.cpu().numpy()
        for i, q in enumerate(qs):
            rk, rc = orc.count_sparse(D, ar, q)
            np.testing.assert_array_equal(keys[off[i]:off[i + 1]], rk)
            np.testing.assert_array_equal(cnts[off[i]:off[i + 1]], rc)
        flat, voff = flatten_queries(qs)
        total = int(off[-1])
        hk = np.zeros(total, np.int64)
        hc = np.zeros(total, np.int32)
        hoff = np.zeros(len(qs) + 1, np.int64)
        rc, t2 = L.fc_count_sparse_batch(db.handle, flat.ctypes.data, voff.ctypes.data, len(qs),
                                         hk.ctypes.data, hc.ctypes.data, total, hoff.ctypes.data,
                                         torch.cuda.current_stream().cuda_stream)
        assert rc == L.FC_OK and t2 == total
        np.testing.assert_array_equal(hoff, off)
        np.testing.assert_array_equal(hk, keys)
        np.testing.assert_array_equal(hc, cnts)


def test_sparse_batch_capacity_and_errors():
    from paper_1804_04640_amd import _lib as L
    from paper_1804_04640_amd.api import flatten_queries
    D, ar, qs = _mixed_sparse_batch()
    with Database(D, ar, bitvectors=False) as db:
        _, _, off = db.count_sparse_batch(qs)
        total = int(off[-1])
        small_k = torch.empty(total - 1, dtype=torch.int64, device="cuda")
        small_c = torch.empty(total - 1, dtype=torch.int32, device="cuda")
        flat, voff = flatten_queries(qs)
        hoff = np.zeros(len(qs) + 1, np.int64)
        rc, t2 = L.fc_count_sparse_batch(db.handle, flat.ctypes.data, voff.ctypes.data, len(qs),
                                         small_k.data_ptr(), small_c.data_ptr(), total - 1,
                                         hoff.ctypes.data, torch.cuda.current_stream().cuda_stream)
        assert rc == L.FC_ERR_RANGE and t2 == total
        np.testing.assert_array_equal(hoff, off)          # sizes come back for a retry
        with pytest.raises(L.FastcountError):
            db.count_sparse_batch(qs, keys_out=small_k, counts_out=small_c)
        k, c, o = db.count_sparse_batch([])
        assert len(k) == 0 and list(o) == [0]
        with pytest.raises(L.FastcountError):
            db.count_sparse_batch([[1, 4, 1]])             # a repeated variable
        with pytest.raises(L.FastcountError):
            db.count_sparse_batch([list(range(9))])        # more than 8 variables


def test_sparse_batch_several_windows():
    """A batch of more than 2^27 keys spans several windows (63 queries of
    m = 2^21 + 5 instances each, the last window ragged).  Every query's pairs
    are valid (counts sum to m, keys strictly increasing inside the key
    space); every fifth query and those around window boundaries equal the
    oracle's; a capacity one short of the total fails with the sizes set."""
    from paper_1804_04640_amd import _lib as L
    from paper_1804_04640_amd.api import flatten_queries
    rng = synth.rng_for(91)
    n, m = 12, (1 << 21) + 5
    ar = rng.integers(2, 100, size=n).astype(np.uint8)
    D = np.stack([rng.integers(0, a, size=m) for a in ar]).astype(np.uint8)
    qs = [rng.choice(n, size=int(rng.integers(1, 9)), replace=False).astype(np.int32)
          for _ in range(130)]
    print("several windows: n=%d m=%d queries=%d" % (n, m, len(qs)), flush=True)
    with Database(D, ar, bitvectors=False) as db:
        keys, cnts, off = db.count_sparse_batch(qs)
        keys, cnts = keys.cpu().numpy(), cnts.cpu().numpy()
        assert off[0] == 0 and off[-1] == len(keys)
        for i, q in enumerate(qs):
            k, c = keys[off[i]:off[i + 1]], cnts[off[i]:off[i + 1]]
            cells = int(np.prod(ar[q].astype(np.float64)))
            assert c.sum() == m and c.min() >= 1
            assert k[0] >= 0 and k[-1] < cells and np.all(np.diff(k) > 0)
            if i % 5 == 0 or i in (61, 62, 63, 64, 125, 126, 127, 129):
                rk, rc = orc.count_sparse(D, ar, q)
                np.testing.assert_array_equal(k, rk)
                np.testing.assert_array_equal(c, rc)
        total = int(off[-1])
        del keys, cnts
        small_k = torch.empty(total - 1, dtype=torch.int64, device="cuda")
        small_c = torch.empty(total - 1, dtype=torch.int32, device="cuda")
        flat, voff = flatten_queries(qs)
        hoff = np.zeros(len(qs) + 1, np.int64)
        rc, t2 = L.fc_count_sparse_batch(db.handle, flat.ctypes.data, voff.ctypes.data, len(qs),
                                         small_k.data_ptr(), small_c.data_ptr(), total - 1,
                                         hoff.ctypes.data, torch.cuda.current_stream().cuda_stream)
        assert rc == L.FC_ERR_RANGE and t2 == total
        np.testing.assert_array_equal(hoff, off)


def test_sparse_batch_more_queries_than_a_group_holds():
    """70,000 queries over m = 3 instances: more queries than one group may
    hold (65,535), so one window is cut into several groups; every query's
    pairs equal the oracle's, with device and host outputs."""
    from paper_1804_04640_amd import _lib as L
    from paper_1804_04640_amd.api import flatten_queries
    rng = synth.rng_for(93)
    n, m = 20, 3
    ar = rng.integers(2, 100, size=n).astype(np.uint8)
    D = np.stack([rng.integers(0, a, size=m) for a in ar]).astype(np.uint8)
    qs = [rng.choice(n, size=int(rng.integers(1, 9)), replace=False).astype(np.int32)
          for _ in range(70000)]
    with Database(D, ar, bitvectors=False) as db:
        keys, cnts, off = db.count_sparse_batch(qs)
        keys, cnts = keys.cpu().numpy(), cnts.cpu().numpy()
        assert off[-1] == len(keys)
        for i, q in enumerate(qs):
            rk, rc = orc.count_sparse(D, ar, q)
            np.testing.assert_array_equal(keys[off[i]:off[i + 1]], rk)
            np.testing.assert_array_equal(cnts[off[i]:off[i + 1]], rc)
        flat, voff = flatten_queries(qs)
        total = int(off[-1])
        hk = np.zeros(total, np.int64)
        hc = np.zeros(total, np.int32)
        hoff = np.zeros(len(qs) + 1, np.int64)
        rc, t2 = L.fc_count_sparse_batch(db.handle, flat.ctypes.data, voff.ctypes.data, len(qs),
                                         hk.ctypes.data, hc.ctypes.data, total, hoff.ctypes.data,
                                         torch.cuda.current_stream().cuda_stream)
        assert rc == L.FC_OK and t2 == total
        np.testing.assert_array_equal(hoff, off)
        np.testing.assert_array_equal(hk, keys)
        np.testing.assert_array_equal(hc, cnts)
