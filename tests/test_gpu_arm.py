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
