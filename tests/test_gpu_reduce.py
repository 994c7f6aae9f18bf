"""GPU parity of the fused float32 reducers against the binary64 oracle."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1804_04640_amd import synth
from paper_1804_04640_amd.api import Database
from tests.golden_io import fig1_database, fig1_expected

pytestmark = pytest.mark.gpu
REL = 1e-6


def check_scores(w, scores, errs, names, ess=1.0, idx=None):
    worst = {}
    for name in names:
        s = scores[name].cpu().numpy()
        e = errs[name].cpu().numpy() if errs is not None else None
        worst[name] = 0.0
        for i in (range(w.nq) if idx is None else idx):
            q = w.query(i)
            T = orc.count(w.D, w.arity, q)
            ref = orc.score(name, T, int(w.arity[q[-1]]), ess)
            diff = abs(float(s[i]) - ref)
            if ref != 0.0:
                rel = diff / abs(ref)
                worst[name] = max(worst[name], rel)
                assert rel <= REL, (name, i, list(q), float(s[i]), ref, rel)
            else:
                assert diff <= 1e-6, (name, i, float(s[i]))
            if e is not None:
                assert diff <= float(e[i]) + 1e-30, ("err estimate too small", name, i, diff, e[i])
    print("worst relative error:", worst, flush=True)


def test_fig1_scores():
    D, ar = fig1_database()
    exp = fig1_expected()
    with Database(D, ar) as db:
        sc, er, _, _ = db.count_reduce([[0, 2, 1]], ("ll", "mdl", "bdeu", "mi"), ess=1.0)
        for name in ("ll", "mdl", "bdeu", "mi"):
            assert float(sc[name][0]) == pytest.approx(exp[name], rel=REL)


def test_bn_family_small_mdl_ll():
    w = synth.bn_family(m=100_003, nq=500)
    with Database(w.D, w.arity) as db:
        sc, er, tables, toff = db.count_reduce((w.vars_flat, w.var_off), ("ll", "mdl"),
                                               keep_tables=True)
        torch.cuda.synchronize()
        check_scores(w, sc, er, ("ll", "mdl"))


def test_batched_uneven_small_bdeu_mi():
    w = synth.batched_uneven(m=80_021, nq=400)
    with Database(w.D, w.arity) as db:
        sc, er, _, _ = db.count_reduce((w.vars_flat, w.var_off), ("bdeu", "mi"), ess=1.0)
        torch.cuda.synchronize()
        check_scores(w, sc, er, ("bdeu", "mi"))


@pytest.mark.parametrize("ess", [0.5, 10.0])
def test_bdeu_other_ess(ess):
    w = synth.bn_family(m=30_000, nq=200)
    with Database(w.D, w.arity) as db:
        sc, er, _, _ = db.count_reduce((w.vars_flat, w.var_off), ("bdeu",), ess=ess)
        check_scores(w, sc, er, ("bdeu",), ess=ess)


def test_stress_tables_near_deterministic_and_independent():
    # near-deterministic families (LL, BDeu cancellation) and exactly
    # independent ones (MI cancellation) at m = 2^22
    rng = np.random.default_rng(11)
    m = 1 << 22
    a = rng.integers(0, 4, m).astype(np.uint8)
    b = rng.integers(0, 3, m).astype(np.uint8)
    det = ((a + b) % 4).astype(np.uint8)
    flip = rng.random(m) < 1e-5
    det[flip] = (det[flip] + 1) % 4
    ind = rng.integers(0, 5, m).astype(np.uint8)
    D = np.stack([a, b, det, ind])
    ar = np.array([4, 3, 4, 5], np.uint8)
    w = synth.Workload("stress", D, ar, *synth.flatten([[0, 1, 2], [0, 2], [0, 1, 3], [3], [2, 0]]))
    with Database(D, ar) as db:
        names = ("ll", "mdl", "bdeu", "mi")
        sc, er, _, _ = db.count_reduce((w.vars_flat, w.var_off), names)
        check_scores(w, sc, er, names)


def test_scores_alone_equal_scores_in_batch():
    w = synth.batched_uneven(m=40_000, nq=120)
    with Database(w.D, w.arity) as db:
        sc, _, _, _ = db.count_reduce((w.vars_flat, w.var_off), ("bdeu", "mi"))
        for i in range(0, w.nq, 11):
            one, _, _, _ = db.count_reduce([w.query(i)], ("bdeu", "mi"))
            for name in ("bdeu", "mi"):
                assert float(one[name][0]) == float(sc[name][i])   # bit-identical
