"""GPU parity of the MFMA co-occurrence Gram and the pair records."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1804_04640_amd import _lib, synth
from paper_1804_04640_amd.api import Database

pytestmark = pytest.mark.gpu


def check(D, minsup, items=None):
    n, m = D.shape
    ar = np.full(n, 2, np.uint8)
    with Database(D, ar) as db:
        recs, G, total = db.pairs(minsup, items=items, gram=True)
        G = G.cpu().numpy()
    sub = D if items is None else D[list(items)]
    ref = orc.gram(sub)
    np.testing.assert_array_equal(G, ref)
    assert np.array_equal(G, G.T)
    exp = orc.pairs(ref, m, minsup)
    assert total == len(exp) == len(recs)
    for r, e in zip(recs, exp):
        assert (int(r["a"]), int(r["b"]), int(r["n_ab"])) == e[:3]
        for got, want in zip((r["support"], r["conf_ab"], r["conf_ba"]), e[3:]):
            assert abs(float(got) - want) <= 2 ** -23 * want   # one f32 rounding
    return G


def test_small_ragged():
    rng = np.random.default_rng(1)
    n, m = 150, 70_001                     # two item tiles, ragged instance tail
    p = rng.random((n, 1)) * 0.2
    D = (rng.random((n, m)) < p).astype(np.uint8)
    D[3] = 1                               # an always-present item
    D[7] = 0                               # an item that never occurs
    check(D, 0.001)


def test_item_subset_and_cap():
    rng = np.random.default_rng(2)
    D = (rng.random((40, 9000)) < 0.3).astype(np.uint8)
    items = [5, 1, 30, 2, 17, 33]
    check(D, 0.05, items=items)
    with Database(D, np.full(40, 2, np.uint8)) as db:
        recs, _, total = db.pairs(0.05, cap=3)
        assert len(recs) == 3 and total > 3


def test_all_pairs_reduced():
    w = synth.all_pairs(m=1 << 17)
    check(w.D, 0.001)


def test_rejects_non_binary():
    D = np.zeros((2, 10), np.uint8)
    with Database(D, np.array([2, 3], np.uint8)) as db:
        with pytest.raises(_lib.FastcountError):
            db.pairs(0.1)
