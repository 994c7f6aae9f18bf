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


def test_minsup_at_or_above_one_admits_no_pair():
    rng = synth.rng_for(96)
    D = (rng.random((6, 5000)) < 0.9).astype(np.uint8)
    D[:, :100] = 1                               # every item pair occurs
    with Database(D, np.full(6, 2, np.uint8)) as db:
        for minsup in (1.0, 7.5, 1e300):
            recs, _, total = db.pairs(minsup)
            assert total == 0 and len(recs) == 0
        recs, _, total = db.pairs(0.0)           # every co-occurring pair
        assert total == 15


def test_rejects_non_binary():
    D = np.zeros((2, 10), np.uint8)
    with Database(D, np.array([2, 3], np.uint8)) as db:
        with pytest.raises(_lib.FastcountError):
            db.pairs(0.1)


def test_gram_beyond_2_24_instances():
    """m = 2^25 + 4097 instances at 75% density: pair counts pass 2^24,
    the most a single fp32 accumulator sums exactly, so the instance range
    must be split.  The diagonal and 60 sampled pairs equal the oracle's
    single-assignment counts; the Gram is symmetric."""
    rng = synth.rng_for(95)
    n, m = 24, (1 << 25) + 4097
    D = (rng.random((n, m), dtype=np.float32) < 0.75).astype(np.uint8)
    ar = np.full(n, 2, np.uint8)
    print("gram beyond 2^24: n=%d m=%d" % (n, m), flush=True)
    with Database(D, ar) as db:
        _, G, _ = db.pairs(0.5, gram=True)
        G = G.cpu().numpy()
    assert np.array_equal(G, G.T)
    assert G[np.triu_indices(n, 1)].min() > (1 << 24)
    for a in range(n):
        assert G[a, a] == orc.count_assignment(D, ar, [a], [1])
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n)]
    for i in rng.choice(len(pairs), size=60, replace=False):
        a, b = pairs[int(i)]
        assert G[a, b] == orc.count_assignment(D, ar, [a, b], [1, 1]), (a, b)
