"""The stored full-size oracle results (tests/golden/fullsize_*.npz) agree
with the oracle and the seeded generators as they are now, on a sample of
queries; and the table digest they hold tells tables apart."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1804_04640_amd import synth
from tests.golden_io import array_sha, load_fullsize, table_digest, table_digests

WORKLOADS = {"bn-family": synth.bn_family, "batched-uneven": synth.batched_uneven,
             "serving": synth.serving}


def test_digest_detects_every_single_cell_change():
    rng = np.random.default_rng(7)
    T = rng.integers(0, 1 << 20, size=300).astype(np.int64)
    d = table_digest(T)
    for c in range(T.size):
        for delta in (1, -1, 12345):
            U = T.copy()
            U[c] += delta
            assert table_digest(U) != d
    # moving a count between two cells changes it too
    U = T.copy()
    U[3] += 5
    U[200] -= 5
    assert table_digest(U) != d


def test_packed_digests_equal_one_by_one():
    rng = np.random.default_rng(8)
    sizes = rng.integers(1, 40, size=500)
    off = np.zeros(501, np.int64)
    off[1:] = np.cumsum(sizes)
    T = rng.integers(0, 1000, size=int(off[-1])).astype(np.int32)
    got = table_digests(T, off, chunk_cells=97)
    exp = [table_digest(T[off[i]:off[i + 1]]) for i in range(500)]
    assert list(got) == exp


@pytest.mark.parametrize("name", sorted(WORKLOADS))
def test_stored_results_match_the_oracle_on_a_sample(name):
    ref = load_fullsize(name)
    w = WORKLOADS[name]()
    assert int(ref["nq"]) == w.nq and int(ref["m"]) == w.m
    assert str(ref["data_sha"]) == array_sha(w.D, w.arity)
    assert str(ref["query_sha"]) == array_sha(w.vars_flat, w.var_off)
    reducers = [str(r) for r in ref["reducers"]]
    assert tuple(reducers) == tuple(w.reducers)
    rng = np.random.default_rng(3)
    for i in rng.choice(w.nq, size=6, replace=False):
        q = w.query(int(i))
        T = orc.count(w.D, w.arity, q)
        assert table_digest(T) == ref["digest"][i]
        r = int(w.arity[q[-1]])
        for slot, red in enumerate(reducers):
            assert orc.score(red, T, r, float(ref["ess"])) == ref["scores"][slot][i]
