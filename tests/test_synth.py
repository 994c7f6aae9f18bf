"""The seeded generators are deterministic and have the documented shapes."""
import hashlib

import numpy as np

from paper_1804_04640_amd import synth


def digest(w):
    h = hashlib.sha256()
    for a in (w.D, w.arity, w.vars_flat, w.var_off):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_generators_are_deterministic():
    a, b = synth.plain_small(), synth.plain_small()
    assert digest(a) == digest(b)
    c, d = synth.batched_uneven(m=20_000, nq=300), synth.batched_uneven(m=20_000, nq=300)
    assert digest(c) == digest(d)


def test_shapes_and_ranges():
    w = synth.plain_small()
    assert w.D.shape == (8, 10_000) and w.nq == 1000
    assert set(np.unique(w.arity)) <= {2, 3, 4}
    assert np.all(w.D < w.arity[:, None])
    ks = np.diff(w.var_off)
    assert ks.min() >= 1 and ks.max() <= 4
    for q in w.queries():
        assert len(set(q.tolist())) == len(q)
    w3 = synth.batched_uneven(m=5000, nq=500)
    assert w3.arity.min() >= 2 and w3.arity.max() <= 8
    assert np.all(w3.D < w3.arity[:, None])
    w2 = synth.bn_family(m=3000, nq=200)
    ks = np.diff(w2.var_off)
    assert ks.min() >= 1 and ks.max() <= 5


def test_zipf_marginals_mean():
    f = synth.zipf_marginals(1024)
    assert abs(f.mean() - 0.01) < 1e-9 and f[0] == 1.0


def test_serving_batches_shape():
    rng = synth.rng_for(99)
    b = synth.hill_climb_batches(rng, 64, 6)
    sizes = [len(x) for x in b]
    assert min(sizes) >= 10 and max(sizes) <= 5000
    for fam in (f for x in b for f in x):
        assert 2 <= len(fam) <= 7 and len(set(fam)) == len(fam)
