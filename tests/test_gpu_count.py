"""GPU parity: tables of every strategy are bit-identical to the CPU oracle."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1804_04640_amd import _lib, synth
from paper_1804_04640_amd.api import Database
from tests.golden_io import fig1_database, fig1_expected

pytestmark = pytest.mark.gpu


def check_tables(w, tables, toff, idx=None):
    T = tables.cpu().numpy() if isinstance(tables, torch.Tensor) else tables
    for i in (range(w.nq) if idx is None else idx):
        q = w.query(i)
        ref = orc.count(w.D, w.arity, q)
        got = T[toff[i]:toff[i] + len(ref)]
        assert np.array_equal(ref, got), "query %d vars %s" % (i, list(q))


def test_fig1_example():
    D, ar = fig1_database()
    with Database(D, ar) as db:
        T = db.count([0, 2, 1])
        torch.cuda.synchronize()
        np.testing.assert_array_equal(T.cpu().numpy(), fig1_expected()["table"])
        assert db.count_assignment([0, 1, 2], [2, 1, 0]) == 2


@pytest.mark.parametrize("strategy", ["auto", "hist", "bitmap", "partition"])
def test_plain_small_full_batch(strategy):
    w = synth.plain_small()
    print("plain-small strategy=%s nq=%d m=%d" % (strategy, w.nq, w.m), flush=True)
    with Database(w.D, w.arity) as db:
        tables, toff = db.count_batch((w.vars_flat, w.var_off), strategy=strategy)
        torch.cuda.synchronize()
        check_tables(w, tables, toff)


def test_plain_small_per_query_path():
    w = synth.plain_small()
    with Database(w.D, w.arity) as db:
        for i in range(0, w.nq, 7):
            q = w.query(i)
            np.testing.assert_array_equal(db.count(q).cpu().numpy(), orc.count(w.D, w.arity, q))


@pytest.mark.parametrize("strategy", ["auto", "hist", "bitmap", "partition"])
def test_bn_family_small_strategies(strategy):
    w = synth.bn_family(m=100_003, nq=400)        # ragged tail: m is not a tile multiple
    print("bn-family small strategy=%s" % strategy, flush=True)
    with Database(w.D, w.arity) as db:
        tables, toff = db.count_batch((w.vars_flat, w.var_off), strategy=strategy)
        torch.cuda.synchronize()
        check_tables(w, tables, toff)


def test_batched_uneven_small_and_host_output():
    w = synth.batched_uneven(m=60_001, nq=300)
    with Database(w.D, w.arity) as db:
        tables, toff = db.count_batch((w.vars_flat, w.var_off))
        torch.cuda.synchronize()
        check_tables(w, tables, toff)
        # host output buffer (numpy): the call stages and synchronises
        host = np.full(int(toff[-1]), -7, np.int32)
        _lib.fc_count_batch(db.handle, w.vars_flat.ctypes.data, w.var_off.ctypes.data, w.nq,
                            host.ctypes.data, 0, 0, 0)
        check_tables(w, host, toff)


def test_large_table_partition_path():
    # 6 variables of arity 8: 262144 cells > LDS, so the one-pass partition runs (32 parts)
    rng = np.random.default_rng(7)
    m = 70_001
    ar = np.full(6, 8, np.uint8)
    D = rng.integers(0, 8, size=(6, m)).astype(np.uint8)
    with Database(D, ar) as db:
        for vs in ([0, 1, 2, 3, 4, 5], [5, 3, 1, 0, 2, 4]):
            got = db.count(vs).cpu().numpy()
            np.testing.assert_array_equal(got, orc.count(D, ar, vs))


def test_partition_one_pass_slices_and_ragged_parts():
    """Tables of 119,070 to 1.66M cells (parts of 8,192 cells, the last one
    ragged) over m = 2,000,003 instances: 45 queries take the one-pass
    partition in two slices of the shared scratch (42 and 3)."""
    rng = np.random.default_rng(21)
    m = 2_000_003
    ar = np.array([7, 9, 11, 13, 7, 9, 11, 13, 5, 6], np.uint8)
    D = np.stack([rng.integers(0, a, size=m) for a in ar]).astype(np.uint8)
    # a skewed column: most instances in one state
    D[3] = np.where(rng.random(m) < 0.7, 12, D[3]).astype(np.uint8)
    import itertools
    combos = list(itertools.combinations(range(10), 6))   # distinct sets: none derived
    qs = [rng.permutation(combos[j]).astype(np.int32)
          for j in rng.choice(len(combos), 45, replace=False)]
    print("one-pass partition: m=%d queries=%d" % (m, len(qs)), flush=True)
    with Database(D, ar) as db:
        summ = db.plan_summary(qs)
        assert summ["hist"] == len(qs), summ
        tables, toff = db.count_batch(qs)
        T = tables.cpu().numpy()
        for i, q in enumerate(qs):
            np.testing.assert_array_equal(T[toff[i]:toff[i + 1]], orc.count(D, ar, q),
                                          err_msg=str(q))
        # the key windows give the same tables
        t = db.tuning()
        t["one_pass_partition"] = 0
        db.set_tuning(t)
        t2, _ = db.count_batch(qs[:6])
        np.testing.assert_array_equal(t2.cpu().numpy(), T[:toff[6]])


def test_row_sweep_rotated_starts_and_ragged_steps():
    """Histogram workgroups start their row chunks at rotated steps (row
    sweeps).  m = 100,003 with 16,384-row chunks gives chunks of 3 or 4
    tiles, so the packed kernels' steps of two tiles end raggedly inside a
    chunk; 600 queries over every LDS class give each XCD enough
    workgroups that the starts wrap.  Tables equal the oracle with sweeps
    on and off, and the flag accepts only 0 and 1."""
    rng = np.random.default_rng(23)
    m = 100_003
    ar = np.array([2, 3, 4, 5, 6, 7, 8, 9, 3, 4, 5, 2], np.uint8)
    D = np.stack([rng.integers(0, a, size=m) for a in ar]).astype(np.uint8)
    qs = [rng.choice(len(ar), size=int(rng.integers(2, 7)), replace=False).astype(np.int32)
          for _ in range(600)]
    refs = [orc.count(D, ar, q) for q in qs]
    print("row sweeps: m=%d queries=%d" % (m, len(qs)), flush=True)
    with Database(D, ar) as db:
        for sweep in (1, 0):
            t = db.tuning()
            t.update(row_sweep=sweep, chunk_rows=16384, derive_tables=0)
            db.set_tuning(t)
            tables, toff = db.count_batch(qs, strategy="hist")
            T = tables.cpu().numpy()
            for i, q in enumerate(qs):
                np.testing.assert_array_equal(T[toff[i]:toff[i + 1]], refs[i],
                                              err_msg="row_sweep=%d query %s" % (sweep, q))
        t = db.tuning()
        t["row_sweep"] = 2
        with pytest.raises(_lib.FastcountError):
            db.set_tuning(t)


def test_partition_beyond_the_part_table_uses_key_windows():
    """62.7M cells (7 variables of arity 13) exceed the one-pass partition's
    2^25 cells: the key windows count it, equal to the oracle."""
    rng = np.random.default_rng(22)
    m = 20_011
    ar = np.full(7, 13, np.uint8)
    D = rng.integers(0, 13, size=(7, m)).astype(np.uint8)
    q = [6, 0, 5, 1, 4, 2, 3]
    print("key windows: cells=%d m=%d" % (13 ** 7, m), flush=True)
    with Database(D, ar) as db:
        got = db.count(q).cpu().numpy()
        np.testing.assert_array_equal(got, orc.count(D, ar, q))


def test_batch_equals_alone():
    w = synth.batched_uneven(m=30_000, nq=200)
    with Database(w.D, w.arity) as db:
        tables, toff = db.count_batch((w.vars_flat, w.var_off))
        T = tables.cpu().numpy()
        for i in range(0, w.nq, 9):
            alone = db.count(w.query(i)).cpu().numpy()
            np.testing.assert_array_equal(T[toff[i]:toff[i + 1]], alone)


def test_repeat_runs_identical():
    w = synth.bn_family(m=50_000, nq=300)
    with Database(w.D, w.arity) as db:
        a, _ = db.count_batch((w.vars_flat, w.var_off))
        b, _ = db.count_batch((w.vars_flat, w.var_off))
        assert torch.equal(a, b)


def test_edge_cases():
    # empty database, k = 1, arity 1, m smaller than a tile
    D = np.zeros((3, 0), np.uint8)
    ar = np.array([2, 3, 1], np.uint8)
    with Database(D, ar) as db:
        assert db.count([0, 1]).cpu().numpy().tolist() == [0] * 6
    rng = np.random.default_rng(3)
    D = np.stack([rng.integers(0, 2, 5), np.zeros(5), rng.integers(0, 255, 5)]).astype(np.uint8)
    ar = np.array([2, 1, 255], np.uint8)
    with Database(D, ar) as db:
        for vs in ([1], [0, 1], [2], [2, 0, 1]):
            np.testing.assert_array_equal(db.count(vs).cpu().numpy(), orc.count(D, ar, vs))


def test_validation_errors_name_the_query():
    w = synth.plain_small()
    with Database(w.D, w.arity) as db:
        bad = [[0, 1], [2, 2], [3]]
        with pytest.raises(_lib.FastcountError) as e:
            db.count_batch(bad)
        assert e.value.code == _lib.FC_ERR_INVALID and "query 1" in str(e.value)
        with pytest.raises(_lib.FastcountError):
            db.count_batch([[0, 99]])
        with pytest.raises(_lib.FastcountError):
            db.count_batch([list(range(9))])
    with pytest.raises(_lib.FastcountError) as e:
        Database(np.array([[0, 3]], np.uint8), np.array([3], np.uint8))
    assert "arity" in str(e.value)


def test_row_major_and_device_input():
    w = synth.plain_small(m=5000, nq=50)
    with Database(np.ascontiguousarray(w.D.T), w.arity, layout="row") as db:
        tables, toff = db.count_batch((w.vars_flat, w.var_off))
        check_tables(w, tables, toff)
    with Database(torch.from_numpy(w.D).cuda(), w.arity) as db:
        tables, toff = db.count_batch((w.vars_flat, w.var_off))
        check_tables(w, tables, toff)


def test_marginals_and_assignment():
    w = synth.bn_family(m=40_000, nq=10)
    with Database(w.D, w.arity) as db:
        cnt, ent = db.marginals()
        off = 0
        for v in range(w.n):
            np.testing.assert_array_equal(cnt[off:off + int(w.arity[v])],
                                          np.bincount(w.D[v], minlength=w.arity[v]))
            off += int(w.arity[v])
        rng = np.random.default_rng(0)
        for _ in range(20):
            k = int(rng.integers(1, 6))
            vs = rng.choice(w.n, k, replace=False)
            st = [int(rng.integers(0, w.arity[v])) for v in vs]
            assert db.count_assignment(vs, st) == orc.count_assignment(w.D, w.arity, vs, st)
    with Database(w.D, w.arity, bitvectors=False) as db:
        assert db.count_assignment([0, 1], [0, 0]) == orc.count_assignment(w.D, w.arity, [0, 1],
                                                                           [0, 0])


def test_entropies_match_scipy():
    """fc_db_marginals' entropies (bits) equal scipy's entropy of the state
    histogram, and survive an append."""
    from scipy.stats import entropy
    w = synth.batched_uneven(m=60_013, nq=4)
    D = w.D.copy()
    D[3, :] = 0                                   # a constant variable: entropy 0
    with Database(D[:, :40_000].copy(), w.arity) as db:
        _, ent = db.marginals()
        for v in range(w.n):
            ref = entropy(np.bincount(D[v, :40_000], minlength=w.arity[v]), base=2)
            assert abs(float(ent[v]) - ref) <= 1e-5 * max(1.0, ref), v
        assert ent[3] == 0.0
        db.append(D[:, 40_000:].copy())
        _, ent = db.marginals()
        for v in range(w.n):
            ref = entropy(np.bincount(D[v], minlength=w.arity[v]), base=2)
            assert abs(float(ent[v]) - ref) <= 1e-5 * max(1.0, ref), v


def test_bitmap_walk_order_does_not_change_tables():
    """The Bitmap tree walked by ascending entropy and in the query's order
    gives the oracle's tables (Section 3.2: the order only prunes)."""
    w = synth.bn_family(m=70_001, nq=600)
    with Database(w.D, w.arity) as db:
        for order in (1, 0):
            t = db.tuning()
            t["bitmap_order"] = order
            t["bitmap_cells"] = [[1] * 6 for _ in range(8)]     # tables up to 128 cells
            db.set_tuning(t)
            for strategy in ("bitmap", "auto"):
                tables, toff = db.count_batch((w.vars_flat, w.var_off), strategy=strategy)
                check_tables(w, tables, toff)


def _nested_queries(w, rng, nsup=80):
    """Supersets of 4..6 variables (some with the largest arities, so their
    tables need key windows), subsets of 3 and 4 of their variables in
    shuffled order, repeats, chains (3 in 4 in 5) and unrelated queries."""
    qs = []
    big = np.argsort(w.arity)[::-1][:6]
    for s in range(nsup):
        k = int(rng.integers(4, 7))
        sup = big.copy() if s % 16 == 0 else rng.choice(w.n, k, replace=False)
        qs.append(rng.permutation(sup).astype(np.int32))
        mid = rng.choice(sup, 4, replace=False) if len(sup) > 4 else sup
        qs.append(rng.permutation(mid).astype(np.int32))
        for _ in range(3):
            qs.append(rng.permutation(rng.choice(mid, 3, replace=False)).astype(np.int32))
        if s % 3 == 0:
            qs.append(rng.permutation(sup).astype(np.int32))            # a repeat
    for _ in range(200):
        qs.append(rng.choice(w.n, int(rng.integers(1, 7)), replace=False).astype(np.int32))
    order = rng.permutation(len(qs))
    return [qs[i] for i in order]


def test_derived_tables_equal_counted_ones():
    """Tables summed out of a superset's table (derive_tables) equal the
    oracle's and those counted from the instances, in dense and caller-offset
    layouts, with reducers and in a replayed graph."""
    w = synth.batched_uneven(m=90_007, nq=2)
    rng = np.random.default_rng(11)
    qs = _nested_queries(w, rng)
    flat, off = synth.flatten(qs)
    wq = synth.Workload("nested", w.D, w.arity, flat, off)
    print("derived tables: %d queries" % wq.nq, flush=True)
    with Database(w.D, w.arity) as db:
        summ = db.plan_summary(qs)
        assert summ["derived"] >= 200 and sum(summ.values()) == wq.nq, summ
        tables, toff = db.count_batch(qs)
        check_tables(wq, tables, toff)
        # caller offsets with gaps between the tables
        gap = np.zeros(wq.nq + 1, np.int64)
        gap[1:] = np.cumsum(np.diff(toff) + 3)
        t2, _ = db.count_batch(qs, table_off=gap)
        T2 = t2.cpu().numpy()
        for i in range(wq.nq):
            np.testing.assert_array_equal(T2[gap[i]:gap[i] + toff[i + 1] - toff[i]],
                                          tables[toff[i]:toff[i + 1]].cpu().numpy())
        sc_on, _, tab_on, _ = db.count_reduce(qs, ("bdeu", "mi"), keep_tables=True)
        g = db.graph(qs, ("bdeu", "mi"))
        for _ in range(3):
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(g.scores[:2 * wq.nq], torch.cat([sc_on["bdeu"], sc_on["mi"]]))
        g.close()
        t = db.tuning()
        t["derive_tables"] = 0
        db.set_tuning(t)
        assert db.plan_summary(qs)["derived"] == 0
        sc_off, _, tab_off, _ = db.count_reduce(qs, ("bdeu", "mi"), keep_tables=True)
        assert torch.equal(tab_on, tab_off)
        for r in ("bdeu", "mi"):
            assert torch.equal(sc_on[r], sc_off[r])


@pytest.mark.parametrize("persistent", [0, 100000])
def test_persistent_and_solo_launches_agree(persistent):
    w = synth.batched_uneven(m=50_001, nq=300)
    with Database(w.D, w.arity) as db:
        t = db.tuning()
        t["persistent_max_queries"] = persistent
        db.set_tuning(t)
        for strategy in ("auto", "hist", "bitmap"):
            tables, toff = db.count_batch((w.vars_flat, w.var_off), strategy=strategy)
            check_tables(w, tables, toff)


def test_graph_replays_match_eager():
    # replays interleaved with eager work, every replay checked
    w = synth.bn_family(m=60_000, nq=250)
    with Database(w.D, w.arity) as db:
        g = db.graph((w.vars_flat, w.var_off), ("mdl", "bdeu"), keep_tables=True)
        eager, _, tables, toff = db.count_reduce((w.vars_flat, w.var_off), ("mdl", "bdeu"),
                                                 keep_tables=True)
        torch.cuda.synchronize()
        for rep in range(4):
            g.replay()
            other, _, _, _ = db.count_reduce([w.query(rep)], ("mdl",))   # eager work between
            torch.cuda.synchronize()
            res = g.result()
            for name in ("mdl", "bdeu"):
                assert torch.equal(res[name], eager[name]), (rep, name)
            assert torch.equal(g.tables, tables)
        check_tables(w, g.tables, toff, idx=range(0, w.nq, 5))
        g.close()


@pytest.mark.parametrize("packed", [0, 1])
def test_packed_and_byte_columns_agree(packed):
    # arities up to 16 (packed columns exist); tables of every histogram class
    rng = synth.rng_for(91)
    n, m = 12, 70_001                                   # ragged tail
    ar = rng.integers(2, 17, size=n).astype(np.uint8)
    ar[0] = 16
    D = np.stack([rng.integers(0, a, size=m) for a in ar]).astype(np.uint8)
    qs = [rng.choice(n, size=k, replace=False).astype(np.int32)
          for k in (1, 2, 2, 3, 3, 3, 4, 4, 5, 6) for _ in range(6)]
    w = synth.Workload("packed-check", D, ar, *synth.flatten(qs), ())
    print("packed=%d cells=%s" % (packed, sorted(int(np.prod(ar[q].astype(np.int64))) for q in qs)[-5:]),
          flush=True)
    with Database(D, ar) as db:
        t = db.tuning()
        t["packed_columns"] = packed
        t["persistent_max_queries"] = 0
        db.set_tuning(t)
        tables, toff = db.count_batch((w.vars_flat, w.var_off), strategy="hist")
        check_tables(w, tables, toff)
        tables, toff = db.count_batch((w.vars_flat, w.var_off), strategy="auto")
        check_tables(w, tables, toff)


# tables whose cell counts sit on both sides of every size-class boundary of
# the histogram kernels (16, 64, 256, 1024, 4096, 16383, 40000 cells)
_BOUNDARY_QUERIES = {
    16: [4, 4], 18: [2, 9], 64: [4, 16], 65: [5, 13], 256: [16, 16], 260: [4, 5, 13],
    1024: [4, 16, 16], 1050: [2, 3, 5, 5, 7], 4096: [16, 16, 16], 4116: [4, 3, 7, 7, 7],
    16380: [4, 9, 5, 7, 13], 16384: [4, 16, 16, 16], 40000: [16, 4, 5, 5, 5, 5],
    40960: [16, 16, 16, 10], 256 * 256: [16, 16, 16, 16],
}


@pytest.mark.parametrize("packed", [0, 1])
def test_size_class_boundaries(packed):
    # one variable per needed arity (repeated arities get several variables),
    # k = 8 queries of binary variables too
    need = {}
    for ars in _BOUNDARY_QUERIES.values():
        for a in set(ars):
            need[a] = max(need.get(a, 0), ars.count(a))
    arity = []
    first = {}
    for a in sorted(need):
        first[a] = len(arity)
        arity += [a] * need[a]
    arity += [2] * 8
    ar = np.array(arity, np.uint8)
    rng = synth.rng_for(93)
    m = 50_003
    D = np.stack([rng.integers(0, a, size=m) for a in ar]).astype(np.uint8)
    qs = []
    for cells, ars in _BOUNDARY_QUERIES.items():
        used = {}
        q = []
        for a in ars:
            q.append(first[a] + used.get(a, 0))
            used[a] = used.get(a, 0) + 1
        assert int(np.prod(ar[q].astype(np.int64))) == cells
        qs.append(np.array(q, np.int32))
        qs.append(np.array(q[::-1], np.int32))
    nb = len(arity) - 8
    qs.append(np.arange(nb, nb + 8, dtype=np.int32))            # k = 8, 256 cells
    qs.append(np.array([first[3], first[5]] + list(range(nb, nb + 6)), np.int32))
    w = synth.Workload("boundaries", D, ar, *synth.flatten(qs), ())
    print("packed=%d queries=%d" % (packed, len(qs)), flush=True)
    with Database(D, ar) as db:
        t = db.tuning()
        t["packed_columns"] = packed
        db.set_tuning(t)
        for strategy in ("hist", "auto"):
            tables, toff = db.count_batch((w.vars_flat, w.var_off), strategy=strategy)
            check_tables(w, tables, toff)


def test_empty_batches():
    w = synth.plain_small(m=2000, nq=5)
    with Database(w.D, w.arity) as db:
        tables, toff = db.count_batch([])
        assert len(toff) == 1 and toff[0] == 0
        scores, _, _, _ = db.count_reduce([], ("mdl", "mi"))
        assert all(v.numel() == 0 for v in scores.values())


def test_arity_above_16_uses_byte_columns():
    rng = synth.rng_for(92)
    ar = np.array([17, 3, 20, 2, 5], np.uint8)
    D = np.stack([rng.integers(0, a, size=20_000) for a in ar]).astype(np.uint8)
    qs = [np.array(q, np.int32) for q in ([0], [0, 1], [2, 3, 4], [1, 2], [4, 3, 1, 0])]
    w = synth.Workload("byte-check", D, ar, *synth.flatten(qs), ())
    with Database(D, ar) as db:
        tables, toff = db.count_batch((w.vars_flat, w.var_off), strategy="hist")
        check_tables(w, tables, toff)


def test_tuning_roundtrip_and_validation():
    w = synth.plain_small()
    with Database(w.D, w.arity) as db:
        t = db.tuning()
        t["chunk_rows"] = 32768
        t["bitmap_cells"][2][3] = 1
        db.set_tuning(t)
        assert db.tuning() == t
        t["packed_columns"] = 0
        db.set_tuning(t)
        assert db.tuning() == t
        t["bitmap_words"] = 3
        with pytest.raises(_lib.FastcountError):
            db.set_tuning(t)
        t["bitmap_words"] = 2
        t["packed_columns"] = 2
        with pytest.raises(_lib.FastcountError):
            db.set_tuning(t)


def test_incremental_appends():
    w = synth.batched_uneven(m=30_011, nq=120)
    parts = [(0, 4000), (4000, 4100), (4100, 9000), (9000, 30_011)]   # in-tile and tile-crossing
    qs = (w.vars_flat, w.var_off)
    with Database(np.ascontiguousarray(w.D[:, :4000]), w.arity) as db:
        for lo, hi in parts[1:]:
            piece = np.ascontiguousarray(w.D[:, lo:hi])
            if hi - lo > 1000:
                db.append(np.ascontiguousarray(piece.T), layout="row")
            else:
                db.append(piece)
        assert db.info()[0] == w.m
        for strategy in ("auto", "bitmap", "hist"):
            tables, toff = db.count_batch(qs, strategy=strategy)
            check_tables(w, tables, toff)
        cnt, _ = db.marginals()
        off = 0
        for v in range(w.n):
            ref = np.bincount(w.D[v], minlength=w.arity[v])
            got = cnt[off:off + int(w.arity[v])]
            assert np.array_equal(got, ref), (v, got.tolist(), ref.tolist())
            off += int(w.arity[v])
        assert db.count_assignment([0, 1], [1, 0]) == orc.count_assignment(w.D, w.arity, [0, 1], [1, 0])


def test_rejected_append_changes_nothing_and_graphs_expire():
    w = synth.plain_small(m=6000, nq=60)
    with Database(w.D, w.arity) as db:
        g = db.graph((w.vars_flat, w.var_off), ("mdl",))
        bad = np.zeros((w.n, 10), np.uint8)
        bad[0, 3] = w.arity[0]                                # state == arity
        with pytest.raises(_lib.FastcountError):
            db.append(bad)
        assert db.info()[0] == w.m
        tables, toff = db.count_batch((w.vars_flat, w.var_off))
        check_tables(w, tables, toff)
        g.replay()                                            # still valid
        db.append(np.zeros((w.n, 5), np.uint8))
        with pytest.raises(_lib.FastcountError):
            g.replay()                                        # captured before the append
        g.close()


def test_concurrent_host_threads_on_separate_streams():
    # the ABI allows concurrent calls on one database from several host
    # threads, each on its own stream; every result equals the serial one
    import threading
    w = synth.batched_uneven(m=40_009, nq=600)
    with Database(w.D, w.arity) as db:
        parts = [(w.vars_flat[w.var_off[a]:w.var_off[b]], w.var_off[a:b + 1] - w.var_off[a])
                 for a, b in ((0, 150), (150, 300), (300, 450), (450, 600))]
        ref = []
        for flat, off in parts:
            sc, _, tables, _ = db.count_reduce((flat, off), ("bdeu", "mi"), keep_tables=True)
            torch.cuda.synchronize()
            ref.append((sc["bdeu"].cpu(), sc["mi"].cpu(), tables.cpu()))
        got = [None] * len(parts)
        errors = []

        def run(i):
            try:
                s = torch.cuda.Stream()
                with torch.cuda.stream(s):
                    for _ in range(5):
                        sc, _, tables, _ = db.count_reduce(parts[i], ("bdeu", "mi"),
                                                           keep_tables=True, stream=s)
                    s.synchronize()
                    got[i] = (sc["bdeu"].cpu(), sc["mi"].cpu(), tables.cpu())
            except Exception as e:      # reported in the main thread
                errors.append(e)

        th = [threading.Thread(target=run, args=(i,)) for i in range(len(parts))]
        for t in th:
            t.start()
        for t in th:
            t.join()
        assert not errors, errors
        for i in range(len(parts)):
            for a, b in zip(ref[i], got[i]):
                assert torch.equal(a, b), i


def test_appends_within_and_beyond_the_allocation():
    """Appends of uneven sizes (1 instance to several tiles): some fit the
    allocated pitch, some grow it. After every append each strategy, both
    column stores, batched single assignments, sparse tables and the
    reducers agree with the oracle on the data so far."""
    w = synth.bn_family(m=60_000, nq=150)
    D, ar = w.D, w.arity
    qs = (w.vars_flat, w.var_off)
    # pitch (rows allocated per column) after each append: 4096, 4096, 8192, 8192, 12288,
    # 12288, 32768, 32768, 49152 (grown 1.5x), 49152, 49152 (the scanned extent grows
    # inside it), 49152, 73728
    cuts = [3000, 3001, 8001, 8101, 12197, 12204, 32204, 32205, 32800, 33000, 41000, 45000,
            60_000]
    rng = np.random.default_rng(5)
    aq = [rng.choice(w.n, size=int(rng.integers(1, 5)), replace=False) for _ in range(40)]
    ast = [[int(rng.integers(0, ar[v])) for v in q] for q in aq]
    with Database(np.ascontiguousarray(D[:, :cuts[0]]), ar) as db:
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            db.append(np.ascontiguousarray(D[:, lo:hi]))
            sub = synth.Workload(w.name, np.ascontiguousarray(D[:, :hi]), ar, w.vars_flat,
                                 w.var_off, w.reducers)
            print("after append to m=%d" % hi, flush=True)
            for packed in (1, 0):
                t = db.tuning()
                t["packed_columns"] = packed
                db.set_tuning(t)
                for strategy in ("auto", "bitmap", "hist"):
                    tables, toff = db.count_batch(qs, strategy=strategy)
                    check_tables(sub, tables, toff)
            got = db.count_assignments(aq, ast)
            for q, s_, g in zip(aq, ast, got):
                assert g == orc.count_assignment(sub.D, ar, q, s_)
            keys, cnt, _ = db.count_sparse(w.query(3))
            rk, rc = orc.count_sparse(sub.D, ar, w.query(3))
            np.testing.assert_array_equal(keys, rk)
            np.testing.assert_array_equal(cnt, rc)
            sc, _, _, _ = db.count_reduce([w.query(0)], ("mdl",))
            ref = orc.score("mdl", orc.count(sub.D, ar, w.query(0)), int(ar[w.query(0)[-1]]), 1.0)
            assert abs(float(sc["mdl"][0]) - ref) <= 1e-6 * max(1.0, abs(ref))


def test_appends_then_pairs():
    """The all-pairs Gram on bit-vectors that grew through appends equals the
    oracle's co-occurrence counts."""
    rng = np.random.default_rng(12)
    n, m = 90, 50_001
    D = (rng.random((n, m)) < rng.random((n, 1)) * 0.3).astype(np.uint8)
    with Database(np.ascontiguousarray(D[:, :7000]), np.full(n, 2, np.uint8)) as db:
        for lo, hi in ((7000, 7001), (7001, 20_000), (20_000, 21_000), (21_000, 29_000), (29_000, m)):
            db.append(np.ascontiguousarray(D[:, lo:hi]))
            _, G, _ = db.pairs(0.01, gram=True)
            np.testing.assert_array_equal(G.cpu().numpy(), orc.gram(np.ascontiguousarray(D[:, :hi])))


def test_trim_releases_idle_workspaces():
    w = synth.batched_uneven(m=50_003, nq=400)
    with Database(w.D, w.arity) as db:
        base = db.info()[3]
        tables, toff = db.count_batch((w.vars_flat, w.var_off))
        sc, _, _, _ = db.count_reduce((w.vars_flat, w.var_off), ("bdeu",))
        db.count_sparse_batch([w.query(i) for i in range(50)])
        torch.cuda.synchronize()
        held = db.info()[3]
        assert held > base                      # plan, tables and sort scratch kept
        db.trim()
        assert db.info()[3] == base
        check_tables(w, *db.count_batch((w.vars_flat, w.var_off)))   # allocates again
        sc2, _, _, _ = db.count_reduce((w.vars_flat, w.var_off), ("bdeu",))
        assert torch.equal(sc["bdeu"], sc2["bdeu"])
        db.trim()
        db.trim()                               # nothing idle: no-op
        assert db.info()[3] == base


def test_empty_database_then_appends():
    """A database created with no instances answers every entry point, then
    grows by appends from empty (its first allocation is one tile)."""
    from paper_1804_04640_amd import arm
    rng = np.random.default_rng(17)
    ar = np.array([2, 3, 2, 4, 2], np.uint8)
    D = np.stack([rng.integers(0, a, size=30_011) for a in ar]).astype(np.uint8)
    with Database(np.zeros((5, 0), np.uint8), ar) as db:
        assert db.count([0, 3]).cpu().numpy().tolist() == [0] * 8
        keys, cnts, off = db.count_sparse_batch([[0, 1], [3]])
        assert len(keys) == 0 and list(off) == [0, 0, 0]
        assert db.count_assignments([[0, 2]], [[1, 1]]).tolist() == [0]
        freq, rules = arm.mine(db, minsup=0.0, minconf=0.0, items=[0, 2, 4])
        assert freq == {} and rules == []
        lo = 0
        for hi in (1, 4097, 9000, 30_011):
            db.append(np.ascontiguousarray(D[:, lo:hi]))
            lo = hi
            for vs in ([0, 3], [1, 2, 4], [3]):
                np.testing.assert_array_equal(db.count(vs).cpu().numpy(),
                                              orc.count(np.ascontiguousarray(D[:, :hi]), ar, vs))
        freq, _ = arm.mine(db, minsup=0.1, minconf=0.5, items=[0, 2, 4])
        ref, _ = orc.arm_bruteforce(D[[0, 2, 4]], 0.1, 0.5, max_size=6)
        assert freq == {tuple([0, 2, 4][i] for i in s): c for s, c in ref.items()}


def test_small_queries_from_state_gram():
    """A batch whose one- and two-variable queries outweigh the Gram of their
    variables' state bit-vectors (15,000 BN-family queries, m = 10^6) takes
    those tables from that Gram (automatic strategy; k_gram_states runs).
    Every small query's table equals the oracle's; all tables equal the
    forced histogram path's, packed and placed (reversed order with gaps);
    fused scores equal the forced path's bitwise; a captured graph replays
    to the same scores twice."""
    w = synth.bn_family()
    qs = w.queries()[:15000]
    small = [i for i, q in enumerate(qs) if len(q) <= 2]
    print("state gram: %d queries, %d small" % (len(qs), len(small)), flush=True)
    with Database(w.D, w.arity) as db:
        _lib.fc_profile_enable(True)
        _lib.fc_profile_read(reset=True)
        t_auto, toff = db.count_batch(qs)
        torch.cuda.synchronize()
        prof = _lib.fc_profile_read(reset=True)
        _lib.fc_profile_enable(False)
        assert "k_gram_states" in prof
        t_hist, toff2 = db.count_batch(qs, strategy="hist")
        assert np.array_equal(toff, toff2)
        A, H = t_auto.cpu().numpy(), t_hist.cpu().numpy()
        assert np.array_equal(A, H)
        for i in small:
            ref = orc.count(w.D, w.arity, qs[i])
            assert np.array_equal(A[toff[i]:toff[i] + len(ref)], ref), (i, list(qs[i]))
        cells = np.diff(toff)
        placed = np.zeros(len(qs) + 1, np.int64)
        pos = 0
        for i in reversed(range(len(qs))):
            placed[i] = pos
            pos += int(cells[i]) + 3
        placed[-1] = pos
        buf = torch.full((pos,), -7, dtype=torch.int32, device="cuda")
        db.count_batch(qs, tables=buf, table_off=placed)
        B = buf.cpu().numpy()
        for i in range(len(qs)):
            assert np.array_equal(B[placed[i]:placed[i] + cells[i]], A[toff[i]:toff[i + 1]]), i
        sa, _, _, _ = db.count_reduce(qs, ("mdl", "bdeu", "mi"))
        sh, _, _, _ = db.count_reduce(qs, ("mdl", "bdeu", "mi"), strategy="hist")
        for r in sa:
            assert torch.equal(sa[r], sh[r]), r
        g = db.graph(qs, ("mdl",))
        for _ in range(2):
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(g.result()["mdl"], sa["mdl"])
        g.close()


def test_state_gram_ragged_and_after_appends():
    """The state-Gram path at m = 10^6 + 37 (a ragged last 64-instance word)
    and on a handle built from the first 600,011 instances with the rest
    appended: every small query's table equals the oracle's, and the
    appended handle's tables equal the fresh handle's."""
    w = synth.bn_family(m=1_000_037, nq=15000)
    qs = w.queries()
    small = [i for i, q in enumerate(qs) if len(q) <= 2]
    with Database(w.D, w.arity) as db:
        _lib.fc_profile_enable(True)
        _lib.fc_profile_read(reset=True)
        t_fresh, toff = db.count_batch(qs)
        torch.cuda.synchronize()
        prof = _lib.fc_profile_read(reset=True)
        _lib.fc_profile_enable(False)
        assert "k_gram_states" in prof
        A = t_fresh.cpu().numpy()
    for i in small:
        ref = orc.count(w.D, w.arity, qs[i])
        assert np.array_equal(A[toff[i]:toff[i] + len(ref)], ref), (i, list(qs[i]))
    m0 = 600_011
    with Database(np.ascontiguousarray(w.D[:, :m0]), w.arity) as db:
        db.append(np.ascontiguousarray(w.D[:, m0:]))
        t_app, toff2 = db.count_batch(qs)
        assert np.array_equal(toff, toff2)
        assert np.array_equal(t_app.cpu().numpy(), A)


def test_state_gram_edge_arities():
    """The state-Gram path with single-state and 255-state variables (689
    states: three 256-row blocks of the Gram), 30,000 one- and two-variable
    queries at m = 2^18 + 3: every table equals the oracle's, including the
    one-cell tables of single-state variables and tables of 65,025 cells."""
    rng = synth.rng_for(97)
    m = (1 << 18) + 3
    ar = np.concatenate([rng.integers(1, 5, size=20), [255, 255, 128]]).astype(np.uint8)
    ar[:2] = 1
    n = len(ar)
    D = np.stack([rng.integers(0, a, size=m) for a in ar]).astype(np.uint8)
    qs = [rng.choice(n, size=int(rng.integers(1, 3)), replace=False).astype(np.int32)
          for _ in range(30000)]
    qs += [np.array([0], np.int32), np.array([1, 20], np.int32), np.array([20, 21], np.int32)]
    with Database(D, ar) as db:
        _lib.fc_profile_enable(True)
        _lib.fc_profile_read(reset=True)
        t, toff = db.count_batch(qs)
        torch.cuda.synchronize()
        prof = _lib.fc_profile_read(reset=True)
        _lib.fc_profile_enable(False)
        assert "k_gram_states" in prof
        T = t.cpu().numpy()
    for i, q in enumerate(qs):
        ref = orc.count(D, ar, q)
        assert np.array_equal(T[toff[i]:toff[i] + len(ref)], ref), (i, list(q))
