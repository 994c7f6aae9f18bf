"""Admission, merging, cancellation and failure isolation of the request
loop, driven on the CPU through a fake backend (no device work)."""
import numpy as np
import pytest

from paper_1804_04640_amd.serving import CountServer, Request, merge, poisson_arrivals, run_load


class FakeBackend:
    """Each launch finishes after `delay` polls; a query's 'score' is the sum
    of its variable ids, so splitting errors are visible."""

    def __init__(self, slots=2, delay=2, bytes_per_query=100):
        self.slots = slots
        self.delay = delay
        self.bpq = bytes_per_query
        self.launched = []          # list of (slot, nq)
        self.live = {}

    def footprint(self, flat, off):
        if np.any(flat < 0):
            raise ValueError("query has a negative variable")
        return self.bpq * (len(off) - 1)

    def launch(self, slot, flat, off):
        h = object()
        self.live[h] = [self.delay, flat.copy(), off.copy()]
        self.launched.append((slot, len(off) - 1))
        return h

    def ready(self, h):
        self.live[h][0] -= 1
        return self.live[h][0] <= 0

    def result(self, h, nq):
        _, flat, off = self.live.pop(h)
        return np.array([[flat[off[i]:off[i + 1]].sum() for i in range(nq)]], np.float32)


def req(rid, queries):
    flat = np.concatenate([np.asarray(q, np.int32) for q in queries])
    off = np.zeros(len(queries) + 1, np.int64)
    off[1:] = np.cumsum([len(q) for q in queries])
    return Request(rid, flat, off, arrival=0.0)


def expected(queries):
    return np.array([sum(q) for q in queries], np.float32)


def test_merge_offsets():
    a, b = req(0, [[1, 2], [3]]), req(1, [[4, 5, 6]])
    flat, off = merge([a, b])
    assert flat.tolist() == [1, 2, 3, 4, 5, 6] and off.tolist() == [0, 2, 3, 6]


def test_requests_merge_and_results_split():
    be = FakeBackend(slots=1, delay=1)
    srv = CountServer(be, mem_budget=10_000)
    qs = {i: [[i, i + 1], [i + 2]] for i in range(5)}
    for i in range(5):
        srv.submit(req(i, qs[i]))
    done = srv.drain()
    assert len(be.launched) == 1 and be.launched[0][1] == 10      # one merged launch
    for r in done:
        np.testing.assert_array_equal(r.scores[0], expected(qs[r.rid]))


def test_memory_budget_is_never_exceeded_and_nothing_fails():
    be = FakeBackend(slots=4, delay=3, bytes_per_query=100)
    srv = CountServer(be, mem_budget=350)                          # 3 queries at a time
    for i in range(12):
        srv.submit(req(i, [[i]]))
    done, peak = [], 0
    while not srv.idle():
        done.extend(srv.poll())
        peak = max(peak, srv.mem_used)
    assert peak <= 350 and len(done) == 12
    assert all(r.error is None for r in done)
    assert [r.rid for r in sorted(done, key=lambda r: r.admitted)] == sorted(r.rid for r in done)


def test_oversized_and_invalid_requests_fail_alone():
    be = FakeBackend(slots=2, delay=1, bytes_per_query=100)
    srv = CountServer(be, mem_budget=250)
    srv.submit(req(0, [[1], [2], [3]]))        # 300 bytes > budget: rejected
    srv.submit(req(1, [[-1, 2]]))              # invalid: rejected
    srv.submit(req(2, [[7], [8]]))             # fine
    done = {r.rid: r for r in srv.drain()}
    assert done[0].error and "budget" in done[0].error
    assert done[1].error and "negative" in done[1].error
    assert done[2].error is None
    np.testing.assert_array_equal(done[2].scores[0], [7, 8])


def test_cancel_before_admission():
    be = FakeBackend(slots=1, delay=5)
    srv = CountServer(be, mem_budget=100)      # one query at a time
    for i in range(3):
        srv.submit(req(i, [[i]]))
    srv.poll()                                 # admits request 0 only
    assert srv.cancel(2) and not srv.cancel(0)
    done = {r.rid: r for r in srv.drain()}
    assert set(done) == {0, 1}


def test_run_load_with_poisson_arrivals():
    be = FakeBackend(slots=2, delay=1)
    srv = CountServer(be, mem_budget=1 << 20)
    rng = np.random.default_rng(0)
    batches = []
    for i in range(50):
        r = req(i, [[i % 7, 3]] * int(rng.integers(1, 5)))
        batches.append((r.flat, r.off))
    arr = poisson_arrivals(rng, 5000.0, len(batches))
    st = run_load(srv, batches, arr)
    assert st["requests"] == 50 and st["failed"] == 0
    assert st["p99_ms"] >= st["p50_ms"] >= 0.0


class MergedCostBackend(FakeBackend):
    """A batch of several requests costs more than its parts (as when the
    planner picks another path for a merged batch); records, for every
    launch, the footprint of exactly the batch launched."""

    def __init__(self, **kw):
        super().__init__(**kw)
        self.live_bytes = {}
        self.peak = 0

    def footprint(self, flat, off):
        nq = len(off) - 1
        return super().footprint(flat, off) + (150 if nq > 1 else 0)

    def launch(self, slot, flat, off):
        h = super().launch(slot, flat, off)
        self.live_bytes[h] = self.footprint(flat, off)
        self.peak = max(self.peak, sum(self.live_bytes.values()))
        return h

    def result(self, h, nq):
        self.live_bytes.pop(h)
        return super().result(h, nq)


def test_merged_footprint_is_admitted_not_the_sum_of_requests():
    be = MergedCostBackend(slots=4, delay=3, bytes_per_query=100)
    srv = CountServer(be, mem_budget=400)
    qs = {i: [[i]] for i in range(10)}
    for i in range(10):
        srv.submit(req(i, qs[i]))
    done = []
    while not srv.idle():
        done.extend(srv.poll())
        assert srv.mem_used <= 400
    # the device figure of what was really in flight never passed the budget
    assert be.peak <= 400
    assert len(done) == 10 and all(r.error is None for r in done)
    for r in done:
        np.testing.assert_array_equal(r.scores[0], expected(qs[r.rid]))
