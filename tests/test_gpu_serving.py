"""GPU request loop: merged results equal results alone, bit for bit;
memory-limited admission completes everything; bad requests fail alone."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1804_04640_amd import synth
from paper_1804_04640_amd.api import Database
from paper_1804_04640_amd.serving import (CountServer, GpuBackend, PerQueryServer, Request,
                                          poisson_arrivals, run_load)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def served():
    w = synth.serving(m=200_003, nbatches=12)
    db = Database(w.D, w.arity)
    yield w, db
    db.close()


def requests(w):
    out = []
    for i, ids in enumerate(w.batches):
        qs = [w.query(int(j)) for j in ids]
        flat = np.concatenate(qs).astype(np.int32)
        off = np.zeros(len(qs) + 1, np.int64)
        off[1:] = np.cumsum([len(q) for q in qs])
        out.append(Request(i, flat, off, arrival=0.0))
    return out


def test_mix_equals_alone_bit_for_bit(served):
    w, db = served
    be = GpuBackend(db, ("mdl", "bdeu"), slots=2)
    srv = CountServer(be, mem_budget=1 << 34)
    reqs = requests(w)
    for r in reqs:
        srv.submit(r)
    done = {r.rid: r for r in srv.drain()}
    assert srv.launches < len(reqs)            # requests were merged
    for r in reqs:
        alone, _, _, _ = db.count_reduce((r.flat, r.off), ("mdl", "bdeu"), with_err=False)
        torch.cuda.synchronize()
        got = done[r.rid].scores
        np.testing.assert_array_equal(got[0], alone["mdl"].cpu().numpy())
        np.testing.assert_array_equal(got[1], alone["bdeu"].cpu().numpy())
    # and the scores are right
    r = reqs[0]
    for i in range(0, r.nq, max(1, r.nq // 25)):
        q = r.flat[r.off[i]:r.off[i + 1]]
        T = orc.count(w.D, w.arity, q)
        ref = orc.mdl(T, int(w.arity[q[-1]]))
        assert abs(float(done[0].scores[0, i]) - ref) <= 1e-6 * abs(ref)


class _MeasuredBackend(GpuBackend):
    """Records the library's own device footprint of every batch it launches
    (the merged batch as launched, not the sum of its requests) and the
    largest total in flight."""

    def __init__(self, *a, **kw):
        super().__init__(*a, **kw)
        self.live, self.peak = {}, 0

    def launch(self, slot, flat, off):
        h = super().launch(slot, flat, off)
        self.live[id(h)] = self.footprint(flat, off)
        self.peak = max(self.peak, sum(self.live.values()))
        return h

    def result(self, handle, nq):
        self.live.pop(id(handle))
        return super().result(handle, nq)


def test_memory_limited_admission(served):
    w, db = served
    be = _MeasuredBackend(db, ("mdl",), slots=4)
    reqs = requests(w)
    biggest = max(be.footprint(r.flat, r.off) for r in reqs)
    srv = CountServer(be, mem_budget=int(biggest * 1.2))
    for r in reqs:
        srv.submit(r)
    peak, done = 0, []
    while not srv.idle():
        done.extend(srv.poll())
        peak = max(peak, srv.mem_used)
    assert len(done) == len(reqs) and all(r.error is None for r in done)
    assert peak <= srv.mem_budget
    assert be.peak <= srv.mem_budget


def test_per_query_server_with_two_reducers(served):
    """The plain per-query path gives every reducer of every query the
    batched path's score."""
    w, db = served
    r = max(requests(w), key=lambda x: x.nq)
    n = min(40, r.nq)
    r = Request(0, r.flat[:r.off[n]].copy(), r.off[:n + 1].copy(), arrival=0.0)
    srv = PerQueryServer(db, ("mdl", "bdeu"))
    srv.submit(r)
    got = srv.poll()[0].scores
    alone, _, _, _ = db.count_reduce((r.flat, r.off), ("mdl", "bdeu"), with_err=False)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got[0], alone["mdl"].cpu().numpy())
    np.testing.assert_array_equal(got[1], alone["bdeu"].cpu().numpy())


def test_bad_request_fails_alone(served):
    w, db = served
    be = GpuBackend(db, ("mdl",), slots=2)
    srv = CountServer(be, mem_budget=1 << 34)
    reqs = requests(w)[:4]
    bad = Request(99, np.array([0, 0], np.int32), np.array([0, 2], np.int64), arrival=0.0)
    srv.submit(reqs[0])
    srv.submit(bad)
    for r in reqs[1:]:
        srv.submit(r)
    done = {r.rid: r for r in srv.drain()}
    assert done[99].error and "twice" in done[99].error
    assert all(done[r.rid].error is None for r in reqs)


def test_poisson_load_smoke(served):
    w, db = served
    be = GpuBackend(db, ("mdl",), slots=4)
    srv = CountServer(be, mem_budget=1 << 34)
    reqs = requests(w)
    batches = [(r.flat, r.off) for r in reqs] * 4
    st = run_load(srv, batches, poisson_arrivals(np.random.default_rng(1), 400.0, len(batches)))
    assert st["failed"] == 0 and st["requests"] == len(batches)
