"""fc_count_reduce_noalloc (the entry point for callers that cannot
allocate) against fc_count_reduce, both called through the C ABI: bitwise
equal scores and error estimates on two calls in a row, the second with a
smaller batch, then the refusals of oversized batches and host outputs."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1804_04640_amd import _lib, synth
from paper_1804_04640_amd.api import Database

pytestmark = pytest.mark.gpu

MASK = _lib.FC_RED_BDEU | _lib.FC_RED_MI | _lib.FC_RED_MDL | _lib.FC_RED_LL


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _both(db, flat, off, ess=1.0):
    """Scores and error estimates of one batch from fc_count_reduce (tables
    consumed) and from fc_count_reduce_noalloc, on one stream."""
    nq = len(off) - 1
    params = _lib.fc_reduce_params(float(ess))
    s = torch.cuda.current_stream().cuda_stream
    out = []
    for fn in ("ref", "noalloc"):
        sc = torch.full((4 * nq,), float("nan"), dtype=torch.float32, device="cuda")
        er = torch.full((4 * nq,), float("nan"), dtype=torch.float32, device="cuda")
        if fn == "ref":
            _lib.fc_count_reduce(db.handle, _ptr(flat), _ptr(off), nq, MASK,
                                 ctypes.addressof(params), sc.data_ptr(), er.data_ptr(),
                                 None, None, 0, s)
        else:
            _lib.fc_count_reduce_noalloc(db.handle, _ptr(flat), _ptr(off), nq, MASK,
                                         ctypes.addressof(params), sc.data_ptr(), er.data_ptr(),
                                         0, s)
        out.append((sc, er))
    torch.cuda.synchronize()
    (a, ea), (b, eb) = out
    return a.cpu().numpy(), ea.cpu().numpy(), b.cpu().numpy(), eb.cpu().numpy()


def _check_same(a, ea, b, eb):
    assert not np.isnan(a).any()
    np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))
    np.testing.assert_array_equal(ea.view(np.uint32), eb.view(np.uint32))


def test_noalloc_matches_count_reduce_on_two_calls():
    w = synth.batched_uneven(m=300_007, nq=3000)
    print("no-alloc: batched-uneven m=%d, %d then 700 queries" % (w.m, w.nq), flush=True)
    with Database(w.D, w.arity) as db:
        flat, off = w.vars_flat, w.var_off
        _check_same(*_both(db, flat, off))
        # a smaller batch next: other queries, fewer cells than the first
        # call left in the scratch
        sub = np.arange(2100, 2800)
        qs = [w.query(int(i))[::-1].copy() for i in sub]
        off2 = np.zeros(len(qs) + 1, np.int64)
        off2[1:] = np.cumsum([len(q) for q in qs])
        flat2 = np.concatenate(qs).astype(np.int32)
        _check_same(*_both(db, flat2, off2))


def test_noalloc_refuses_oversized_batches_and_host_outputs():
    w = synth.batched_uneven(m=50_001, nq=400)
    print("no-alloc refusals: m=%d" % w.m, flush=True)
    with Database(w.D, w.arity) as db:
        order = np.argsort(w.arity)[::-1]
        big = order[:6].astype(np.int32)                 # the largest table there is
        cells = int(np.prod(w.arity[big].astype(np.int64)))
        reps = (64 << 20) // (4 * cells) + 2             # more cells than the scratch holds
        flat = np.tile(big, reps).astype(np.int32)
        off = np.arange(0, len(flat) + 1, len(big), dtype=np.int64)
        nq = reps
        params = _lib.fc_reduce_params(1.0)
        s = torch.cuda.current_stream().cuda_stream
        sc = torch.empty(4 * nq, dtype=torch.float32, device="cuda")
        with pytest.raises(_lib.FastcountError) as e:
            _lib.fc_count_reduce_noalloc(db.handle, _ptr(flat), _ptr(off), nq, MASK,
                                         ctypes.addressof(params), sc.data_ptr(), None, 0, s)
        assert e.value.code == _lib.FC_ERR_RANGE and "scratch" in str(e.value)
        host = np.zeros(4 * w.nq, np.float32)
        with pytest.raises(_lib.FastcountError) as e:
            _lib.fc_count_reduce_noalloc(db.handle, _ptr(w.vars_flat), _ptr(w.var_off), w.nq,
                                         MASK, ctypes.addressof(params), _ptr(host), None, 0, s)
        assert e.value.code == _lib.FC_ERR_INVALID
        # the handle still answers after the refusals
        _check_same(*_both(db, w.vars_flat, w.var_off))
