"""Continuous-batching request loop over a database resident on the GPU.

A structure-search driver (or any client) submits requests, each a batch of
family queries to be counted and scored.  The server keeps the database
resident and, on every tick:

1. retires finished device batches (a HIP event per batch), hands each
   request its scores and frees its slot and memory;
2. admits waiting requests in arrival order while a slot (a HIP stream) is
   free and their device footprint (fc_batch_footprint) fits the memory
   budget; every request admitted in one tick is merged into one device
   batch, so requests that arrived while others were on the GPU ride the next
   launch, and batches on different slots overlap on the device.

Counts are exact and every table's score is reduced in an order that depends
on that table alone, so a request's scores are bit-identical whether it ran
alone or merged with others.  A request that the library rejects (an invalid
query) fails alone; a request larger than the whole budget is rejected;
pending requests can be cancelled.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    flat: np.ndarray                  # int32 variables, child last per query
    off: np.ndarray                   # int64 [nq+1]
    arrival: float                    # perf_counter() time of arrival
    admitted: Optional[float] = None
    done: Optional[float] = None
    scores: Optional[np.ndarray] = None   # float32 [n_reducers, nq]
    error: Optional[str] = None
    cancelled: bool = False

    @property
    def nq(self) -> int:
        return len(self.off) - 1

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


def merge(reqs: Sequence[Request]):
    """Concatenate the requests' queries into one flat batch."""
    flats = [r.flat for r in reqs]
    offs, base = [np.zeros(1, np.int64)], 0
    for r in reqs:
        offs.append(r.off[1:] + base)
        base += int(r.off[-1])
    return (np.concatenate(flats).astype(np.int32) if flats else np.zeros(0, np.int32),
            np.concatenate(offs).astype(np.int64))


class GpuBackend:
    """Launches merged batches with fc_count_reduce on per-slot HIP streams."""

    def __init__(self, db, reducers=("mdl",), ess: float = 1.0, slots: int = 4):
        import torch
        self.torch = torch
        self.db = db
        self.reducers = tuple(reducers)
        self.ess = ess
        self.streams = [torch.cuda.Stream(device=db.device) for _ in range(slots)]

    @property
    def slots(self) -> int:
        return len(self.streams)

    def footprint(self, flat, off) -> int:
        nq = len(off) - 1
        return int(self.db.footprint((flat, off))) + 8 * len(self.reducers) * nq

    def launch(self, slot: int, flat, off):
        torch = self.torch
        s = self.streams[slot]
        nq = len(off) - 1
        with torch.cuda.stream(s):
            dev = torch.empty(len(self.reducers) * nq, dtype=torch.float32, device=self.db.device)
            self.db.count_reduce((flat, off), self.reducers, ess=self.ess, out=dev,
                                 with_err=False, stream=s)
            host = torch.empty(dev.shape, dtype=torch.float32, pin_memory=True)
            host.copy_(dev, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, host, dev)

    def ready(self, handle) -> bool:
        return handle[0].query()

    def result(self, handle, nq: int) -> np.ndarray:
        handle[0].synchronize()
        return handle[1].numpy().reshape(len(self.reducers), nq).copy()


@dataclasses.dataclass
class _Flight:
    slot: int
    reqs: List[Request]
    handle: object
    nbytes: int
    nq: int


class CountServer:
    def __init__(self, backend, mem_budget: int, max_merge_queries: int = 32768,
                 clock: Callable[[], float] = time.perf_counter):
        self.backend = backend
        self.mem_budget = int(mem_budget)
        self.max_merge = int(max_merge_queries)
        self.clock = clock
        self.pending: collections.deque = collections.deque()
        self.inflight: List[_Flight] = []
        self.free_slots = list(range(backend.slots))
        self.mem_used = 0
        self.launches = 0

    # ---------------------------------------------------------------- client
    def submit(self, req: Request) -> None:
        self.pending.append(req)

    def cancel(self, rid: int) -> bool:
        """Cancel a request that has not been admitted yet."""
        for r in list(self.pending):
            if r.rid == rid:
                self.pending.remove(r)
                r.cancelled = True
                r.done = self.clock()
                return True
        return False

    def idle(self) -> bool:
        return not self.pending and not self.inflight

    # ---------------------------------------------------------------- loop
    def poll(self) -> List[Request]:
        """One tick: retire finished batches, then admit and launch.  Returns
        the requests completed (or failed) during this tick."""
        out: List[Request] = []
        for f in list(self.inflight):
            if self.backend.ready(f.handle):
                out.extend(self._retire(f))
        out.extend(self._admit())
        return out

    def drain(self, timeout: float = 60.0) -> List[Request]:
        out, t0 = [], self.clock()
        while not self.idle():
            out.extend(self.poll())
            if self.clock() - t0 > timeout:
                raise TimeoutError("server did not drain in %.1fs" % timeout)
        return out

    def _retire(self, f: _Flight) -> List[Request]:
        res = self.backend.result(f.handle, f.nq)
        now = self.clock()
        base = 0
        for r in f.reqs:
            r.scores = res[:, base:base + r.nq]
            base += r.nq
            r.done = now
        self.inflight.remove(f)
        self.free_slots.append(f.slot)
        self.mem_used -= f.nbytes
        return f.reqs

    def _admit(self) -> List[Request]:
        failed: List[Request] = []
        while self.pending and self.free_slots:
            group: List[Request] = []
            nbytes, nq = 0, 0
            while self.pending:
                r = self.pending[0]
                try:
                    need = self.backend.footprint(r.flat, r.off)
                except Exception as e:          # invalid request: fails alone
                    self.pending.popleft()
                    r.error, r.done = str(e), self.clock()
                    failed.append(r)
                    continue
                if need > self.mem_budget:      # can never fit
                    self.pending.popleft()
                    r.error = "request needs %d bytes, budget is %d" % (need, self.mem_budget)
                    r.done = self.clock()
                    failed.append(r)
                    continue
                if group and (nq + r.nq > self.max_merge):
                    break
                if self.mem_used + nbytes + need > self.mem_budget:
                    break                       # wait for memory to free up
                group.append(self.pending.popleft())
                nbytes += need
                nq += r.nq
            if not group:
                break
            flat, off = merge(group)
            if len(group) > 1:
                # a merged batch's footprint is not the sum of its requests'
                # (the plan may take another path for the whole batch): admit
                # what the merged figure lets fit, return the rest
                try:
                    merged = self.backend.footprint(flat, off)
                except Exception:
                    merged = nbytes
                while len(group) > 1 and self.mem_used + merged > self.mem_budget:
                    r = group.pop()
                    self.pending.appendleft(r)
                    nq -= r.nq
                    flat, off = merge(group)
                    merged = self.backend.footprint(flat, off)
                if self.mem_used + merged > self.mem_budget:
                    self.pending.appendleft(group.pop())
                    break                       # wait for memory to free up
                nbytes = merged
            slot = self.free_slots.pop()
            now = self.clock()
            try:
                handle = self.backend.launch(slot, flat, off)
            except Exception as e:
                # the library validates a batch before any launch; retry the
                # merged requests one by one so a bad one fails alone
                self.free_slots.append(slot)
                if len(group) == 1:
                    group[0].error, group[0].done = str(e), self.clock()
                    failed.append(group[0])
                else:
                    for r in reversed(group):
                        self.pending.appendleft(r)
                    failed.extend(self._admit_singly(len(group)))
                continue
            for r in group:
                r.admitted = now
            self.inflight.append(_Flight(slot, group, handle, nbytes, nq))
            self.mem_used += nbytes
            self.launches += 1
        return failed

    def _admit_singly(self, count: int) -> List[Request]:
        failed = []
        for _ in range(count):
            if not self.pending or not self.free_slots:
                break
            r = self.pending[0]
            try:
                need = self.backend.footprint(r.flat, r.off)
            except Exception as e:
                self.pending.popleft()
                r.error, r.done = str(e), self.clock()
                failed.append(r)
                continue
            if self.mem_used + need > self.mem_budget:
                break                           # wait for memory to free up
            self.pending.popleft()
            slot = self.free_slots.pop()
            try:
                handle = self.backend.launch(slot, r.flat, r.off)
            except Exception as e:
                self.free_slots.append(slot)
                r.error, r.done = str(e), self.clock()
                failed.append(r)
                continue
            r.admitted = self.clock()
            self.inflight.append(_Flight(slot, [r], handle, need, r.nq))
            self.mem_used += need
            self.launches += 1
        return failed


class PerQueryServer:
    """The plain per-query path as a server: requests in arrival order, every
    query of a request one fc_count_reduce call (one counting launch) on a
    single stream."""

    def __init__(self, db, reducers=("mdl",), ess: float = 1.0,
                 clock: Callable[[], float] = time.perf_counter):
        import torch
        self.torch = torch
        self.db, self.reducers, self.ess, self.clock = db, tuple(reducers), ess, clock
        self.stream = torch.cuda.Stream(device=db.device)
        self.pending: collections.deque = collections.deque()

    def submit(self, req: Request) -> None:
        self.pending.append(req)

    def idle(self) -> bool:
        return not self.pending

    def poll(self) -> List[Request]:
        if not self.pending:
            return []
        torch = self.torch
        r = self.pending.popleft()
        r.admitted = self.clock()
        # one contiguous row of len(reducers) scores per query (a call with
        # one query writes its reducer slots side by side)
        dev = torch.empty((r.nq, len(self.reducers)), dtype=torch.float32,
                          device=self.db.device)
        with torch.cuda.stream(self.stream):
            for i in range(r.nq):
                self.db.count_reduce([r.flat[r.off[i]:r.off[i + 1]]], self.reducers,
                                     ess=self.ess, out=dev[i], with_err=False,
                                     stream=self.stream)
        self.stream.synchronize()
        r.scores = np.ascontiguousarray(dev.cpu().numpy().T)
        r.done = self.clock()
        return [r]


def poisson_arrivals(rng: np.random.Generator, rate: float, n: int) -> np.ndarray:
    """Arrival offsets (seconds) of a Poisson process of the given rate."""
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def run_load(server, batches: Sequence[tuple], arrivals: np.ndarray,
             clock: Callable[[], float] = time.perf_counter, timeout: float = 120.0) -> Dict:
    """Drives the server with requests arriving at `arrivals` (seconds from
    start) and returns latency / throughput statistics."""
    reqs, done = [], []
    t0 = clock()
    i, n = 0, len(batches)
    while len(done) < n:
        now = clock()
        while i < n and arrivals[i] <= now - t0:
            flat, off = batches[i]
            r = Request(i, flat, off, arrival=t0 + float(arrivals[i]))
            reqs.append(r)
            server.submit(r)
            i += 1
        got = server.poll()
        done.extend(got)
        if not got and i < n and server.idle():
            # nothing to do until the next arrival
            wait = t0 + float(arrivals[i]) - clock()
            if wait > 2e-4:
                time.sleep(wait - 1e-4)
        if clock() - t0 > timeout:
            raise TimeoutError("load did not finish in %.1fs" % timeout)
    t1 = clock()
    lat = np.array([r.latency for r in done if r.error is None], dtype=np.float64) * 1e3
    nqs = sum(r.nq for r in done if r.error is None)
    return {"requests": n, "failed": sum(1 for r in done if r.error is not None),
            "queries": nqs, "seconds": t1 - t0, "queries_per_s": nqs / (t1 - t0),
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else math.nan,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else math.nan,
            "mean_ms": float(lat.mean()) if len(lat) else math.nan,
            "launches": getattr(server, "launches", None), "done": done}
