#!/usr/bin/env python3
"""Benchmark of the counting hot path on one MI355X.

One step = one batch of counting queries through the whole path: plan and
upload, count every query's contingency table (bitmap / histogram /
partition kernels), stream the tables into the fused reducers, scores left
on the device.  The database is resident in HBM before timing starts.

Default workload: batched uneven queries -- n=100 variables with arities
min(8, 2+Geometric(0.4)), m=4,000,000 instances forward-sampled from a random
DAG (in-degree <= 3, Dirichlet(0.5) CPTs), 200,000 queries of 1..6 variables,
fused BDeu (ess 1) and mutual information.  Its 400 MB column store is larger
than the 256 MB MALL.  `--workload bn-family` (m=10^6, 50,000 families, MDL)
runs from the caches: its bandwidth figures are labelled cache-resident.

The JSON line carries query-rows/s (sum over queries of m per second), the
batched vs per-query comparison, p50/p99 latencies, the dominant kernel's
roofline figures (measured with HIP events on the launch stream) and the CPU
oracle timed on this host's cores.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import glob
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP4_PEAK_TFLOPS = 10100.0       # MI355X dense fp4 (e2m1) MFMA
CLOCK_HZ = 2.4e9               # MI355X peak engine clock
N_CU = 256                     # MI355X compute units
# VALU issue: a CU's four SIMDs each take a 64-lane instruction every four
# clocks, so one 64-lane VALU instruction per clock per CU
VALU_PEAK_TOPS = N_CU * 64 * CLOCK_HZ / 1e12       # 39.32 T lane-operations/s
CACHE_RESIDENT = {"plain-small", "bn-family"}      # databases well inside the MALL


def src_hash(files=None) -> str:
    """Hash of the kernel sources a counter figure depends on: the listed
    files of the library's csrc/ (the kernel's own file and the shared
    header), or all of them."""
    csrc = os.path.join(ROOT, "paper_1804_04640_amd", "csrc")
    paths = ([os.path.join(csrc, f) for f in sorted(files)] if files
             else sorted(glob.glob(os.path.join(csrc, "*"))))
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_traffic(workload_name: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the
    kernel's sources changed after the counters were taken."""
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(tfile) as f:
            ent = json.load(f).get(workload_name, {}).get(kernel)
        if ent and ent.get("src_hash") == src_hash(ent.get("src_files")):
            return ent["bytes_per_launch"]
    except (OSError, ValueError):
        pass
    return None


def counter_figures(workload_name: str, kernel: str):
    """Per-launch VALU and LDS wave instructions of `kernel` from the
    committed rocprofv3 counter summary, or None when the kernel's sources
    changed after the counters were taken."""
    try:
        with open(os.path.join(ROOT, "profiles", "counters.json")) as f:
            ent = json.load(f).get(workload_name, {}).get(kernel)
        if ent and ent.get("src_hash") == src_hash(ent.get("src_files")):
            return ent
    except (OSError, ValueError):
        pass
    return None


def workload(name: str):
    from paper_1804_04640_amd import synth
    if name == "bn-family":
        return synth.bn_family(), ("mdl",)
    if name == "plain-small":
        return synth.plain_small(), ("mdl",)
    if name == "batched-uneven":
        return synth.batched_uneven(), ("bdeu", "mi")
    if name == "serving":
        return synth.serving(), ("mdl",)
    if name == "all-pairs":
        return synth.all_pairs(), ()
    raise SystemExit("unknown workload %s" % name)


def percentile(xs, p):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), p)) if len(xs) else None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def usable_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def cpu_baseline(w, reducers, budget_s: float, gpu_scores=None, gpu_err=None):
    """The CPU oracle, as it stands, on bounded samples of the same queries:
    one leg on a single thread, one with query-level threads (the paper's
    solver runs concurrent queries on OpenMP threads).  The thread count is
    the cores this process may use, at most 16 (the host share one GPU
    comes with).  With the GPU's scores (float32, [reducer][query]) it also
    reports their largest relative error against the oracle's binary64
    scores over the threaded sample, and whether every error lies within the
    GPU's own per-result estimate."""
    from oracle import oracle as orc

    def one(i):
        q = w.query(i)
        T = orc.count(w.D, w.arity, q)
        r = int(w.arity[q[-1]])
        return [orc.score(name, T, r, w.ess) for name in reducers]

    # single thread: queries in order until half the budget is spent
    t0 = time.perf_counter()
    n1 = 0
    while n1 < w.nq and (n1 < 8 or time.perf_counter() - t0 < 0.5 * budget_s):
        one(n1)
        n1 += 1
    dt1 = time.perf_counter() - t0
    rate1 = n1 * w.m / dt1
    # threaded: a sample sized for about the other half of the budget
    nproc = usable_cores()
    threads = max(1, min(16, nproc))
    sample = int(min(w.nq, max(64, 0.5 * budget_s * threads * n1 / dt1)))
    ids = list(range(sample))
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        ref = list(ex.map(one, ids))
    dt = time.perf_counter() - t0
    out = {"value": sample * w.m / dt, "unit": "query-rows/s", "cores": threads,
           "kind": "oracle",
           "sample": "first %d of %d queries (m=%d), count + %s, %d threads, %.1f s wall"
                     % (sample, w.nq, w.m, "+".join(reducers), threads, dt),
           "single_thread": {"value": rate1, "unit": "query-rows/s",
                             "sample": "first %d queries, 1 thread, %.1f s" % (n1, dt1)},
           "thread_speedup": (sample * w.m / dt) / rate1,
           "nproc": os.cpu_count(), "usable_cores": nproc, "cpu_model": cpu_model()}
    if gpu_scores is not None:
        worst, within = {}, True
        for slot, name in enumerate(reducers):
            g = gpu_scores[slot * w.nq:slot * w.nq + sample]
            e = gpu_err[slot * w.nq:slot * w.nq + sample] if gpu_err is not None else None
            rel = 0.0
            for i in range(sample):
                d = abs(float(g[i]) - ref[i][slot])
                if ref[i][slot] != 0.0:
                    rel = max(rel, d / abs(ref[i][slot]))
                if e is not None and d > float(e[i]):
                    within = False
            worst[name] = rel
        out["gpu_score_max_rel_err_vs_fp64"] = worst
        out["gpu_score_err_within_estimate"] = within
    return out


def bench_serve(args):
    """Serving: D resident, hill-climbing family batches (10..5000 queries of
    2..7 variables) arriving as a Poisson process at fractions of the
    measured saturation rate; continuous batching against the plain
    per-query path."""
    import torch
    from paper_1804_04640_amd import synth
    from paper_1804_04640_amd.api import Database
    from paper_1804_04640_amd.serving import (CountServer, GpuBackend, PerQueryServer,
                                              poisson_arrivals, run_load)

    t0 = time.time()
    w = synth.serving(nbatches=256)
    print("# %s generated in %.1fs" % (w.desc, time.time() - t0), file=sys.stderr, flush=True)
    db = Database(w.D, w.arity)
    batches = []
    for ids in w.batches:
        qs = [w.query(int(j)) for j in ids]
        off = np.zeros(len(qs) + 1, np.int64)
        off[1:] = np.cumsum([len(q) for q in qs])
        batches.append((np.concatenate(qs).astype(np.int32), off))
    sample = [q for b in batches[:16] for q in
              (b[0][b[1][i]:b[1][i + 1]] for i in range(len(b[1]) - 1))]
    tuning = db.autotune(sample[:4000])
    n = args.serve_requests
    load = [batches[i % len(batches)] for i in range(n)]
    free, _ = torch.cuda.mem_get_info()
    budget = int(free * 0.5)
    rng = np.random.default_rng(5)

    def server():
        return CountServer(GpuBackend(db, ("mdl",), slots=4), mem_budget=budget)

    run_load(server(), load[:64], np.zeros(64))                       # warm up
    sat = run_load(server(), load, np.zeros(n))                       # all at once
    lam_sat = n / sat["seconds"]
    print("# saturation %.1f requests/s, %.3e queries/s" % (lam_sat, sat["queries_per_s"]),
          file=sys.stderr, flush=True)
    rates = []
    for frac in (0.25, 0.5, 0.75, 0.9):
        st = run_load(server(), load, poisson_arrivals(rng, frac * lam_sat, n))
        st.pop("done")
        st["rate_frac"], st["rate_rps"] = frac, frac * lam_sat
        rates.append(st)
        print("# lambda=%.2f*sat: p50 %.2f ms p99 %.2f ms" % (frac, st["p50_ms"], st["p99_ms"]),
              file=sys.stderr, flush=True)
    # the plain per-query path as a server: its own saturation, then Poisson
    # load at half of it (it cannot sustain the batched server's rates)
    npq = min(24, n)
    pq = run_load(PerQueryServer(db, ("mdl",)), load[:npq], np.zeros(npq))
    pq_sat = npq / pq["seconds"]
    pq_half = run_load(PerQueryServer(db, ("mdl",)), load[:npq],
                       poisson_arrivals(rng, 0.5 * pq_sat, npq))
    for d in (pq, pq_half, sat):
        d.pop("done", None)
    out = {"metric": "serving: queries/s and p50/p99 ms from arrival to result",
           "value": sat["queries_per_s"], "unit": "queries/s (saturation)",
           "config": {"workload": w.name, "desc": w.desc, "requests": n, "slots": 4,
                      "mem_budget_bytes": budget, "tuning": tuning},
           "saturation": {"requests_per_s": lam_sat, **sat},
           "poisson": rates,
           "per_query_path": {"saturation_requests_per_s": pq_sat,
                              "saturation_queries_per_s": pq["queries_per_s"],
                              "at_half_its_saturation": pq_half,
                              "note": "requests of the same stream, one launch per query"},
           "batched_vs_per_query_saturation": sat["queries_per_s"] / pq["queries_per_s"]}
    db.close()
    print(json.dumps(out), flush=True)


def bench_parents(args):
    """Exact parent-set assignment (every child, every |Pa| <= MAX_PA, MDL)
    over a 37-variable random-DAG sample with m = 100,000 instances."""
    import torch
    from paper_1804_04640_amd import _lib, parents, synth
    from paper_1804_04640_amd.api import Database

    w = synth.bn_family(m=100_000, nq=1)
    db = Database(w.D, w.arity)
    rng = np.random.default_rng(0)
    sample = [np.concatenate([rng.choice(np.delete(np.arange(w.n), c), size=int(rng.integers(0, args.parents + 1)), replace=False), [c]]).astype(np.int32)
              for c in rng.integers(0, w.n, size=4000)]
    tuning = db.autotune(sample)
    parents.best_parents(db, max_pa=1)                                # warm up
    _lib.fc_profile_enable(True)
    _lib.fc_profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    best, stats = parents.best_parents(db, max_pa=args.parents, score="mdl")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _lib.fc_profile_enable(False)
    prof = _lib.fc_profile_read(reset=True)
    gpu_ms = sum(v["ms"] for v in prof.values())
    out = {"metric": "exact parent-set assignment time (all children, MDL)",
           "value": dt, "unit": "s", "higher_is_better": False,
           "config": {"workload": "bn-family n=37 m=100000", "max_parents": args.parents,
                      "tuning": tuning},
           "families_scored": stats["scored"], "families_pruned": stats["pruned"],
           "levels": stats["levels"], "gpu_kernel_s": gpu_ms / 1e3,
           "kernels": {k: {"launches": v["launches"], "ms": v["ms"]}
                       for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])[:12]},
           "query_rows_per_s": stats["scored"] * w.m / dt,
           "best_parents": {int(c): list(p) for c, (p, _) in sorted(best.items())}}
    db.close()
    print(json.dumps(out), flush=True)


def bench_arm(args, w):
    """Bottom-up association-rule mining (itemsets of up to 6 items, minsup
    0.001, minconf 0.3) on the planted-transaction database: the whole
    level-wise search in the library, the result in host arrays."""
    import torch
    from paper_1804_04640_amd import _lib, arm
    from paper_1804_04640_amd.api import Database

    db = Database(w.D, w.arity)
    arm.mine_arrays(db, minsup=w.minsup, minconf=0.3, max_size=6)    # warm up
    _lib.fc_profile_enable(True)
    _lib.fc_profile_read(reset=True)
    times = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = arm.mine_arrays(db, minsup=w.minsup, minconf=0.3, max_size=6)
        torch.cuda.synchronize()
        times.append(1e3 * (time.perf_counter() - t0))
    _lib.fc_profile_enable(False)
    prof = _lib.fc_profile_read(reset=True)
    sizes = np.diff(r["set_off"])
    levels = {int(k): int((sizes == k).sum()) for k in np.unique(sizes)}
    a = prof.get("k_assign_batch", {"ms": 0.0, "launches": 1, "alg_bytes": 0.0})
    out = {"metric": "association-rule mining time (bottom-up, single-assignment counts)",
           "value": float(np.median(times)), "unit": "ms", "higher_is_better": False,
           "config": {"workload": w.name, "desc": w.desc, "minsup": w.minsup, "minconf": 0.3,
                      "max_size": 6},
           "frequent_itemsets_by_size": levels, "rules": int(len(r["rule_cons"])),
           "gpu_kernel_ms": sum(v["ms"] for v in prof.values()) / args.steps,
           "kernels": {k: {"launches": v["launches"], "avg_us": 1e3 * v["ms"] / v["launches"]}
                       for k, v in prof.items()},
           "assign_batch_GBps": (a["alg_bytes"] / (a["ms"] * 1e-3) / 1e9) if a["ms"] else None}
    db.close()
    print(json.dumps(out), flush=True)


def bench_sparse(args):
    """Sparse tables of high-arity queries: one step = the 64 queries of the
    high-arity workload in one batched call (composite-key radix sorts and
    run-length encoding), (key, count) pairs left on the device.  The same
    queries one call each are timed beside it."""
    import torch
    from oracle import oracle as orc
    from paper_1804_04640_amd import _lib, synth
    from paper_1804_04640_amd.api import Database

    w = synth.high_arity()
    q = (w.vars_flat, w.var_off)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        db = Database(w.D, w.arity, bitvectors=False, stream=stream)
        keys = torch.empty(w.nq * w.m, dtype=torch.int64, device="cuda")
        cnts = torch.empty(w.nq * w.m, dtype=torch.int32, device="cuda")
        off = None

        def step():
            return db.count_sparse_batch(q, stream=stream, keys_out=keys, counts_out=cnts)[2]

        for _ in range(args.warmup):
            off = step()
        _lib.fc_profile_enable(True)
        _lib.fc_profile_read(reset=True)
        times = []
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            off = step()
            torch.cuda.synchronize()
            times.append(1e3 * (time.perf_counter() - t0))
        _lib.fc_profile_enable(False)
        prof = _lib.fc_profile_read(reset=True)
        # the plain per-query call, for comparison
        one_k, one_c = keys[:w.m], cnts[:w.m]
        for i in range(4):
            db.count_sparse(w.query(i), stream=stream, keys_out=one_k, counts_out=one_c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(w.nq):
            db.count_sparse(w.query(i), stream=stream, keys_out=one_k, counts_out=one_c)
        torch.cuda.synchronize()
        per_query_s = time.perf_counter() - t0
    name, g = max(prof.items(), key=lambda kv: kv[1]["ms"])
    ms = float(np.mean(times))
    ks = np.diff(w.var_off)
    nnz = np.diff(off)
    value = w.nq * w.m / (ms * 1e-3)
    achieved = g["alg_bytes"] / (g["ms"] * 1e-3) / 1e9
    out = {
        "metric": "exact query-rows counted/s (sparse tables of high-arity queries)",
        "value": value, "unit": "query-rows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8 states, u32/u64 composite keys, int32 counts", "data": "synthetic",
        "config": {"workload": w.name, "desc": w.desc, "queries": w.nq, "m": w.m,
                   "k_min": int(ks.min()), "k_max": int(ks.max()),
                   "mean_nnz": float(np.mean(nnz)),
                   "min_cells": float(min(np.prod(w.arity[w.query(i)].astype(np.float64))
                                          for i in range(w.nq)))},
        "p50_ms": percentile(times, 50), "p99_ms": percentile(times, 99),
        "kernels": {k: {"launches": v["launches"], "avg_us": 1e3 * v["ms"] / v["launches"]}
                    for k, v in prof.items()},
        "per_query": {"value": w.nq * w.m / per_query_s, "unit": "query-rows/s",
                      "sample": "the same %d queries, one fc_count_sparse call each" % w.nq},
        "batched_vs_per_query": value / (w.nq * w.m / per_query_s),
        "roofline": {"bound": "hbm", "kernel": name, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "avg_launch_us": 1e3 * g["ms"] / g["launches"],
                     "alg_bytes_per_launch": g["alg_bytes"] / g["launches"],
                     "traffic": None},
        "cpu_baseline": None,
    }
    if args.cpu_budget > 0:
        t0 = time.perf_counter()
        done = 0
        while done < w.nq and (done < 4 or time.perf_counter() - t0 < args.cpu_budget):
            orc.count_sparse(w.D, w.arity, w.query(done))
            done += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": done * w.m / dt, "unit": "query-rows/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "first %d of %d queries (m=%d), 1 thread, %.1f s"
                                         % (done, w.nq, w.m, dt)}
    db.close()
    print(json.dumps(out), flush=True)


def bench_append(args, w):
    """Appends: one step = the second half of the database appended, in
    batches of 50,000 instances from device memory, to a handle created on
    the first half (the creation is outside the timed region)."""
    import torch
    from paper_1804_04640_amd import _lib
    from paper_1804_04640_amd.api import Database

    m0 = w.m // 2
    batch = 50_000
    Dd = torch.from_numpy(w.D).cuda()
    parts = [Dd[:, lo:min(w.m, lo + batch)].contiguous() for lo in range(m0, w.m, batch)]
    stream = torch.cuda.Stream()
    times, host_times = [], []
    with torch.cuda.stream(stream):
        for it in range(args.warmup + args.steps):
            db = Database(Dd[:, :m0], w.arity, stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for p in parts:
                db.append(p, stream=stream)
            torch.cuda.synchronize()
            if it >= args.warmup:
                times.append(1e3 * (time.perf_counter() - t0))
            db.close()
        for it in range(2):                  # host-memory source (PCIe included)
            db = Database(Dd[:, :m0], w.arity, stream=stream)
            hparts = [np.ascontiguousarray(w.D[:, lo:min(w.m, lo + batch)])
                      for lo in range(m0, w.m, batch)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for p in hparts:
                db.append(p, stream=stream)
            torch.cuda.synchronize()
            if it:
                host_times.append(1e3 * (time.perf_counter() - t0))
            last = db
            if it == 0:
                db.close()
        # the appended handle answers like one created on the whole data
        ref = Database(Dd, w.arity, stream=stream)
        q = (w.vars_flat[:w.var_off[200]], w.var_off[:201])
        a, _ = last.count_batch(q, stream=stream)
        b, _ = ref.count_batch(q, stream=stream)
        same = bool(torch.equal(a, b))
        last.close()
        ref.close()
    ms = float(np.mean(times))
    added = w.m - m0
    sum_r = int(w.arity.astype(np.int64).sum())
    per_inst = 2 * w.n + w.n / 2 + sum_r / 8.0     # read + column write + packed + bit-vectors
    achieved = added * per_inst / (ms * 1e-3) / 1e9
    out = {
        "metric": "instances appended/s (device-resident batches)",
        "value": added / (ms * 1e-3), "unit": "instances/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8 states", "data": "synthetic",
        "config": {"workload": w.name, "desc": w.desc, "base_m": m0, "appended": added,
                   "batch": batch, "batches": len(parts)},
        "host_source_instances_per_s": added / (float(np.mean(host_times)) * 1e-3),
        "tables_match_fresh_handle": same,
        "roofline": {"bound": "hbm", "kernel": "fc_db_append (whole call)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "alg_bytes_per_instance": per_inst,
                     "traffic": None},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def bench_pairs(args, w):
    """All-pairs co-occurrence: one step = Gram on MFMA + pair records."""
    import torch
    from oracle import oracle as orc
    from paper_1804_04640_amd import _lib
    from paper_1804_04640_amd.api import Database

    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        db = Database(w.D, w.arity, stream=stream)
        n, m = w.n, w.m
        cap = n * (n - 1) // 2

        def step():
            return db.pairs(w.minsup, cap=cap, stream=stream)

        for _ in range(args.warmup):
            recs, _, total = step()
        _lib.fc_profile_enable(True)
        _lib.fc_profile_read(reset=True)
        times = []
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            recs, _, total = step()
            torch.cuda.synchronize()
            times.append(1e3 * (time.perf_counter() - t0))
        _lib.fc_profile_enable(False)
        prof = _lib.fc_profile_read(reset=True)
    g = prof["k_gram"]
    ms = float(np.mean(times))
    pair_rows = n * (n - 1) / 2 * m
    achieved = g["alg_ops"] / (g["ms"] * 1e-3) / 1e12
    out = {
        "metric": "exact query-rows counted/s + HBM GB/s frac; batched vs per-query; p50/p99 ms",
        "value": pair_rows / (ms * 1e-3), "unit": "pair-rows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "e2m1 (fp4) MFMA operands of 0/1, fp32 accumulation (exact below 2^24), "
                 "int32 totals", "data": "synthetic",
        "config": {"workload": w.name, "desc": w.desc, "items": n, "m": m,
                   "minsup": w.minsup, "pairs_above_minsup": int(total)},
        "p50_ms": percentile(times, 50), "p99_ms": percentile(times, 99),
        "roofline": {"bound": "mfma", "kernel": "k_gram", "achieved": achieved,
                     "peak": FP4_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP4_PEAK_TFLOPS,
                     "avg_launch_us": 1e3 * g["ms"] / g["launches"],
                     "alg_ops_per_launch": g["alg_ops"] / g["launches"],
                     "traffic": counter_traffic(w.name, "k_gram")},
        "cpu_baseline": None,
    }
    if args.cpu_budget > 0:
        t0 = time.perf_counter()
        sub = max(1, min(m, int(m * args.cpu_budget / 60.0)))
        orc.gram(np.ascontiguousarray(w.D[:, :sub]))
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n * (n - 1) / 2 * sub / dt, "unit": "pair-rows/s",
                               "cores": 1, "kind": "oracle",
                               "sample": "co-occurrence of all %d items over the first %d "
                                         "instances, 1 thread" % (n, sub)}
    db.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched-uneven", choices=["plain-small", "bn-family", "batched-uneven", "all-pairs", "serving"])
    ap.add_argument("--strategy", default="auto", choices=["auto", "hist", "bitmap", "partition"])
    ap.add_argument("--per-query", type=int, default=2000,
                    help="queries timed on the plain per-query path (0: skip)")
    ap.add_argument("--cpu-budget", type=float, default=20.0,
                    help="seconds of oracle work in the CPU baseline, half on one thread, half "
                         "threaded (0: skip)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="run the device autotuner on a sample of the batch before timing")
    ap.add_argument("--tune", default=None,
                    help="JSON tuning to install instead (keys of fc_tuning)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of autotuner results to reuse / fill")
    ap.add_argument("--compare-strategies", type=int, default=1,
                    help="also time the batch with the bitmap and the histogram strategy forced")
    ap.add_argument("--graph", type=int, default=1,
                    help="also time the batch captured once into a hipGraph and replayed")
    ap.add_argument("--serve", action="store_true",
                    help="serving mode (hill-climbing batches, Poisson arrivals, p50/p99)")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--parents", type=int, default=0, metavar="MAX_PA",
                    help="exact parent-set assignment with |Pa| <= MAX_PA on a 37-variable "
                         "DAG sample of m=100,000 (MDL)")
    ap.add_argument("--arm", action="store_true",
                    help="with --workload all-pairs: bottom-up association-rule mining")
    ap.add_argument("--sparse", action="store_true",
                    help="sparse tables of the high-arity workload (n=30, arities up to 99, "
                         "queries of more than 2^24 cells)")
    ap.add_argument("--append", action="store_true",
                    help="instances appended per second (second half of the workload's data in "
                         "batches of 50,000)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (counter scale)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "launches": 3}))
        return
    if args.gpus != 1:
        print("bench.py: the counting path runs on one GPU; --gpus %d is not supported "
              "(sharding across GPUs is a design note only)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1804_04640_amd import _lib
    from paper_1804_04640_amd.api import Database

    torch.cuda.set_device(0)
    if args.sparse:
        return bench_sparse(args)
    t0 = time.time()
    w, reducers = workload(args.workload)
    print("# workload %s generated in %.1fs: %s" % (w.name, time.time() - t0, w.desc),
          file=sys.stderr, flush=True)
    if args.parents:
        return bench_parents(args)
    if args.append:
        return bench_append(args, w)
    if args.workload == "all-pairs" and args.arm:
        return bench_arm(args, w)
    if args.workload == "all-pairs":
        return bench_pairs(args, w)
    if args.serve:
        return bench_serve(args)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        db = Database(w.D, w.arity, stream=stream)
        q = (w.vars_flat, w.var_off)
        nq = w.nq
        ks = np.diff(w.var_off)
        rows = float(nq) * w.m
        alg_bytes = float(ks.sum()) * w.m
        scores = torch.empty(len(reducers) * nq, dtype=torch.float32, device="cuda")
        errs = torch.empty_like(scores)
        tuning = None
        if args.tune:
            t = db.tuning()
            t.update(json.loads(args.tune))
            db.set_tuning(t)
            tuning = db.tuning()
        elif args.autotune:
            t0 = time.time()
            # the batch itself: row-chunk choices depend on how many
            # workgroups a launch group has, so a smaller sample misleads
            tuning = db.autotune(q, cache=args.tune_cache, stream=stream)
            print("# autotuned on %d queries in %.1fs: %s" % (nq, time.time() - t0,
                                                              json.dumps(tuning)),
                  file=sys.stderr, flush=True)

        plan = db.plan_summary(q, strategy=args.strategy)

        def step():
            db.count_reduce(q, reducers, ess=w.ess, strategy=args.strategy, out=scores,
                            err_out=errs, stream=stream)

        for _ in range(args.warmup):
            step()
        stream.synchronize()
        print("# warmup done", file=sys.stderr, flush=True)
        _lib.fc_profile_enable(True)
        _lib.fc_profile_read(reset=True)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for a, b in evs:
            a.record(stream)
            step()
            b.record(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        _lib.fc_profile_enable(False)
        prof = _lib.fc_profile_read(reset=True)
        step_ms = [a.elapsed_time(b) for a, b in evs]
        print("# timed %d steps: %.2f ms/step (wall)" % (args.steps, 1e3 * wall / args.steps),
              file=sys.stderr, flush=True)
        # the same steps without the per-launch profiling events, which
        # lengthen launch-bound batches (the timed region above keeps them:
        # the roofline's kernel times come from it)
        uev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        for a, b in uev:
            a.record(stream)
            step()
            b.record(stream)
        stream.synchronize()
        unprof_ms = [a.elapsed_time(b) for a, b in uev]

        # plain per-query path: one call (one counting launch + reduce) per query
        per_query = None
        if args.per_query > 0:
            n = min(args.per_query, nq)
            lat = []
            one = torch.empty(len(reducers), dtype=torch.float32, device="cuda")
            for i in range(min(20, n)):                       # warm the path
                db.count_reduce([w.query(i)], reducers, ess=w.ess, out=one, with_err=False,
                                stream=stream)
            stream.synchronize()
            t1 = time.perf_counter()
            for i in range(n):
                s0 = time.perf_counter()
                db.count_reduce([w.query(i)], reducers, ess=w.ess, out=one, with_err=False,
                                stream=stream)
                stream.synchronize()
                lat.append(1e3 * (time.perf_counter() - s0))
            dt = time.perf_counter() - t1
            per_query = {"value": n * w.m / dt, "unit": "query-rows/s",
                         "sample": "first %d queries, one call each, synchronised" % n,
                         "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99)}

        # the same batch captured once into a hipGraph and replayed: every
        # device step of the path, no host planning per step
        graph = None
        if args.graph:
            g = db.graph(q, reducers, ess=w.ess, stream=stream)
            g.replay(stream)
            stream.synchronize()
            gev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(args.steps)]
            for a, b in gev:
                a.record(stream)
                g.replay(stream)
                b.record(stream)
            stream.synchronize()
            g_ms = [a.elapsed_time(b) for a, b in gev]
            same = bool(torch.equal(g.scores[:scores.numel()], scores))
            g.close()
            gm = float(np.mean(g_ms))
            graph = {"ms_per_step": gm, "value": rows / (gm * 1e-3),
                     "p50_ms": percentile(g_ms, 50), "p99_ms": percentile(g_ms, 99),
                     "scores_equal_eager": same}

        # forced strategies beside auto (the same batch and reducers; a
        # forced bitmap falls back to the histogram for tables it cannot hold)
        strategies = None
        if args.compare_strategies:
            strategies = {}
            for strat in ("bitmap", "hist"):
                sev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                       for _ in range(3)]
                db.count_reduce(q, reducers, ess=w.ess, strategy=strat, out=scores, err_out=errs,
                                stream=stream)
                for a, b in sev:
                    a.record(stream)
                    db.count_reduce(q, reducers, ess=w.ess, strategy=strat, out=scores,
                                    err_out=errs, stream=stream)
                    b.record(stream)
                stream.synchronize()
                sm = float(np.median([a.elapsed_time(b) for a, b in sev]))
                strategies[strat] = {"ms_per_step": sm, "value": rows / (sm * 1e-3)}
            db.count_reduce(q, reducers, ess=w.ess, strategy=args.strategy, out=scores,
                            err_out=errs, stream=stream)
            stream.synchronize()

    ms = float(np.mean(step_ms))
    value = rows / (ms * 1e-3)
    # dominant kernel: the counting kernel (algorithmic bytes > 0) with the
    # largest summed time; the reducer's share is reported with the kernels
    counting = {k: v for k, v in prof.items() if v["alg_bytes"] > 0}
    dom_name, dom = max((counting or prof).items(), key=lambda kv: kv[1]["ms"])
    c_ms = sum(v["ms"] for v in counting.values())
    c_bytes = sum(v["alg_bytes"] for v in counting.values())
    # histogram kernels add one LDS counter per (query, instance); their
    # algorithmic bytes are K per unit
    h_units, h_ms = 0.0, 0.0
    for name, v in counting.items():
        if name.startswith("k_hist"):
            kk = int(name.split("<")[1].split(",")[0].rstrip(">"))
            h_units += v["alg_bytes"] / kk
            h_ms += v["ms"]
    launch_s = dom["ms"] * 1e-3 / dom["launches"] if dom["launches"] else 0.0
    alg_per_launch = dom["alg_bytes"] / dom["launches"] if dom["launches"] else 0.0
    # algorithmic work of a counting launch: k digit steps per (query,
    # instance) -- one per query variable, the O(|Pa| m) of Radix -- the same
    # count as its k algorithmic bytes per query-row
    achieved = alg_per_launch / launch_s / 1e12 if launch_s > 0 else 0.0
    traffic = counter_traffic(args.workload, dom_name)
    # the issue rate the kernel reaches: its counted VALU wave instructions
    # per launch over the live launch time, against one 64-lane instruction
    # per clock per CU at 2.4 GHz on 256 CUs
    cfig = counter_figures(args.workload, dom_name)
    valu_frac = (cfig["valu_inst_per_launch"] / (launch_s * CLOCK_HZ * N_CU)
                 if cfig and launch_s > 0 else None)
    cache_resident = args.workload in CACHE_RESIDENT
    out = {
        "metric": "exact query-rows counted/s + HBM GB/s frac; batched vs per-query; p50/p99 ms",
        "value": value,
        "unit": "query-rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8 states, int32 counts, f32 reducers",
        "data": "synthetic",
        "config": {"workload": w.name, "desc": w.desc, "queries": nq, "m": w.m, "n": w.n,
                   "reducers": list(reducers), "strategy": args.strategy, "tuning": tuning,
                   "column_store_bytes": int(w.n) * int(w.m), "cache_resident": cache_resident,
                   "parallelism": "single GPU"},
        "batched": {"p50_ms": percentile(step_ms, 50), "p99_ms": percentile(step_ms, 99),
                    "plan": plan,
                    "effective_GBps": alg_bytes / (ms * 1e-3) / 1e9,
                    "effective_over_hbm_peak": alg_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "counting_kernels_GBps": c_bytes / (c_ms * 1e-3) / 1e9 if c_ms else None,
                    "histogram_lds_adds_per_s": h_units / (h_ms * 1e-3) if h_ms else None,
                    "kernels": {k: {"launches": v["launches"], "avg_us": 1e3 * v["ms"] / v["launches"],
                                    "share": v["ms"] / sum(x["ms"] for x in prof.values())}
                                for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])}},
        "unprofiled": {"ms_per_step": float(np.mean(unprof_ms)),
                       "value": rows / (float(np.mean(unprof_ms)) * 1e-3),
                       "p50_ms": percentile(unprof_ms, 50), "p99_ms": percentile(unprof_ms, 99)},
        "graph_replay": graph,
        "forced_strategies": strategies,
        "per_query": per_query,
        "batched_vs_per_query": (value / per_query["value"]) if per_query else None,
        "roofline": {"bound": "alu", "kernel": dom_name, "achieved": achieved,
                     "peak": VALU_PEAK_TOPS, "unit": "Tops/s", "frac": achieved / VALU_PEAK_TOPS,
                     "traffic": traffic,
                     "work": "k digit steps per (query, instance) = k algorithmic bytes "
                             "per query-row; peak = one 64-lane VALU instruction per clock "
                             "per CU x 256 CUs x 2.4 GHz",
                     "avg_launch_us": 1e6 * launch_s,
                     "alg_ops_per_launch": alg_per_launch,
                     "valu_issue_frac": valu_frac,
                     "valu_lane_ops_per_alg_op": (64 * cfig["valu_inst_per_launch"] / alg_per_launch
                                                  if cfig and alg_per_launch else None),
                     "lds_inst_per_launch": cfig["lds_inst_per_launch"] if cfig else None,
                     "alg_GBps": achieved * 1e3,
                     "alg_GBps_over_hbm_peak": achieved * 1e3 / HBM_PEAK_GBS,
                     "cache_resident": cache_resident,
                     "traffic_note": "FETCH_SIZE + WRITE_SIZE bytes per launch (copy-calibrated): "
                                     "L2-miss traffic served by the MALL or HBM; no counter of "
                                     "this platform separates the two, so HBM bytes are at most "
                                     "this"},
        "cpu_baseline": None,
    }
    if args.cpu_budget > 0:
        out["cpu_baseline"] = cpu_baseline(w, reducers, args.cpu_budget,
                                           scores.cpu().numpy(), errs.cpu().numpy())
    db.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
