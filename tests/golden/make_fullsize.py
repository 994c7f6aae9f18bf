#!/usr/bin/env python3
"""Writes the oracle's results for every query of the full-size workloads.

For bn-family (50,000 family queries, m = 10^6, MDL), batched-uneven
(200,000 queries, m = 4*10^6, BDeu with ess 1 and MI) and the serving
database's hill-climbing batches (m = 2^22, MDL) this script counts every
query's contingency table with the CPU oracle (the plain definition of a
count, Section 2), computes the oracle's binary64 scores from it, and stores
per query the table's digest (tests/golden_io.table_digest) and the scores in
tests/golden/fullsize_<workload>.npz, together with SHA-256 hashes of the
generated database and query stream (so that a test notices when the seeded
generators no longer produce the same inputs).

Only the oracle computes anything stored here; the inputs come from the
seeded generators.  Run from the repository root:

    python tests/golden/make_fullsize.py [bn-family] [batched-uneven] [serving] [--threads N]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as orc                         # noqa: E402
from paper_1804_04640_amd import synth                    # noqa: E402
from tests.golden_io import array_sha, fullsize_path, table_digest   # noqa: E402

WORKLOADS = {
    "bn-family": lambda: synth.bn_family(),
    "batched-uneven": lambda: synth.batched_uneven(),
    "serving": lambda: synth.serving(),
}


def make(name: str, threads: int) -> None:
    t0 = time.time()
    w = WORKLOADS[name]()
    reducers = tuple(w.reducers)
    print("%s: %s generated in %.1f s" % (name, w.desc, time.time() - t0), flush=True)

    def one(i):
        q = w.query(i)
        T = orc.count(w.D, w.arity, q)
        r = int(w.arity[q[-1]])
        return table_digest(T), [orc.score(red, T, r, w.ess) for red in reducers]

    digest = np.zeros(w.nq, np.uint64)
    scores = np.zeros((len(reducers), w.nq), np.float64)
    t0 = time.time()
    step = 2000
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        for lo in range(0, w.nq, step):
            ids = range(lo, min(w.nq, lo + step))
            for i, (d, s) in zip(ids, ex.map(one, ids)):
                digest[i] = d
                scores[:, i] = s
            done = min(w.nq, lo + step)
            el = time.time() - t0
            print("  %d / %d queries, %.0f s" % (done, w.nq, el), flush=True)
    dt = time.time() - t0
    np.savez(fullsize_path(name),
             digest=digest, scores=scores,
             reducers=np.array(reducers, dtype="U8"),
             ess=np.float64(w.ess), m=np.int64(w.m), nq=np.int64(w.nq),
             data_sha=np.array(array_sha(w.D, w.arity)),
             query_sha=np.array(array_sha(w.vars_flat, w.var_off)),
             desc=np.array(w.desc))
    print("%s: %d queries, %.3e query-rows in %.0f s on %d threads -> %s"
          % (name, w.nq, float(w.nq) * w.m, dt, threads, fullsize_path(name)), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("workloads", nargs="*", default=list(WORKLOADS))
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    for name in a.workloads:
        make(name, a.threads)


if __name__ == "__main__":
    main()
