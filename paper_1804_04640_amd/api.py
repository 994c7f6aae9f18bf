"""torch-facing wrapper over the C ABI: device memory and streams come from
torch, every step of the counting path runs in the HIP library.

    db = Database(D, arity)                      # D: uint8 [n][m] numpy or torch
    T = db.count([0, 2, 1])                      # int32 tensor on the device
    tables, off = db.count_batch(queries)        # packed tables + offsets
    scores = db.count_reduce(queries, ("bdeu", "mi"), ess=1.0)
    n = db.count_assignment([0, 1], [2, 0])
    recs = db.pairs(minsup=0.001)
"""
from __future__ import annotations

import ctypes
import hashlib
import math
import json
import os
from typing import Dict, Iterable, Optional, Sequence

import numpy as np
import torch

from . import _lib as L

REDUCER_BITS = {"ll": L.FC_RED_LL, "mdl": L.FC_RED_MDL, "bdeu": L.FC_RED_BDEU, "mi": L.FC_RED_MI}
STRATEGIES = {"auto": L.FC_STRAT_AUTO, "hist": L.FC_STRAT_HIST, "bitmap": L.FC_STRAT_BITMAP,
              "partition": L.FC_STRAT_PARTITION, "sort": L.FC_STRAT_SORT}


def _np_ptr(a: np.ndarray) -> int:
    return a.ctypes.data if a.size else 0


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def flatten_queries(queries):
    """(vars_flat int32, var_off int64) from a list of variable lists, or
    pass an existing (flat, off) pair through."""
    if isinstance(queries, tuple) and len(queries) == 2 and isinstance(queries[1], np.ndarray):
        flat, off = queries
        return np.ascontiguousarray(flat, np.int32), np.ascontiguousarray(off, np.int64)
    qs = [np.asarray(q, dtype=np.int32).ravel() for q in queries]
    off = np.zeros(len(qs) + 1, dtype=np.int64)
    if qs:
        off[1:] = np.cumsum([len(q) for q in qs])
    flat = np.concatenate(qs).astype(np.int32) if qs else np.zeros(0, np.int32)
    return np.ascontiguousarray(flat), off


class Database:
    """A complete categorical database resident on one GPU."""

    def __init__(self, D, arity, bitvectors: bool = True, layout: str = "col", stream=None,
                 device=None):
        arity = np.ascontiguousarray(np.asarray(arity, dtype=np.uint8))
        lay = L.FC_COL_MAJOR if layout == "col" else L.FC_ROW_MAJOR
        flags = L.FC_DB_BITVECTORS if bitvectors else 0
        self.device = torch.device(device) if device is not None else torch.device(
            "cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            if isinstance(D, torch.Tensor):
                Dt = D.contiguous()
                if Dt.dtype != torch.uint8:
                    raise TypeError("D must be uint8")
                if Dt.is_cuda:
                    flags |= L.FC_DB_DATA_ON_DEVICE
                ptr = Dt.data_ptr() if Dt.numel() else 0
                shape = tuple(Dt.shape)
            else:
                Dt = np.ascontiguousarray(np.asarray(D, dtype=np.uint8))
                ptr = _np_ptr(Dt)
                shape = Dt.shape
            if len(shape) != 2:
                raise ValueError("D must be 2-D")
            n, m = (shape[0], shape[1]) if lay == L.FC_COL_MAJOR else (shape[1], shape[0])
            if len(arity) != n:
                raise ValueError("arity has %d entries for %d variables" % (len(arity), n))
            self._h = L.fc_db_create(ptr, m, n, _np_ptr(arity), lay, flags, _stream(stream))
        self.n, self.m = int(n), int(m)
        self.arity = arity.copy()
        self.bitvectors = bitvectors

    def append(self, D, layout: str = "col", stream=None) -> None:
        """Append instances (uint8 [n][m_new] column-major, or [m_new][n] with
        layout="row"); counts, marginals and bit-vectors cover them at once."""
        lay = L.FC_COL_MAJOR if layout == "col" else L.FC_ROW_MAJOR
        flags = 0
        if isinstance(D, torch.Tensor):
            Dt = D.contiguous()
            if Dt.is_cuda:
                flags |= L.FC_DB_DATA_ON_DEVICE
            ptr, shape = (Dt.data_ptr() if Dt.numel() else 0), tuple(Dt.shape)
        else:
            Dt = np.ascontiguousarray(np.asarray(D, dtype=np.uint8))
            ptr, shape = _np_ptr(Dt), Dt.shape
        n, m_new = (shape[0], shape[1]) if lay == L.FC_COL_MAJOR else (shape[1], shape[0])
        if n != self.n:
            raise ValueError("appended data has %d variables, the database %d" % (n, self.n))
        L.fc_db_append(self.handle, ptr, m_new, lay, flags, _stream(stream))
        self.m += int(m_new)

    # ----------------------------------------------------------- lifecycle
    def trim(self) -> None:
        """Free the handle's idle device workspaces (see fc_db_trim)."""
        L.fc_db_trim(self.handle)

    def close(self):
        if getattr(self, "_h", None):
            L.fc_db_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self) -> int:
        if not self._h:
            raise L.FastcountError(L.FC_ERR_INVALID, "database is closed")
        return self._h

    # ----------------------------------------------------------- facts
    def info(self):
        return L.fc_db_info(self.handle)

    def marginals(self):
        cnt = np.zeros(int(self.arity.astype(np.int64).sum()), np.int64)
        ent = np.zeros(self.n, np.float32)
        L.fc_db_marginals(self.handle, _np_ptr(cnt), _np_ptr(ent))
        return cnt, ent

    def table_cells(self, vars_) -> int:
        v = np.ascontiguousarray(vars_, np.int32)
        return L.fc_table_cells(self.handle, _np_ptr(v), len(v))

    def _empty(self, n, dtype):
        return torch.empty(int(n), dtype=dtype, device=self.device)

    # ----------------------------------------------------------- counting
    def count(self, vars_, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        v = np.ascontiguousarray(vars_, np.int32)
        cells = self.table_cells(v)
        if out is None:
            out = self._empty(cells, torch.int32)
        L.fc_count(self.handle, _np_ptr(v), len(v), out.data_ptr(), cells, _stream(stream))
        return out

    def count_assignment(self, vars_, states, stream=None) -> int:
        v = np.ascontiguousarray(vars_, np.int32)
        s = np.ascontiguousarray(states, np.uint8)
        return L.fc_count_assignment(self.handle, _np_ptr(v), _np_ptr(s), len(v), _stream(stream))

    def count_sparse(self, vars_, cap: Optional[int] = None, stream=None,
                     keys_out: Optional[torch.Tensor] = None,
                     counts_out: Optional[torch.Tensor] = None):
        """(keys int64, counts int32) of the configurations that occur, in
        increasing mixed-radix key order: host numpy arrays, or views of
        keys_out / counts_out (int64 / int32 device tensors of equal length,
        which then set cap) when both are given."""
        v = np.ascontiguousarray(vars_, np.int32)
        if keys_out is not None or counts_out is not None:
            if keys_out is None or counts_out is None or keys_out.dtype != torch.int64 \
                    or counts_out.dtype != torch.int32 or keys_out.numel() != counts_out.numel():
                raise ValueError("keys_out (int64) and counts_out (int32) of equal length are "
                                 "needed together")
            cap = keys_out.numel()
            nnz = L.fc_count_sparse(self.handle, _np_ptr(v), len(v),
                                    keys_out.data_ptr() if cap else 0,
                                    counts_out.data_ptr() if cap else 0, cap, _stream(stream))
            n = min(nnz, cap)
            return keys_out[:n], counts_out[:n], nnz
        cap = self.m if cap is None else int(cap)
        keys = np.zeros(max(cap, 1), np.int64)
        cnt = np.zeros(max(cap, 1), np.int32)
        nnz = L.fc_count_sparse(self.handle, _np_ptr(v), len(v), _np_ptr(keys), _np_ptr(cnt), cap,
                                _stream(stream))
        n = min(nnz, cap)
        return keys[:n], cnt[:n], nnz

    def count_sparse_batch(self, queries, stream=None, keys_out: Optional[torch.Tensor] = None,
                           counts_out: Optional[torch.Tensor] = None):
        """Sparse tables of many queries: (keys int64, counts int32, out_off
        int64 numpy [nq+1]); query i's pairs are keys[out_off[i]:out_off[i+1]].
        Outputs are device tensors: keys_out / counts_out when given (their
        length is the capacity; a batch that does not fit raises), else new
        ones of the nq * m upper bound."""
        flat, off = flatten_queries(queries)
        nq = len(off) - 1
        if keys_out is None or counts_out is None:
            if keys_out is not None or counts_out is not None:
                raise ValueError("keys_out and counts_out are needed together")
            cap = nq * self.m
            keys_out = self._empty(max(cap, 1), torch.int64)
            counts_out = self._empty(max(cap, 1), torch.int32)
        elif keys_out.dtype != torch.int64 or counts_out.dtype != torch.int32 \
                or keys_out.numel() != counts_out.numel():
            raise ValueError("keys_out (int64) and counts_out (int32) of equal length are needed")
        cap = keys_out.numel() if nq else 0
        out_off = np.zeros(nq + 1, np.int64)
        rc, total = L.fc_count_sparse_batch(self.handle, _np_ptr(flat), _np_ptr(off), nq,
                                            keys_out.data_ptr() if cap else 0,
                                            counts_out.data_ptr() if cap else 0, cap,
                                            _np_ptr(out_off), _stream(stream))
        if rc != L.FC_OK:
            raise L.FastcountError(rc, "%d configurations do not fit the %d-entry outputs"
                                   % (total, cap))
        return keys_out[:total], counts_out[:total], out_off

    def count_assignments(self, queries, states, stream=None) -> np.ndarray:
        """Batched single-assignment counts; `states` mirrors `queries`
        (a list of state lists, or a flat uint8 array aligned with vars_flat).
        Returns an int64 numpy array."""
        flat, off = flatten_queries(queries)
        if isinstance(states, np.ndarray) and states.ndim == 1 and len(states) == len(flat):
            st = np.ascontiguousarray(states, np.uint8)
        else:
            st = np.concatenate([np.asarray(x, np.uint8).ravel() for x in states]) \
                if len(states) else np.zeros(0, np.uint8)
            st = np.ascontiguousarray(st, np.uint8)
        if len(st) != len(flat):
            raise ValueError("states do not match the queries")
        out = np.zeros(len(off) - 1, np.int64)
        L.fc_count_assignments(self.handle, _np_ptr(flat), _np_ptr(off), _np_ptr(st), len(off) - 1,
                               _np_ptr(out), _stream(stream))
        return out

    def table_offsets(self, queries) -> np.ndarray:
        flat, off = flatten_queries(queries)
        # out-of-range variables are clipped here only to size the buffer; the
        # library rejects such queries with a message naming them
        ar = np.take(self.arity.astype(np.int64), flat, mode="clip")
        cells = np.array([int(np.prod(ar[off[i]:off[i + 1]])) for i in range(len(off) - 1)],
                         dtype=np.int64)
        toff = np.zeros(len(cells) + 1, np.int64)
        toff[1:] = np.cumsum(cells)
        return toff

    def count_batch(self, queries, strategy: str = "auto", tables: Optional[torch.Tensor] = None,
                    table_off: Optional[np.ndarray] = None, stream=None):
        """Returns (tables int32 tensor, table_off int64 numpy [nq+1])."""
        flat, off = flatten_queries(queries)
        nq = len(off) - 1
        if table_off is None:
            toff = self.table_offsets((flat, off))
            tptr = 0
        else:
            toff = np.ascontiguousarray(table_off, np.int64)
            tptr = _np_ptr(toff)
        if tables is None:
            tables = self._empty(max(1, int(toff[-1])), torch.int32)
        flags = STRATEGIES[strategy]
        L.fc_count_batch(self.handle, _np_ptr(flat), _np_ptr(off), nq, tables.data_ptr(), tptr,
                         flags, _stream(stream))
        return tables, toff

    def count_reduce(self, queries, reducers: Sequence[str] = ("mdl",), ess: float = 1.0,
                     keep_tables: bool = False, strategy: str = "auto", with_err: bool = True,
                     stream=None, out: Optional[torch.Tensor] = None,
                     err_out: Optional[torch.Tensor] = None):
        """Returns (scores {name: tensor[nq]}, err {name: tensor[nq]} or None,
        tables or None, table_off or None)."""
        flat, off = flatten_queries(queries)
        nq = len(off) - 1
        names = [r for r in ("ll", "mdl", "bdeu", "mi") if r in reducers]
        if len(names) != len(set(reducers)):
            raise ValueError("unknown reducer in %r" % (reducers,))
        mask = 0
        for r in names:
            mask |= REDUCER_BITS[r]
        scores = out if out is not None else self._empty(len(names) * max(nq, 1), torch.float32)
        err = (err_out if err_out is not None else
               self._empty(len(names) * max(nq, 1), torch.float32)) if with_err else None
        tables, toff = None, None
        if keep_tables:
            toff = self.table_offsets((flat, off))
            tables = self._empty(max(1, int(toff[-1])), torch.int32)
        params = L.fc_reduce_params(float(ess))
        L.fc_count_reduce(self.handle, _np_ptr(flat), _np_ptr(off), nq, mask,
                          ctypes.addressof(params), scores.data_ptr(),
                          err.data_ptr() if err is not None else 0,
                          tables.data_ptr() if tables is not None else 0, 0,
                          STRATEGIES[strategy], _stream(stream))
        sc = {r: scores[i * nq:(i + 1) * nq] for i, r in enumerate(names)}
        er = {r: err[i * nq:(i + 1) * nq] for i, r in enumerate(names)} if err is not None else None
        return sc, er, tables, toff

    def score_parent_sets(self, child: int, cand, size: int, reducers: Sequence[str] = ("mdl",),
                          ess: float = 1.0, prune_mdl: float = 0.0, stream=None):
        """Scores of every `size`-subset of `cand` as the parent set of
        `child` (lexicographic order of positions in `cand`), enumerated by
        the library: {name: tensor[C(len(cand), size)]}.  prune_mdl > 0 (MDL
        only): sets whose penalty alone reaches it score +inf, uncounted."""
        c = np.ascontiguousarray(np.asarray(cand, dtype=np.int32).ravel())
        names = [r for r in ("ll", "mdl", "bdeu", "mi") if r in reducers]
        if len(names) != len(set(reducers)):
            raise ValueError("unknown reducer in %r" % (reducers,))
        mask = 0
        for r in names:
            mask |= REDUCER_BITS[r]
        nsets = math.comb(len(c), size) if 0 <= size <= len(c) else 0
        scores = self._empty(len(names) * max(nsets, 1), torch.float32)
        params = L.fc_reduce_params(float(ess))
        L.fc_score_parent_sets(self.handle, int(child), _np_ptr(c), len(c), int(size), mask,
                               ctypes.addressof(params), float(prune_mdl), scores.data_ptr(),
                               nsets, _stream(stream))
        return {r: scores[i * nsets:(i + 1) * nsets] for i, r in enumerate(names)}

    def graph(self, queries, reducers: Sequence[str] = ("mdl",), ess: float = 1.0,
              keep_tables: bool = False, strategy: str = "auto", stream=None) -> "BatchGraph":
        """Capture the batch once (plan, upload, every device step) and
        return an object whose replay() reruns all of its device work."""
        return BatchGraph(self, queries, reducers, ess, keep_tables, strategy, stream)

    def plan_summary(self, queries, strategy: str = "auto") -> dict:
        """How many queries of the batch each path answers (planned, not run):
        {"hist", "bitmap", "gram", "derived"}."""
        flat, off = flatten_queries(queries)
        return L.fc_plan_summary(self.handle, _np_ptr(flat), _np_ptr(off), len(off) - 1,
                                 STRATEGIES[strategy])

    def footprint(self, queries, strategy: str = "auto") -> int:
        flat, off = flatten_queries(queries)
        return L.fc_batch_footprint(self.handle, _np_ptr(flat), _np_ptr(off), len(off) - 1,
                                    STRATEGIES[strategy])

    # ----------------------------------------------------------- tuning
    def tuning(self) -> dict:
        return L.fc_db_get_tuning(self.handle).to_dict()

    def set_tuning(self, d: dict) -> None:
        L.fc_db_set_tuning(self.handle, L.fc_tuning.from_dict(d))

    def tuning_key(self) -> str:
        props = torch.cuda.get_device_properties(self.device)
        arch = getattr(props, "gcnArchName", props.name)
        h = hashlib.sha1(self.arity.tobytes()).hexdigest()[:12]
        return "%s/n%d/m%d/r%s/bits%d" % (arch, self.n, self.m, h, int(self.bitvectors))

    def autotune(self, sample_queries, cache: Optional[str] = None, stream=None) -> dict:
        """Run the device autotuner on a representative batch and install the
        result; with `cache`, reuse/store the choice in a JSON file keyed by GPU
        architecture and database shape."""
        key = self.tuning_key()
        db_json = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                db_json = json.load(f)
            if key in db_json:
                self.set_tuning(db_json[key])
                return db_json[key]
        flat, off = flatten_queries(sample_queries)
        L.fc_autotune(self.handle, _np_ptr(flat), _np_ptr(off), len(off) - 1, _stream(stream))
        t = self.tuning()
        if cache:
            db_json[key] = t
            tmp = cache + ".tmp%d" % os.getpid()
            with open(tmp, "w") as f:
                json.dump(db_json, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return t

    # ----------------------------------------------------------- pairs
    def pairs(self, minsup: float, items: Optional[Iterable[int]] = None, gram: bool = False,
              cap: Optional[int] = None, stream=None):
        """Association-rule pairs (Section 4.3).  Returns (records numpy
        structured array, gram tensor or None)."""
        it = None if items is None else np.ascontiguousarray(list(items), np.int32)
        ni = self.n if it is None else len(it)
        g = self._empty(ni * ni, torch.int32) if gram else None
        cap = ni * (ni - 1) // 2 if cap is None else int(cap)
        recs = (L.fc_pair_rec * max(cap, 1))()
        total = L.fc_pairs(self.handle, _np_ptr(it) if it is not None else 0, ni, float(minsup),
                           g.data_ptr() if g is not None else 0, ctypes.addressof(recs), cap,
                           _stream(stream))
        dt = np.dtype([("a", np.int32), ("b", np.int32), ("n_ab", np.int32),
                       ("support", np.float32), ("conf_ab", np.float32), ("conf_ba", np.float32)])
        arr = np.frombuffer(recs, dtype=dt, count=min(total, cap)).copy()
        return arr, (g.view(ni, ni) if g is not None else None), total


class BatchGraph:
    """A batch captured into a hipGraph; outputs live in tensors it owns."""

    def __init__(self, db: Database, queries, reducers, ess, keep_tables, strategy, stream):
        flat, off = flatten_queries(queries)
        nq = len(off) - 1
        self.db = db
        self.names = [r for r in ("ll", "mdl", "bdeu", "mi") if r in reducers]
        mask = 0
        for r in self.names:
            mask |= REDUCER_BITS[r]
        self.scores = db._empty(max(1, len(self.names) * nq), torch.float32)
        self.err = db._empty(max(1, len(self.names) * nq), torch.float32) if self.names else None
        self.tables, self.table_off = None, None
        if keep_tables or not self.names:
            self.table_off = db.table_offsets((flat, off))
            self.tables = db._empty(max(1, int(self.table_off[-1])), torch.int32)
        params = L.fc_reduce_params(float(ess))
        self._g = L.fc_graph_create(db.handle, _np_ptr(flat), _np_ptr(off), nq, mask,
                                    ctypes.addressof(params),
                                    self.scores.data_ptr() if self.names else 0,
                                    self.err.data_ptr() if self.err is not None else 0,
                                    self.tables.data_ptr() if self.tables is not None else 0, 0,
                                    STRATEGIES[strategy], _stream(stream))
        self.nq = nq

    def replay(self, stream=None):
        L.fc_graph_launch(self._g, _stream(stream))

    def result(self) -> Dict[str, torch.Tensor]:
        return {r: self.scores[i * self.nq:(i + 1) * self.nq] for i, r in enumerate(self.names)}

    def close(self):
        if getattr(self, "_g", None):
            L.fc_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
