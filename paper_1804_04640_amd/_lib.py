"""ctypes binding of the C ABI in include/fastcount.h (same names, same order
of arguments).  Argument marshalling only: every step runs in the HIP
library; if the library is not built, every call fails loudly."""
from __future__ import annotations

import ctypes
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfastcount.so")

FC_OK = 0
FC_ERR_INVALID = -1
FC_ERR_RANGE = -2
FC_ERR_NOMEM = -3
FC_ERR_DEVICE = -4
FC_MAX_VARS = 8
FC_COL_MAJOR = 0
FC_ROW_MAJOR = 1
FC_DB_BITVECTORS = 1
FC_DB_DATA_ON_DEVICE = 2
FC_STRAT_AUTO = 0
FC_STRAT_HIST = 1
FC_STRAT_BITMAP = 2
FC_STRAT_PARTITION = 3
FC_STRAT_SORT = FC_STRAT_PARTITION
FC_RED_LL = 1
FC_RED_MDL = 2
FC_RED_BDEU = 4
FC_RED_MI = 8

# every symbol the header declares
EXPORTS = ("fc_db_create", "fc_db_append", "fc_db_destroy", "fc_db_trim", "fc_db_info", "fc_db_marginals", "fc_table_cells",
           "fc_count", "fc_count_assignment", "fc_count_assignments", "fc_count_sparse", "fc_count_sparse_batch", "fc_count_batch", "fc_count_reduce", "fc_count_reduce_noalloc",
           "fc_score_parent_sets", "fc_pairs", "fc_mine", "fc_arm_sizes", "fc_arm_read", "fc_arm_free",
           "fc_batch_footprint", "fc_plan_summary", "fc_graph_create", "fc_graph_launch", "fc_graph_destroy",
           "fc_db_get_tuning", "fc_db_set_tuning", "fc_autotune",
           "fc_profile_enable", "fc_profile_read", "fc_last_error")


class FastcountError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("fastcount error %d: %s" % (code, msg))
        self.code = code


class fc_reduce_params(ctypes.Structure):
    _fields_ = [("ess", ctypes.c_double)]


class fc_tuning(ctypes.Structure):
    _fields_ = [("chunk_rows", ctypes.c_int64), ("bitmap_chunk_rows", ctypes.c_int64),
                ("bitmap_words", ctypes.c_int32), ("persistent_max_queries", ctypes.c_int32),
                ("bitmap_cells", (ctypes.c_uint8 * 6) * FC_MAX_VARS),
                ("packed_columns", ctypes.c_int32), ("bitmap_order", ctypes.c_int32),
                ("derive_tables", ctypes.c_int32), ("one_pass_partition", ctypes.c_int32),
                ("row_sweep", ctypes.c_int32)]

    def to_dict(self):
        return {"chunk_rows": int(self.chunk_rows), "bitmap_chunk_rows": int(self.bitmap_chunk_rows),
                "bitmap_words": int(self.bitmap_words),
                "persistent_max_queries": int(self.persistent_max_queries),
                "bitmap_cells": [[int(x) for x in row] for row in self.bitmap_cells],
                "packed_columns": int(self.packed_columns),
                "bitmap_order": int(self.bitmap_order),
                "derive_tables": int(self.derive_tables),
                "one_pass_partition": int(self.one_pass_partition),
                "row_sweep": int(self.row_sweep)}

    @classmethod
    def from_dict(cls, d):
        t = cls()
        t.chunk_rows = int(d["chunk_rows"])
        t.bitmap_chunk_rows = int(d["bitmap_chunk_rows"])
        t.bitmap_words = int(d["bitmap_words"])
        t.persistent_max_queries = int(d.get("persistent_max_queries", 256))
        for k, row in enumerate(d["bitmap_cells"]):
            for b, x in enumerate(row):
                t.bitmap_cells[k][b] = int(x)
        t.packed_columns = int(d.get("packed_columns", 1))
        t.bitmap_order = int(d.get("bitmap_order", 1))
        t.derive_tables = int(d.get("derive_tables", 1))
        t.one_pass_partition = int(d.get("one_pass_partition", 1))
        t.row_sweep = int(d.get("row_sweep", 1))
        return t


class fc_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("alg_bytes", ctypes.c_double), ("alg_ops", ctypes.c_double)]


class fc_pair_rec(ctypes.Structure):
    _fields_ = [("a", ctypes.c_int32), ("b", ctypes.c_int32), ("n_ab", ctypes.c_int32),
                ("support", ctypes.c_float), ("conf_ab", ctypes.c_float),
                ("conf_ba", ctypes.c_float)]


_lock = threading.Lock()
_lib = None


def load():
    """Load libfastcount.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise FastcountError(FC_ERR_DEVICE,
                                 "HIP library %s is not built; run __graft_entry__.build() or "
                                 "python paper_1804_04640_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        sig = {
            "fc_db_create": (ctypes.c_int, [P, i64, i32, P, i32, u32, P, P]),
            "fc_db_append": (ctypes.c_int, [P, P, i64, i32, u32, P]),
            "fc_db_destroy": (None, [P]),
            "fc_db_trim": (ctypes.c_int, [P]),
            "fc_db_info": (ctypes.c_int, [P, P, P, P, P]),
            "fc_db_marginals": (ctypes.c_int, [P, P, P]),
            "fc_table_cells": (i64, [P, P, i32]),
            "fc_count": (ctypes.c_int, [P, P, i32, P, i64, P]),
            "fc_count_assignment": (ctypes.c_int, [P, P, P, i32, P, P]),
            "fc_count_assignments": (ctypes.c_int, [P, P, P, P, i64, P, P]),
            "fc_count_sparse": (ctypes.c_int, [P, P, i32, P, P, i64, P, P]),
            "fc_count_sparse_batch": (ctypes.c_int, [P, P, P, i64, P, P, i64, P, P, P]),
            "fc_count_batch": (ctypes.c_int, [P, P, P, i64, P, P, u32, P]),
            "fc_count_reduce": (ctypes.c_int, [P, P, P, i64, u32, P, P, P, P, P, u32, P]),
            "fc_count_reduce_noalloc": (ctypes.c_int, [P, P, P, i64, u32, P, P, P, u32, P]),
            "fc_score_parent_sets": (ctypes.c_int, [P, i32, P, i32, i32, u32, P, ctypes.c_double,
                                                    P, i64, P]),
            "fc_pairs": (ctypes.c_int, [P, P, i32, ctypes.c_double, P, P, i64, P, P]),
            "fc_mine": (ctypes.c_int, [P, P, i32, ctypes.c_double, ctypes.c_double, i32, P, P]),
            "fc_arm_sizes": (ctypes.c_int, [P, P, P, P, P]),
            "fc_arm_read": (ctypes.c_int, [P, P, P, P, P, P, P, P, P]),
            "fc_arm_free": (None, [P]),
            "fc_batch_footprint": (ctypes.c_int, [P, P, P, i64, u32, P]),
            "fc_plan_summary": (ctypes.c_int, [P, P, P, i64, u32, P]),
            "fc_graph_create": (ctypes.c_int, [P, P, P, i64, u32, P, P, P, P, P, u32, P, P]),
            "fc_graph_launch": (ctypes.c_int, [P, P]),
            "fc_graph_destroy": (None, [P]),
            "fc_db_get_tuning": (ctypes.c_int, [P, P]),
            "fc_db_set_tuning": (ctypes.c_int, [P, P]),
            "fc_autotune": (ctypes.c_int, [P, P, P, i64, P]),
            "fc_profile_enable": (ctypes.c_int, [ctypes.c_int]),
            "fc_profile_read": (ctypes.c_int, [P, i32, i32]),
            "fc_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        return _lib


def last_error() -> str:
    return load().fc_last_error().decode("utf-8", "replace")


def check(rc: int) -> int:
    if rc < 0:
        raise FastcountError(int(rc), last_error())
    return rc


# Thin wrappers with the C names; pointers are plain integers (host or device).
def fc_db_create(data, m, n, arity, layout, flags, stream):
    h = ctypes.c_void_p()
    check(load().fc_db_create(data, m, n, arity, layout, flags, stream, ctypes.byref(h)))
    return h.value


def fc_db_append(db, data, m_new, layout, flags, stream):
    return check(load().fc_db_append(db, data, m_new, layout, flags, stream))


def fc_db_destroy(db):
    load().fc_db_destroy(db)


def fc_db_trim(db):
    return check(load().fc_db_trim(db))


def fc_db_info(db):
    m, n, hb, nb = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    check(load().fc_db_info(db, ctypes.byref(m), ctypes.byref(n), ctypes.byref(hb),
                            ctypes.byref(nb)))
    return m.value, n.value, bool(hb.value), nb.value


def fc_db_marginals(db, counts, entropy_bits):
    return check(load().fc_db_marginals(db, counts, entropy_bits))


def fc_table_cells(db, vars_, k):
    return check(load().fc_table_cells(db, vars_, k))


def fc_count(db, vars_, k, table, cells, stream):
    return check(load().fc_count(db, vars_, k, table, cells, stream))


def fc_count_assignment(db, vars_, states, k, stream):
    out = ctypes.c_int64()
    check(load().fc_count_assignment(db, vars_, states, k, ctypes.byref(out), stream))
    return out.value


def fc_count_assignments(db, vars_flat, var_off, states_flat, nq, counts, stream):
    return check(load().fc_count_assignments(db, vars_flat, var_off, states_flat, nq, counts,
                                             stream))


def fc_count_sparse(db, vars_, k, keys, counts, cap, stream):
    nnz = ctypes.c_int64()
    check(load().fc_count_sparse(db, vars_, k, keys, counts, cap, ctypes.byref(nnz), stream))
    return nnz.value


def fc_count_sparse_batch(db, vars_flat, var_off, nq, keys, counts, cap, out_off, stream):
    """Returns (rc, total_nnz): rc is FC_OK or FC_ERR_RANGE (the total does not
    fit cap; out_off is filled); other errors raise."""
    total = ctypes.c_int64()
    rc = load().fc_count_sparse_batch(db, vars_flat, var_off, nq, keys, counts, cap, out_off,
                                      ctypes.byref(total), stream)
    if rc == FC_ERR_RANGE and total.value > cap:
        return rc, total.value
    check(rc)
    return rc, total.value


def fc_count_batch(db, vars_flat, var_off, nq, tables, table_off, flags, stream):
    return check(load().fc_count_batch(db, vars_flat, var_off, nq, tables, table_off, flags,
                                       stream))


def fc_count_reduce(db, vars_flat, var_off, nq, reducers, params, scores, err, tables, table_off,
                    flags, stream):
    return check(load().fc_count_reduce(db, vars_flat, var_off, nq, reducers, params, scores, err,
                                        tables, table_off, flags, stream))


def fc_count_reduce_noalloc(db, vars_flat, var_off, nq, reducers, params, scores, err, flags,
                            stream):
    return check(load().fc_count_reduce_noalloc(db, vars_flat, var_off, nq, reducers, params,
                                                scores, err, flags, stream))


def fc_score_parent_sets(db, child, cand, ncand, size, reducers, params, prune_mdl, scores,
                         nsets, stream):
    return check(load().fc_score_parent_sets(db, child, cand, ncand, size, reducers, params,
                                             prune_mdl, scores, nsets, stream))


def fc_pairs(db, items, ni, minsup, gram, out, cap, stream):
    n_out = ctypes.c_int64()
    check(load().fc_pairs(db, items, ni, minsup, gram, out, cap, ctypes.byref(n_out), stream))
    return n_out.value


def fc_mine(db, items, ni, minsup, minconf, max_size, stream):
    h = ctypes.c_void_p()
    check(load().fc_mine(db, items, ni, minsup, minconf, max_size, ctypes.byref(h), stream))
    return h.value


def fc_arm_sizes(r):
    a, b, c, d = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    check(load().fc_arm_sizes(r, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                              ctypes.byref(d)))
    return a.value, b.value, c.value, d.value


def fc_arm_read(r, set_items, set_off, set_count, rule_items, rule_off, rule_cons, rule_support,
                rule_conf):
    return check(load().fc_arm_read(r, set_items, set_off, set_count, rule_items, rule_off,
                                    rule_cons, rule_support, rule_conf))


def fc_arm_free(r):
    load().fc_arm_free(r)


def fc_batch_footprint(db, vars_flat, var_off, nq, flags):
    b = ctypes.c_int64()
    check(load().fc_batch_footprint(db, vars_flat, var_off, nq, flags, ctypes.byref(b)))
    return b.value


def fc_plan_summary(db, vars_flat, var_off, nq, flags):
    out = (ctypes.c_int64 * 4)()
    check(load().fc_plan_summary(db, vars_flat, var_off, nq, flags, out))
    return {"hist": int(out[0]), "bitmap": int(out[1]), "gram": int(out[2]),
            "derived": int(out[3])}


def fc_graph_create(db, vars_flat, var_off, nq, reducers, params, scores, err, tables, table_off,
                    flags, stream):
    h = ctypes.c_void_p()
    check(load().fc_graph_create(db, vars_flat, var_off, nq, reducers, params, scores, err, tables,
                                 table_off, flags, stream, ctypes.byref(h)))
    return h.value


def fc_graph_launch(g, stream):
    return check(load().fc_graph_launch(g, stream))


def fc_graph_destroy(g):
    load().fc_graph_destroy(g)


def fc_db_get_tuning(db):
    t = fc_tuning()
    check(load().fc_db_get_tuning(db, ctypes.byref(t)))
    return t


def fc_db_set_tuning(db, t):
    return check(load().fc_db_set_tuning(db, ctypes.byref(t)))


def fc_autotune(db, vars_flat, var_off, nq, stream):
    return check(load().fc_autotune(db, vars_flat, var_off, nq, stream))


def fc_profile_enable(on):
    return check(load().fc_profile_enable(1 if on else 0))


def fc_profile_read(reset=True):
    """Per-kernel aggregates since the last reset: {name: dict}."""
    n = check(load().fc_profile_read(None, 0, 0))
    arr = (fc_kernel_stat * max(n, 1))()
    n = check(load().fc_profile_read(ctypes.addressof(arr), n, 1 if reset else 0))
    out = {}
    for i in range(min(n, len(arr))):
        s = arr[i]
        out[s.name.decode()] = {"launches": int(s.launches), "ms": float(s.ms),
                                "alg_bytes": float(s.alg_bytes), "alg_ops": float(s.alg_ops)}
    return out
