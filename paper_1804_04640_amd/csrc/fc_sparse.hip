// Sparse contingency tables for queries whose full table dwarfs the data
// (prod r_v >> m): only the configurations that occur, at most min(q r, m) of
// them (Section 3.2), as (mixed-radix key, count) pairs in increasing key
// order.  Sort-and-segment: every instance's key is formed on the device,
// radix-sorted over just the key's significant bits, and run-length encoded
// -- the MSD ordering of Section 3.3 taken to completion, without any dense
// table.
//
// Batches: query j of a group of G consecutive queries contributes the
// composite keys (j << B) | key_j(p), B bits being enough for the largest key
// space of the group, so one radix sort over G*m keys orders every query's
// keys after the query index and one run-length encoding yields every
// query's runs in the packed output order.  Composite keys are 32-bit when
// B + bits(G) <= 32.  A single query is a group of one.
#include <algorithm>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_run_length_encode.hpp>

#include "fc_internal.h"

namespace fc {
namespace {

struct BatchSpec {
    int32_t var[FC_MAX_VARS];
    uint64_t stride[FC_MAX_VARS];
    int32_t k;
    int32_t pad;
};

constexpr int kKeysPerThread = 8;

// Keys of 8 consecutive instances per thread: one 8-byte load per column
// (columns are padded to whole tiles, so the load stays inside the column),
// all loads issued before the arithmetic.
template <typename K>
__global__ __launch_bounds__(256) void k_keys_batch(const uint8_t *__restrict__ cols, int64_t m,
                                                    int64_t pitch,
                                                    const BatchSpec *__restrict__ specs,
                                                    int32_t bits, K *__restrict__ keys) {
    const int32_t j = blockIdx.y;
    const BatchSpec q = specs[j];
    const K hi = bits >= (int32_t)(8 * sizeof(K)) ? (K)0 : (K)((K)j << bits);
    K *out = keys + (int64_t)j * m;
    const int64_t groups = (m + kKeysPerThread - 1) / kKeysPerThread;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < groups;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p0 = g * kKeysPerThread;
        uint64_t w[FC_MAX_VARS];
#pragma unroll
        for (int t = 0; t < FC_MAX_VARS; ++t)
            w[t] = t < q.k ? *(const uint64_t *)(cols + (int64_t)q.var[t] * pitch + p0) : 0;
        uint64_t key[kKeysPerThread];
#pragma unroll
        for (int e = 0; e < kKeysPerThread; ++e) key[e] = 0;
#pragma unroll
        for (int t = 0; t < FC_MAX_VARS; ++t) {
            if (t < q.k) {
                const uint64_t st = q.stride[t];
#pragma unroll
                for (int e = 0; e < kKeysPerThread; ++e)
                    key[e] += ((w[t] >> (8 * e)) & 0xFF) * st;
            }
        }
        if (p0 + kKeysPerThread <= m) {
#pragma unroll
            for (int e = 0; e < kKeysPerThread; ++e) out[p0 + e] = hi | (K)key[e];
        } else {
            for (int e = 0; e < kKeysPerThread && p0 + e < m; ++e) out[p0 + e] = hi | (K)key[e];
        }
    }
}

// Runs [0, nruns) land at base + r (base = *total).  truncate: the first
// cap - base runs are written; otherwise a group that does not fit whole
// writes nothing.  Either way *overflow is set when the runs exceed cap.
template <typename K>
__global__ void k_emit_runs(const K *__restrict__ uniq, const uint32_t *__restrict__ cnt,
                            const uint32_t *__restrict__ nruns, const int64_t *__restrict__ total,
                            K mask, int64_t *__restrict__ keys, int32_t *__restrict__ counts,
                            int64_t cap, int32_t truncate, int32_t *__restrict__ overflow) {
    const int64_t nr = *nruns, base = *total;
    int64_t n = nr;
    if (base + nr > cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *overflow = 1;
        if (!truncate) return;
        n = cap > base ? cap - base : 0;
    }
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        keys[base + r] = (int64_t)(uniq[r] & mask);
        counts[base + r] = (int32_t)cnt[r];
    }
}

// off[j] = *total + (first run of query j) for j in [0, G]; then thread 0
// advances *total past the group (one workgroup: every thread has read
// *total before the barrier).
template <typename K>
__global__ void k_group_offsets(const K *__restrict__ uniq, const uint32_t *__restrict__ nruns,
                                int32_t G, int32_t bits, int64_t *__restrict__ total,
                                int64_t *__restrict__ off) {
    const int64_t nr = *nruns, base = *total;
    for (int32_t j = threadIdx.x; j <= G; j += blockDim.x) {
        int64_t lo = 0, hi = nr;
        if (j == G) {
            lo = nr;
        } else {
            const K first = bits >= (int32_t)(8 * sizeof(K)) ? (K)0 : (K)((K)j << bits);
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (uniq[mid] < first) lo = mid + 1; else hi = mid;
            }
        }
        off[j] = base + lo;
    }
    __syncthreads();
    if (threadIdx.x == 0) *total = base + nr;
}

int sparse_spec(const fc_db *db, const int32_t *vars, int32_t k, const char *who, BatchSpec *spec,
                int32_t *bits) {
    if (k < 1 || k > FC_MAX_VARS) {
        set_error("%s: %d variables (need 1..%d)", who, k, FC_MAX_VARS);
        return FC_ERR_INVALID;
    }
    std::memset(spec, 0, sizeof *spec);
    unsigned __int128 cells = 1;
    for (int32_t t = k - 1; t >= 0; --t) {
        const int32_t v = vars[t];
        if (v < 0 || v >= db->n) {
            set_error("%s: variable %d out of range [0, %d)", who, v, db->n);
            return FC_ERR_INVALID;
        }
        for (int32_t u = 0; u < t; ++u)
            if (vars[u] == v) {
                set_error("%s: variable %d appears twice", who, v);
                return FC_ERR_INVALID;
            }
        spec->var[t] = v;
        spec->stride[t] = (uint64_t)cells;
        cells *= db->arity[v];
    }
    if (cells >= ((unsigned __int128)1 << 63)) {
        set_error("%s: the key space of %d variables exceeds 2^63", who, k);
        return FC_ERR_RANGE;
    }
    spec->k = k;
    int32_t b = 0;
    while (b < 63 && ((uint64_t)1 << b) < (uint64_t)cells) ++b;
    *bits = b;
    return FC_OK;
}

int32_t bits_for(int64_t G) {  // bits of a query index in [0, G)
    int32_t b = 0;
    while (b < 62 && ((int64_t)1 << b) < G) ++b;
    return b;
}

// Consecutive slices of one workspace, 256-byte aligned; with base ==
// nullptr it only measures.
struct Carve {
    char *base = nullptr;
    size_t off = 0;
    template <typename T>
    T *take(size_t n) {
        off = (off + 255) & ~(size_t)255;
        T *p = (T *)(base + off);
        off += sizeof(T) * (n ? n : 1);
        return p;
    }
};

struct Group {
    int64_t q0;
    int32_t G, B;
    bool wide;  // 64-bit composite keys
};

unsigned group_end_bit(const Group &g) {
    return (unsigned)std::max<int32_t>(1, g.B + bits_for(g.G));
}

// Scratch of one group of nk keys of type K, carved from c.
template <typename K>
struct GroupScratch {
    K *kin = nullptr, *ksort = nullptr, *uniq = nullptr;
    uint32_t *cnt = nullptr, *nruns = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    int carve(Carve &c, int64_t nk, unsigned end_bit, hipStream_t s) {
        size_t t_sort = 0, t_rle = 0;
        FC_HIP(rocprim::radix_sort_keys(nullptr, t_sort, (K *)nullptr, (K *)nullptr, (size_t)nk,
                                        0u, end_bit, s));
        FC_HIP(rocprim::run_length_encode(nullptr, t_rle, (K *)nullptr, (unsigned)nk, (K *)nullptr,
                                          (uint32_t *)nullptr, (uint32_t *)nullptr, s));
        kin = c.take<K>((size_t)nk);
        ksort = c.take<K>((size_t)nk);
        uniq = c.take<K>((size_t)nk);
        cnt = c.take<uint32_t>((size_t)nk);
        nruns = c.take<uint32_t>(1);
        tmp_bytes = std::max(t_sort, t_rle);
        tmp = c.take<char>(tmp_bytes);
        return FC_OK;
    }
};

// One group through key formation, sort, run-length encoding, emission and
// offsets, all enqueued on s.
template <typename K>
int sparse_group(fc_db *db, const Group &g, const BatchSpec *d_specs, double col_bytes,
                 char *ws, int64_t *d_total, int64_t *d_off, int64_t *keys, int32_t *counts,
                 int64_t cap, int32_t truncate, int32_t *d_overflow, hipStream_t s) {
    const int64_t m = db->m, nk = (int64_t)g.G * m;
    const unsigned end_bit = group_end_bit(g);
    Carve c;
    c.base = ws;
    GroupScratch<K> S;
    const int rc = S.carve(c, nk, end_bit, s);
    if (rc != FC_OK) return rc;
    const bool wide = sizeof(K) == 8;
    {
        // algorithmic bytes: the group's columns read, its keys written
        ProfScope ps(wide ? "k_keys_batch<u64>" : "k_keys_batch<u32>", s,
                     col_bytes + (double)sizeof(K) * (double)nk, 0.0);
        const int64_t per_q = (m + kKeysPerThread - 1) / kKeysPerThread;
        const int64_t bx = std::max<int64_t>(
            1, std::min<int64_t>((per_q + 255) / 256, (8 * (int64_t)db->cu_count + g.G - 1) / g.G));
        hipLaunchKernelGGL(k_keys_batch<K>, dim3((unsigned)bx, (unsigned)g.G), dim3(256), 0, s,
                           db->d_cols, m, db->pitch, d_specs + g.q0, g.B, S.kin);
        FC_HIP(hipGetLastError());
        ps.end(s);
    }
    {
        // algorithmic bytes: the keys read and written once
        ProfScope ps(wide ? "sort+rle<u64>" : "sort+rle<u32>", s,
                     2.0 * (double)sizeof(K) * (double)nk, 0.0);
        size_t tb = S.tmp_bytes;
        FC_HIP(rocprim::radix_sort_keys(S.tmp, tb, S.kin, S.ksort, (size_t)nk, 0u, end_bit, s));
        tb = S.tmp_bytes;
        FC_HIP(rocprim::run_length_encode(S.tmp, tb, S.ksort, (unsigned)nk, S.uniq, S.cnt,
                                          S.nruns, s));
        ps.end(s);
    }
    const K mask = g.B >= (int32_t)(8 * sizeof(K)) ? ~(K)0 : (K)(((K)1 << g.B) - 1);
    const int64_t eb = std::max<int64_t>(1, std::min<int64_t>((nk + 255) / 256,
                                                              16 * (int64_t)db->cu_count));
    hipLaunchKernelGGL(k_emit_runs<K>, dim3((unsigned)eb), dim3(256), 0, s, S.uniq, S.cnt,
                       S.nruns, d_total, mask, keys, counts, cap, truncate, d_overflow);
    FC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_group_offsets<K>, dim3(1), dim3(256), 0, s, S.uniq, S.nruns, g.G, g.B,
                       d_total, d_off);
    FC_HIP(hipGetLastError());
    return FC_OK;
}

// The shared driver: groups formed over validated specs; offsets (nq+1) and
// the total land in host memory; keys/counts (device or host memory)
// receive the pairs.  truncate: single-query semantics (the first cap pairs).
int sparse_run(fc_db *db, const std::vector<BatchSpec> &specs, const std::vector<int32_t> &qbits,
               int64_t *keys, int32_t *counts, int64_t cap, int32_t truncate, int64_t *out_off,
               int64_t *total_out, bool *overflow_out, const char *who, hipStream_t s) {
    const int64_t nq = (int64_t)specs.size(), m = db->m;
    // groups of consecutive queries: composite keys within 64 bits, at most
    // kGroupKeys keys (m alone when m is larger), at most kGroupMax queries
    // (the grid's y extent)
    constexpr int64_t kGroupKeys = int64_t(1) << 26;
    constexpr int32_t kGroupMax = 65535;
    std::vector<Group> groups;
    for (int64_t i = 0; i < nq;) {
        int32_t G = 1, B = qbits[(size_t)i];
        while (i + G < nq) {
            const int32_t B2 = std::max(B, qbits[(size_t)(i + G)]);
            if (B2 + bits_for(G + 1) > 64 || (int64_t)(G + 1) * m > kGroupKeys ||
                G + 1 > kGroupMax)
                break;
            B = B2;
            ++G;
        }
        groups.push_back({i, G, B, B + bits_for(G) > 32});
        i += G;
    }
    const bool kd = cap > 0 && is_device_ptr(keys), cd = cap > 0 && is_device_ptr(counts);
    if (kd != cd) {
        set_error("%s: keys and counts must both be device or both host memory", who);
        return FC_ERR_INVALID;
    }
    const int64_t dev_cap = cap > 0 ? (kd ? cap : std::min<int64_t>(cap, nq * m)) : 0;
    // one workspace: specs, total, offsets, overflow flag, device copies of
    // host outputs, then the largest group's scratch
    Carve head;
    head.take<BatchSpec>((size_t)nq);
    head.take<int64_t>(1);
    head.take<int64_t>((size_t)nq + 1);
    head.take<int32_t>(2);
    if (cap > 0 && !kd) {
        head.take<int64_t>((size_t)dev_cap);
        head.take<int32_t>((size_t)dev_cap);
    }
    const size_t head_bytes = (head.off + 255) & ~(size_t)255;
    size_t group_bytes = 0;
    for (const Group &g : groups) {
        Carve c;
        const int64_t nk = (int64_t)g.G * m;
        int rc;
        if (g.wide) {
            GroupScratch<uint64_t> S;
            rc = S.carve(c, nk, group_end_bit(g), s);
        } else {
            GroupScratch<uint32_t> S;
            rc = S.carve(c, nk, group_end_bit(g), s);
        }
        if (rc != FC_OK) return rc;
        group_bytes = std::max(group_bytes, c.off);
    }
    Workspace *w = workspace_acquire(db, head_bytes + group_bytes, s);
    if (!w) {
        set_error("%s: a device workspace of %zu bytes could not be allocated", who,
                  head_bytes + group_bytes);
        return FC_ERR_NOMEM;
    }
    struct Release {
        fc_db *db;
        Workspace *w;
        hipStream_t s;
        ~Release() { workspace_release(db, w, s); }
    } release{db, w, s};
    Carve h;
    h.base = (char *)w->p;
    BatchSpec *d_specs = h.take<BatchSpec>((size_t)nq);
    int64_t *d_total = h.take<int64_t>(1);
    int64_t *d_off = h.take<int64_t>((size_t)nq + 1);
    int32_t *d_ovf = h.take<int32_t>(2);
    int64_t *kout = keys;
    int32_t *cout_ = counts;
    if (cap > 0 && !kd) {
        kout = h.take<int64_t>((size_t)dev_cap);
        cout_ = h.take<int32_t>((size_t)dev_cap);
    }
    char *gws = (char *)w->p + head_bytes;

    Staging *st = staging_acquire(sizeof(BatchSpec) * (size_t)nq);
    if (!st) {
        set_error("%s: pinned staging allocation failed", who);
        return FC_ERR_NOMEM;
    }
    std::memcpy(st->host, specs.data(), sizeof(BatchSpec) * (size_t)nq);
    const hipError_t ce = hipMemcpyAsync(d_specs, st->host, sizeof(BatchSpec) * (size_t)nq,
                                         hipMemcpyHostToDevice, s);
    staging_release(st, s);
    FC_HIP(ce);
    FC_HIP(fill_zero_i32((int32_t *)d_total, 2, s));
    FC_HIP(fill_zero_i32(d_ovf, 2, s));
    for (const Group &g : groups) {
        double col_bytes = 0.0;  // one byte per variable and instance
        for (int32_t j = 0; j < g.G; ++j)
            col_bytes += (double)specs[(size_t)(g.q0 + j)].k * (double)m;
        // each group writes off[q0 .. q0+G]; the next one rewrites off[q0+G]
        // with the same value
        const int rc = g.wide
            ? sparse_group<uint64_t>(db, g, d_specs, col_bytes, gws, d_total, d_off + g.q0, kout,
                                     cout_, dev_cap, truncate, d_ovf, s)
            : sparse_group<uint32_t>(db, g, d_specs, col_bytes, gws, d_total, d_off + g.q0, kout,
                                     cout_, dev_cap, truncate, d_ovf, s);
        if (rc != FC_OK) return rc;
    }
    int64_t total = 0;
    int32_t ovf = 0;
    FC_HIP(hipMemcpyAsync(out_off, d_off, sizeof(int64_t) * (size_t)(nq + 1),
                          hipMemcpyDeviceToHost, s));
    FC_HIP(hipMemcpyAsync(&total, d_total, sizeof total, hipMemcpyDeviceToHost, s));
    FC_HIP(hipMemcpyAsync(&ovf, d_ovf, sizeof ovf, hipMemcpyDeviceToHost, s));
    FC_HIP(hipStreamSynchronize(s));
    *total_out = total;
    *overflow_out = ovf != 0 || total > cap;
    const int64_t n_copy = truncate ? std::min(total, cap) : (*overflow_out ? 0 : total);
    if (n_copy > 0 && !kd) {
        FC_HIP(hipMemcpyAsync(keys, kout, sizeof(int64_t) * (size_t)n_copy, hipMemcpyDeviceToHost,
                              s));
        FC_HIP(hipMemcpyAsync(counts, cout_, sizeof(int32_t) * (size_t)n_copy,
                              hipMemcpyDeviceToHost, s));
        FC_HIP(hipStreamSynchronize(s));
    }
    return FC_OK;
}

}  // namespace
}  // namespace fc

using namespace fc;

extern "C" int fc_count_sparse(fc_db *db, const int32_t *vars, int32_t k, int64_t *keys,
                               int32_t *counts, int64_t cap, int64_t *nnz, void *stream) {
    clear_error();
    const char *who = "fc_count_sparse";
    if (!db || !vars || !nnz || cap < 0 || (cap > 0 && (!keys || !counts))) {
        set_error("%s: need a database, vars, nnz, and keys/counts when cap > 0", who);
        return FC_ERR_INVALID;
    }
    std::vector<BatchSpec> specs(1);
    std::vector<int32_t> qbits(1);
    const int rc = sparse_spec(db, vars, k, who, &specs[0], &qbits[0]);
    if (rc != FC_OK) return rc;
    FC_HIP(hipSetDevice(db->device));
    if (db->m == 0) {
        *nnz = 0;
        return FC_OK;
    }
    int64_t off[2];
    bool ovf = false;
    return sparse_run(db, specs, qbits, keys, counts, cap, 1, off, nnz, &ovf, who,
                      (hipStream_t)stream);
}

extern "C" int fc_count_sparse_batch(fc_db *db, const int32_t *vars_flat, const int64_t *var_off,
                                     int64_t nq, int64_t *keys, int32_t *counts, int64_t cap,
                                     int64_t *out_off, int64_t *total_nnz, void *stream) {
    clear_error();
    const char *who = "fc_count_sparse_batch";
    if (!db || nq < 0 || (nq > 0 && (!vars_flat || !var_off)) || !out_off || !total_nnz ||
        cap < 0 || (cap > 0 && (!keys || !counts))) {
        set_error("%s: need a database, nq >= 0, vars_flat/var_off, out_off, total_nnz, and "
                  "keys/counts when cap > 0", who);
        return FC_ERR_INVALID;
    }
    if (nq > 0 && var_off[0] != 0) {
        set_error("%s: var_off[0] must be 0", who);
        return FC_ERR_INVALID;
    }
    std::vector<BatchSpec> specs((size_t)nq);
    std::vector<int32_t> qbits((size_t)nq);
    for (int64_t i = 0; i < nq; ++i) {
        const int64_t k = var_off[i + 1] - var_off[i];
        if (k < 1 || k > FC_MAX_VARS) {
            set_error("%s: query %lld has %lld variables (need 1..%d)", who, (long long)i,
                      (long long)k, FC_MAX_VARS);
            return FC_ERR_INVALID;
        }
        const int rc = sparse_spec(db, vars_flat + var_off[i], (int32_t)k, who,
                                   &specs[(size_t)i], &qbits[(size_t)i]);
        if (rc != FC_OK) return rc;
    }
    if (nq == 0 || db->m == 0) {
        for (int64_t i = 0; i <= nq; ++i) out_off[i] = 0;
        *total_nnz = 0;
        return FC_OK;
    }
    FC_HIP(hipSetDevice(db->device));
    bool ovf = false;
    const int rc = sparse_run(db, specs, qbits, keys, counts, cap, 0, out_off, total_nnz, &ovf,
                              who, (hipStream_t)stream);
    if (rc != FC_OK) return rc;
    if (ovf) {
        set_error("%s: %lld configurations do not fit cap = %lld (out_off and total_nnz are set; "
                  "keys and counts are unspecified)", who, (long long)*total_nnz, (long long)cap);
        return FC_ERR_RANGE;
    }
    return FC_OK;
}
