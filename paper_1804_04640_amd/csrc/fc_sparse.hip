// Sparse contingency tables for queries whose full table dwarfs the data
// (prod r_v >> m): only the configurations that occur, at most min(q r, m) of
// them (Section 3.2), as (mixed-radix key, count) pairs in increasing key
// order.  Sort-and-segment: every instance's 64-bit key is formed on the
// device, radix-sorted over just the key's significant bits, and run-length
// encoded -- the MSD ordering of Section 3.3 taken to completion, without any
// dense table.
#include <algorithm>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_run_length_encode.hpp>

#include "fc_internal.h"

namespace fc {
namespace {

struct KeySpec {
    int32_t var[FC_MAX_VARS];
    uint64_t stride[FC_MAX_VARS];
};

__global__ void k_keys(const uint8_t *__restrict__ cols, int64_t m, int64_t m_pad, KeySpec q,
                       int32_t k, uint64_t *__restrict__ keys) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m;
         p += (int64_t)gridDim.x * blockDim.x) {
        uint64_t key = 0;
        for (int32_t t = 0; t < k; ++t)
            key += (uint64_t)cols[(int64_t)q.var[t] * m_pad + p] * q.stride[t];
        keys[p] = key;
    }
}

// Batched form: query j of a group of G queries contributes the composite
// keys (j << B) | key_j(p), B bits being enough for the largest key space of
// the group, so one radix sort over G*m keys orders every query's keys after
// the query index, and one run-length encoding yields every query's runs in
// the packed output order.
struct BatchSpec {
    int32_t var[FC_MAX_VARS];
    uint64_t stride[FC_MAX_VARS];
    int32_t k;
    int32_t pad;
};

template <typename K>
__global__ void k_keys_batch(const uint8_t *__restrict__ cols, int64_t m, int64_t m_pad,
                             const BatchSpec *__restrict__ specs, int32_t bits,
                             K *__restrict__ keys) {
    const int32_t j = blockIdx.y;
    const BatchSpec q = specs[j];
    const K hi = bits >= (int32_t)(8 * sizeof(K)) ? (K)0 : (K)((K)j << bits);
    K *out = keys + (int64_t)j * m;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m;
         p += (int64_t)gridDim.x * blockDim.x) {
        uint64_t key = 0;
        for (int32_t t = 0; t < q.k; ++t)
            key += (uint64_t)cols[(int64_t)q.var[t] * m_pad + p] * q.stride[t];
        out[p] = hi | (K)key;
    }
}

// Runs [0, nruns) land at base + r (base = *total); written only when the
// whole group fits under cap, otherwise *overflow is set.
template <typename K>
__global__ void k_emit_runs(const K *__restrict__ uniq, const uint32_t *__restrict__ cnt,
                            const uint32_t *__restrict__ nruns, const int64_t *__restrict__ total,
                            K mask, int64_t *__restrict__ keys, int32_t *__restrict__ counts,
                            int64_t cap, int32_t *__restrict__ overflow) {
    const int64_t nr = *nruns, base = *total;
    if (base + nr > cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *overflow = 1;
        return;
    }
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nr;
         r += (int64_t)gridDim.x * blockDim.x) {
        keys[base + r] = (int64_t)(uniq[r] & mask);
        counts[base + r] = (int32_t)cnt[r];
    }
}

// off[j] = *total + (first run of query j), for j in [0, G]; then the last
// thread advances *total past the group (it alone reads and writes it after
// every other thread of the launch has read it: one workgroup, a barrier).
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

__global__ void k_u32_to_i32(const uint32_t *__restrict__ in, int64_t n, int32_t *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (int32_t)in[i];
}

}  // namespace
}  // namespace fc

using namespace fc;

extern "C" int fc_count_sparse(fc_db *db, const int32_t *vars, int32_t k, int64_t *keys,
                               int32_t *counts, int64_t cap, int64_t *nnz, void *stream) {
    clear_error();
    if (!db || !vars || !nnz || cap < 0 || (cap > 0 && (!keys || !counts))) {
        set_error("fc_count_sparse: need a database, vars, nnz, and keys/counts when cap > 0");
        return FC_ERR_INVALID;
    }
    if (k < 1 || k > FC_MAX_VARS) {
        set_error("fc_count_sparse: %d variables (need 1..%d)", k, FC_MAX_VARS);
        return FC_ERR_INVALID;
    }
    KeySpec q;
    std::memset(&q, 0, sizeof q);
    unsigned __int128 cells = 1;
    for (int32_t t = k - 1; t >= 0; --t) {
        const int32_t v = vars[t];
        if (v < 0 || v >= db->n) {
            set_error("fc_count_sparse: variable %d out of range [0, %d)", v, db->n);
            return FC_ERR_INVALID;
        }
        for (int32_t u = 0; u < t; ++u)
            if (vars[u] == v) {
                set_error("fc_count_sparse: variable %d appears twice", v);
                return FC_ERR_INVALID;
            }
        q.var[t] = v;
        q.stride[t] = (uint64_t)cells;
        cells *= db->arity[v];
    }
    if (cells >= ((unsigned __int128)1 << 63)) {
        set_error("fc_count_sparse: the key space of %d variables exceeds 2^63", k);
        return FC_ERR_RANGE;
    }
    hipStream_t s = (hipStream_t)stream;
    FC_HIP(hipSetDevice(db->device));
    const int64_t m = db->m;
    if (m == 0) {
        *nnz = 0;
        return FC_OK;
    }
    unsigned end_bit = 1;
    while (end_bit < 64 && ((uint64_t)1 << end_bit) < (uint64_t)cells) ++end_bit;
    DevBuf dk, ds, du, dc, dn, dt;
    FC_HIP(dk.alloc(sizeof(uint64_t) * (size_t)m, s));
    FC_HIP(ds.alloc(sizeof(uint64_t) * (size_t)m, s));
    FC_HIP(du.alloc(sizeof(uint64_t) * (size_t)m, s));
    FC_HIP(dc.alloc(sizeof(uint32_t) * (size_t)m, s));
    FC_HIP(dn.alloc(sizeof(uint32_t), s));
    uint64_t *kin = (uint64_t *)dk.p, *ksort = (uint64_t *)ds.p, *uniq = (uint64_t *)du.p;
    uint32_t *cnt = (uint32_t *)dc.p, *nruns = (uint32_t *)dn.p;
    size_t t_sort = 0, t_rle = 0;
    FC_HIP(rocprim::radix_sort_keys(nullptr, t_sort, kin, ksort, (size_t)m, 0u, end_bit, s));
    FC_HIP(rocprim::run_length_encode(nullptr, t_rle, ksort, (unsigned)m, uniq, cnt, nruns, s));
    FC_HIP(dt.alloc(std::max(t_sort, t_rle), s));
    {
        ProfScope ps("k_keys+sort+rle", s, (double)k * (double)m, 0.0);
        const int64_t blocks = std::min<int64_t>((m + 255) / 256, 16 * (int64_t)db->cu_count);
        hipLaunchKernelGGL(k_keys, dim3((unsigned)blocks), dim3(256), 0, s, db->d_cols, m,
                           db->m_pad, q, k, kin);
        FC_HIP(hipGetLastError());
        FC_HIP(rocprim::radix_sort_keys(dt.p, t_sort, kin, ksort, (size_t)m, 0u, end_bit, s));
        FC_HIP(rocprim::run_length_encode(dt.p, t_rle, ksort, (unsigned)m, uniq, cnt, nruns, s));
        ps.end(s);
    }
    uint32_t h = 0;
    FC_HIP(hipMemcpyAsync(&h, nruns, sizeof h, hipMemcpyDeviceToHost, s));
    FC_HIP(hipStreamSynchronize(s));
    *nnz = h;
    const int64_t n_out = std::min<int64_t>(h, cap);
    if (n_out > 0) {
        const bool kd = is_device_ptr(keys), cd = is_device_ptr(counts);
        FC_HIP(hipMemcpyAsync(keys, uniq, sizeof(int64_t) * (size_t)n_out,
                              kd ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
        if (cd) {
            hipLaunchKernelGGL(k_u32_to_i32, dim3((unsigned)std::min<int64_t>((n_out + 255) / 256, 4096)),
                               dim3(256), 0, s, cnt, n_out, counts);
            FC_HIP(hipGetLastError());
        } else {
            FC_HIP(hipMemcpyAsync(counts, cnt, sizeof(int32_t) * (size_t)n_out,
                                  hipMemcpyDeviceToHost, s));
        }
        FC_HIP(hipStreamSynchronize(s));
    }
    return FC_OK;
}

namespace {

int sparse_bits(const fc_db *db, const int32_t *vars, int32_t k, const char *who, BatchSpec *spec,
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

// One group of queries [q0, q0+G) through sort and run-length encoding.
template <typename K>
int sparse_group(fc_db *db, const BatchSpec *d_specs, int32_t G, int32_t B, int64_t *d_total,
                 int64_t *d_off, int64_t *keys, int32_t *counts, int64_t cap, int32_t *d_overflow,
                 double alg_bytes, hipStream_t s) {
    const int64_t m = db->m, nk = (int64_t)G * m;
    const unsigned end_bit = (unsigned)std::max<int32_t>(1, B + bits_for(G));
    DevBuf dk, ds, du, dc, dn, dt;
    FC_HIP(dk.alloc(sizeof(K) * (size_t)nk, s));
    FC_HIP(ds.alloc(sizeof(K) * (size_t)nk, s));
    FC_HIP(du.alloc(sizeof(K) * (size_t)nk, s));
    FC_HIP(dc.alloc(sizeof(uint32_t) * (size_t)nk, s));
    FC_HIP(dn.alloc(sizeof(uint32_t), s));
    K *kin = (K *)dk.p, *ksort = (K *)ds.p, *uniq = (K *)du.p;
    uint32_t *cnt = (uint32_t *)dc.p, *nruns = (uint32_t *)dn.p;
    size_t t_sort = 0, t_rle = 0;
    FC_HIP(rocprim::radix_sort_keys(nullptr, t_sort, kin, ksort, (size_t)nk, 0u, end_bit, s));
    FC_HIP(rocprim::run_length_encode(nullptr, t_rle, ksort, (unsigned)nk, uniq, cnt, nruns, s));
    FC_HIP(dt.alloc(std::max(t_sort, t_rle), s));
    const char *name = sizeof(K) == 4 ? "k_keys_batch+sort+rle<u32>" : "k_keys_batch+sort+rle<u64>";
    ProfScope ps(name, s, alg_bytes, 0.0);
    const int64_t bx = std::max<int64_t>(1, std::min<int64_t>((m + 255) / 256,
                                                               (16 * (int64_t)db->cu_count + G - 1) / G));
    hipLaunchKernelGGL(k_keys_batch<K>, dim3((unsigned)bx, (unsigned)G), dim3(256), 0, s,
                       db->d_cols, m, db->m_pad, d_specs, B, kin);
    FC_HIP(hipGetLastError());
    FC_HIP(rocprim::radix_sort_keys(dt.p, t_sort, kin, ksort, (size_t)nk, 0u, end_bit, s));
    FC_HIP(rocprim::run_length_encode(dt.p, t_rle, ksort, (unsigned)nk, uniq, cnt, nruns, s));
    const K mask = B >= (int32_t)(8 * sizeof(K)) ? ~(K)0 : (((K)1 << B) - 1);
    const int64_t eb = std::min<int64_t>((nk + 255) / 256, 16 * (int64_t)db->cu_count);
    hipLaunchKernelGGL(k_emit_runs<K>, dim3((unsigned)std::max<int64_t>(1, eb)), dim3(256), 0, s,
                       uniq, cnt, nruns, d_total, mask, keys, counts, cap, d_overflow);
    FC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_group_offsets<K>, dim3(1), dim3(256), 0, s, uniq, nruns, G, B, d_total,
                       d_off);
    FC_HIP(hipGetLastError());
    ps.end(s);
    return FC_OK;
}

}  // namespace

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
        const int rc = sparse_bits(db, vars_flat + var_off[i], (int32_t)k, who, &specs[(size_t)i],
                                   &qbits[(size_t)i]);
        if (rc != FC_OK) return rc;
    }
    const int64_t m = db->m;
    if (nq == 0 || m == 0) {
        for (int64_t i = 0; i <= nq; ++i) out_off[i] = 0;
        *total_nnz = 0;
        return FC_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    FC_HIP(hipSetDevice(db->device));
    // groups of consecutive queries: composite keys within 64 bits, at most
    // kGroupKeys keys (m alone when m is larger)
    constexpr int64_t kGroupKeys = int64_t(1) << 26;
    constexpr int32_t kGroupMax = 65535;  // queries of a group: the grid's y extent
    std::vector<std::pair<int64_t, int32_t>> groups;  // (first query, size)
    std::vector<int32_t> gbits;
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
        groups.push_back({i, G});
        gbits.push_back(B);
        i += G;
    }
    const bool kd = is_device_ptr(keys), cd = is_device_ptr(counts);
    if (cap > 0 && kd != cd) {
        set_error("%s: keys and counts must both be device or both host memory", who);
        return FC_ERR_INVALID;
    }
    const int64_t dev_cap = cap > 0 ? (kd ? cap : std::min<int64_t>(cap, nq * m)) : 0;
    DevBuf dspec, dtot, doff, dovf, dko, dco;
    FC_HIP(dspec.alloc(sizeof(BatchSpec) * (size_t)nq, s));
    FC_HIP(dtot.alloc(sizeof(int64_t), s));
    FC_HIP(doff.alloc(sizeof(int64_t) * (size_t)(nq + 1), s));
    FC_HIP(dovf.alloc(sizeof(int32_t) * 2, s));
    int64_t *kout = keys;
    int32_t *cout_ = counts;
    if (cap > 0 && !kd) {
        FC_HIP(dko.alloc(sizeof(int64_t) * (size_t)dev_cap, s));
        FC_HIP(dco.alloc(sizeof(int32_t) * (size_t)dev_cap, s));
        kout = (int64_t *)dko.p;
        cout_ = (int32_t *)dco.p;
    }
    Staging *st = staging_acquire(sizeof(BatchSpec) * (size_t)nq);
    if (!st) {
        set_error("%s: pinned staging allocation failed", who);
        return FC_ERR_NOMEM;
    }
    std::memcpy(st->host, specs.data(), sizeof(BatchSpec) * (size_t)nq);
    const hipError_t ce = hipMemcpyAsync(dspec.p, st->host, sizeof(BatchSpec) * (size_t)nq,
                                         hipMemcpyHostToDevice, s);
    staging_release(st, s);
    FC_HIP(ce);
    FC_HIP(fill_zero_i32((int32_t *)dtot.p, 2, s));
    FC_HIP(fill_zero_i32((int32_t *)dovf.p, 2, s));
    const BatchSpec *d_specs = (const BatchSpec *)dspec.p;
    int64_t *d_off = (int64_t *)doff.p;
    for (size_t g = 0; g < groups.size(); ++g) {
        const int64_t q0 = groups[g].first;
        const int32_t G = groups[g].second, B = gbits[g];
        double alg = 0.0;  // the group's columns, one byte per variable and instance
        for (int32_t j = 0; j < G; ++j) alg += (double)specs[(size_t)(q0 + j)].k * (double)m;
        // every group but the last writes off[q0 .. q0+G]; the next group
        // rewrites off[q0+G] with the same value
        const int rc = (B + bits_for(G) <= 32)
            ? sparse_group<uint32_t>(db, d_specs + q0, G, B, (int64_t *)dtot.p, d_off + q0, kout,
                                     cout_, dev_cap, (int32_t *)dovf.p, alg, s)
            : sparse_group<uint64_t>(db, d_specs + q0, G, B, (int64_t *)dtot.p, d_off + q0, kout,
                                     cout_, dev_cap, (int32_t *)dovf.p, alg, s);
        if (rc != FC_OK) return rc;
    }
    int64_t total = 0;
    int32_t ovf = 0;
    FC_HIP(hipMemcpyAsync(out_off, d_off, sizeof(int64_t) * (size_t)(nq + 1),
                          hipMemcpyDeviceToHost, s));
    FC_HIP(hipMemcpyAsync(&total, dtot.p, sizeof total, hipMemcpyDeviceToHost, s));
    FC_HIP(hipMemcpyAsync(&ovf, dovf.p, sizeof ovf, hipMemcpyDeviceToHost, s));
    FC_HIP(hipStreamSynchronize(s));
    *total_nnz = total;
    if (ovf || total > cap) {
        set_error("%s: %lld configurations do not fit cap = %lld (out_off and total_nnz are set; "
                  "keys and counts are unspecified)", who, (long long)total, (long long)cap);
        return FC_ERR_RANGE;
    }
    if (total > 0 && !kd) {
        FC_HIP(hipMemcpyAsync(keys, kout, sizeof(int64_t) * (size_t)total, hipMemcpyDeviceToHost, s));
        FC_HIP(hipMemcpyAsync(counts, cout_, sizeof(int32_t) * (size_t)total,
                              hipMemcpyDeviceToHost, s));
        FC_HIP(hipStreamSynchronize(s));
    }
    return FC_OK;
}
