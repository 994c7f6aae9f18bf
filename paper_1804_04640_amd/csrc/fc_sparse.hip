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
