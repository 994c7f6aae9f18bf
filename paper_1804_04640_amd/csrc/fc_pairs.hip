// All-pairs co-occurrence counts of binary items and association-rule pair
// records (Section 4.3: support and confidence of rules between two items).
//
// The count of every pair Count(X_a = 1 AND X_b = 1) is one entry of the
// Gram matrix A^T A of the m x n one-hot {0,1} instance-by-item matrix, a
// dense contraction over the instances.  It runs on int8 MFMA with exact
// int32 accumulation (counts < 2^31): the item bit-vectors of state 1 are
// expanded to one byte per instance on chip, never materialised in HBM.
//  * tiles of 128 x 128 items, upper block triangle only (the matrix is
//    symmetric); split-K over the instances, partial tiles summed with int32
//    atomics;
//  * per K step each workgroup expands 4 words (256 instances) of its 2 x 128
//    items into LDS panels, 4 waves each run a 4 x 4 grid of
//    16x16x64 i8 MFMAs on their 64 x 64 quarter of the tile;
//  * the (tile, split) order is XCD aware: one XCD works through one row
//    range of every tile pair, so a split's bit-vectors stay in its L2.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fc_internal.h"

namespace fc {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kGT = 128;                 // items per tile side
constexpr int kGW = 2;                   // 64-instance words per K step
constexpr int kPanel = kGW * 4 * kGT * 16;  // bytes: [word][group][item][16]

__device__ __forceinline__ void map_pair(int64_t b, int32_t npairs, int32_t splits, int32_t &p,
                                         int32_t &sp) {
    if (splits % kXcds == 0) {
        int32_t x = (int32_t)(b % kXcds);
        int64_t t = b / kXcds;
        p = (int32_t)(t % npairs);
        sp = (int32_t)(t / npairs) * kXcds + x;
    } else {
        p = (int32_t)(b / splits);
        sp = (int32_t)(b % splits);
    }
}

// 16 instance bits -> 16 bytes of 0/1 (instance order = byte order).
__device__ __forceinline__ uint4 expand16(uint32_t b) {
    uint4 r;
    r.x = ((b & 0xFu) * 0x00204081u) & 0x01010101u;
    r.y = (((b >> 4) & 0xFu) * 0x00204081u) & 0x01010101u;
    r.z = (((b >> 8) & 0xFu) * 0x00204081u) & 0x01010101u;
    r.w = (((b >> 12) & 0xFu) * 0x00204081u) & 0x01010101u;
    return r;
}

__global__ __launch_bounds__(256) void k_gram(const uint64_t *__restrict__ bits, int64_t words,
                                              const int32_t *__restrict__ rowidx, int32_t ntiles,
                                              int32_t npairs, int32_t splits,
                                              int32_t *__restrict__ C, int32_t ldc) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    int32_t p, sp;
    map_pair(blockIdx.x, npairs, splits, p, sp);
    int32_t I = 0, J = 0;
    {  // pair index -> (I, J) with I <= J
        int32_t rem = p;
        while (rem >= ntiles - I) {
            rem -= ntiles - I;
            ++I;
        }
        J = I + rem;
    }
    const bool diag = I == J;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int item = t >> 1, half = t & 1;
    const int32_t ra = rowidx[I * kGT + item];
    const int32_t rb = rowidx[J * kGT + item];
    const uint64_t *pa = bits + (int64_t)(ra < 0 ? 0 : ra) * words;
    const uint64_t *pb = bits + (int64_t)(rb < 0 ? 0 : rb) * words;

    const int64_t tiles = words / (kTileRows / 64);
    const int64_t w0 = (int64_t)sp * tiles / splits * (kTileRows / 64);
    const int64_t w1 = (int64_t)(sp + 1) * tiles / splits * (kTileRows / 64);

    v4i acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4i{0, 0, 0, 0};

    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    const int grp = lane >> 4, col = lane & 15;
    // Double-buffered panels (A and B of buffer `cur` at lds + cur * 2 * kPanel)
    // and register prefetch of the next step's words: one barrier per step.
    uint64_t xa[kGW], xb[kGW];
#pragma unroll
    for (int g = 0; g < kGW; ++g) {
        xa[g] = (ra >= 0 && w0 < w1) ? pa[w0 + g] : 0ull;
        xb[g] = (rb >= 0 && w0 < w1 && !diag) ? pb[w0 + g] : 0ull;
    }
    int cur = 0;
    for (int64_t w = w0; w < w1; w += kGW) {  // (w1 - w0) is a multiple of 64 words
        uint8_t *PA = lds + cur * 2 * kPanel;
        uint8_t *PB = diag ? PA : PA + kPanel;
#pragma unroll
        for (int g = 0; g < kGW; ++g) {
            const uint32_t va = (uint32_t)(xa[g] >> (32 * half));
            const uint32_t vb = (uint32_t)(xb[g] >> (32 * half));
#pragma unroll
            for (int gg = 0; gg < 2; ++gg) {
                const int group = 2 * half + gg;
                const int off = ((g * 4 + group) * kGT + item) * 16;
                *reinterpret_cast<uint4 *>(PA + off) = expand16((va >> (16 * gg)) & 0xFFFFu);
                if (!diag)
                    *reinterpret_cast<uint4 *>(PB + off) = expand16((vb >> (16 * gg)) & 0xFFFFu);
            }
        }
        if (w + kGW < w1) {  // next step's words, in flight during the MFMAs
#pragma unroll
            for (int g = 0; g < kGW; ++g) {
                xa[g] = ra >= 0 ? pa[w + kGW + g] : 0ull;
                xb[g] = (rb >= 0 && !diag) ? pb[w + kGW + g] : 0ull;
            }
        }
        __syncthreads();  // panels of `cur` complete; the other buffer is free
#pragma unroll
        for (int g = 0; g < kGW; ++g) {
            v4i a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = *reinterpret_cast<const v4i *>(PA + ((g * 4 + grp) * kGT + wr + i * 16 + col) * 16);
                b[i] = *reinterpret_cast<const v4i *>(PB + ((g * 4 + grp) * kGT + wc + i * 16 + col) * 16);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        cur ^= 1;
    }
    // D layout of a 16x16 MFMA tile: lane l, element e -> row 4*(l/16)+e, column l%16
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int32_t v = acc[i][j][e];
                if (v) {
                    const int64_t row = (int64_t)I * kGT + wr + i * 16 + 4 * grp + e;
                    const int64_t cc = (int64_t)J * kGT + wc + j * 16 + col;
                    atomicAdd(&C[row * ldc + cc], v);
                }
            }
}

// Number of qualifying pairs (a < b, n_ab >= nmin) of every row a.
__global__ void k_pair_count(const int32_t *__restrict__ C, int32_t ldc, int32_t ni, int32_t nmin,
                             int32_t *__restrict__ cnt) {
    const int lane = threadIdx.x & 63;
    const int32_t a = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (a >= ni) return;
    int32_t c = 0;
    for (int32_t b = a + 1 + lane; b < ni; b += 64) c += C[(int64_t)a * ldc + b] >= nmin;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if (lane == 0) cnt[a] = c;
}

// Writes the records of every row a at its offset, in increasing b.
__global__ void k_pair_write(const int32_t *__restrict__ C, int32_t ldc, int32_t ni, int32_t nmin,
                             const int64_t *__restrict__ off, int64_t cap, float inv_m,
                             fc_pair_rec *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int32_t a = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (a >= ni) return;
    int64_t base = off[a];
    const int32_t na = C[(int64_t)a * ldc + a];
    for (int32_t b0 = a + 1; b0 < ni; b0 += 64) {
        const int32_t b = b0 + lane;
        const int32_t v = b < ni ? C[(int64_t)a * ldc + b] : 0;
        const bool f = b < ni && v >= nmin;
        const uint64_t mask = __ballot(f);
        const int64_t pos = base + __popcll(mask & ((1ull << lane) - 1ull));
        if (f && pos < cap) {
            const int32_t nb = C[(int64_t)b * ldc + b];
            fc_pair_rec r;
            r.a = a;
            r.b = b;
            r.n_ab = v;
            r.support = (float)v * inv_m;
            r.conf_ab = (float)v / (float)na;
            r.conf_ba = (float)v / (float)nb;
            out[pos] = r;
        }
        base += __popcll(mask);
    }
}

// Full symmetric output from the computed upper triangle.
__global__ void k_mirror(const int32_t *__restrict__ C, int32_t ldc, int32_t ni,
                         int32_t *__restrict__ G) {
    const int64_t n2 = (int64_t)ni * ni;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = (int32_t)(i / ni), b = (int32_t)(i % ni);
        G[i] = a <= b ? C[(int64_t)a * ldc + b] : C[(int64_t)b * ldc + a];
    }
}

}  // namespace

}  // namespace fc

using namespace fc;

extern "C" int fc_pairs(fc_db *db, const int32_t *items, int32_t ni, double minsup, int32_t *gram,
                        fc_pair_rec *out, int64_t cap, int64_t *n_out, void *stream) {
    clear_error();
    if (!db || !n_out || ni < 1 || cap < 0 || (cap > 0 && !out)) {
        set_error("fc_pairs: need a database, ni >= 1, n_out, and out when cap > 0");
        return FC_ERR_INVALID;
    }
    if (!db->d_bits) {
        set_error("fc_pairs needs a database created with FC_DB_BITVECTORS");
        return FC_ERR_INVALID;
    }
    if (!(minsup >= 0.0) || !std::isfinite(minsup)) {
        set_error("fc_pairs: minsup must be a finite value >= 0");
        return FC_ERR_INVALID;
    }
    if (!items && ni != db->n) {
        set_error("fc_pairs: items is NULL but ni=%d != n=%d", ni, db->n);
        return FC_ERR_INVALID;
    }
    const int32_t ntiles = (ni + kGT - 1) / kGT;
    const int32_t np = ntiles * kGT;
    std::vector<int32_t> rowidx((size_t)np, -1);
    std::vector<uint8_t> seen((size_t)db->n, 0);
    for (int32_t i = 0; i < ni; ++i) {
        const int32_t v = items ? items[i] : i;
        if (v < 0 || v >= db->n) {
            set_error("fc_pairs: item %d: variable %d out of range", i, v);
            return FC_ERR_INVALID;
        }
        if (db->arity[v] != 2) {
            set_error("fc_pairs: item %d: variable %d has arity %d, items must be binary", i, v,
                      db->arity[v]);
            return FC_ERR_INVALID;
        }
        if (seen[v]++) {
            set_error("fc_pairs: item %d: variable %d listed twice", i, v);
            return FC_ERR_INVALID;
        }
        rowidx[(size_t)i] = db->state_off[v] + 1;  // bit-vector of state 1
    }
    // smallest count whose support n/m exceeds minsup, decided in binary64
    const double m = (double)db->m;
    int64_t nmin = (int64_t)std::floor(minsup * m) - 2;
    if (nmin < 0) nmin = 0;
    while (!((double)nmin / m > minsup) && nmin <= db->m) ++nmin;
    if (db->m == 0) nmin = 1;  // no instance: no pair has support
    hipStream_t s = (hipStream_t)stream;
    FC_HIP(hipSetDevice(db->device));
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_gram, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  4 * kPanel);
        (void)hipGetLastError();
        attr = true;
    }
    DevBuf dC, dRow, dCnt, dOff, dRec, dG;
    const int64_t ldc = np;
    FC_HIP(dC.alloc(sizeof(int32_t) * (size_t)np * (size_t)np, s));
    FC_HIP(dRow.alloc(sizeof(int32_t) * (size_t)np, s));
    FC_HIP(hipMemcpyAsync(dRow.p, rowidx.data(), sizeof(int32_t) * (size_t)np,
                          hipMemcpyHostToDevice, s));
    int32_t *C = (int32_t *)dC.p;
    FC_HIP(fill_zero_i32(C, (int64_t)np * np, s));
    const int32_t npairs = ntiles * (ntiles + 1) / 2;
    const int64_t tiles = db->words / (kTileRows / 64);
    int64_t splits = (4 * (int64_t)db->cu_count + npairs - 1) / npairs;
    splits = std::max<int64_t>(splits, 64);
    splits = std::min<int64_t>(splits, tiles);
    if (splits >= kXcds) splits -= splits % kXcds;
    if (splits < 1) splits = 1;
    if (db->m > 0) {
        const double ops = 2.0 * (double)db->m * (double)ni * (double)(ni + 1) / 2.0;
        ProfScope ps("k_gram", s, 0.0, ops);
        hipLaunchKernelGGL(k_gram, dim3((unsigned)(npairs * splits)), dim3(256), 4 * kPanel, s,
                           db->d_bits, db->words, (const int32_t *)dRow.p, ntiles, npairs,
                           (int32_t)splits, C, (int32_t)ldc);
        FC_HIP(hipGetLastError());
        ps.end(s);
    }
    // records: per-row counts -> offsets (host) -> ordered writes
    FC_HIP(dCnt.alloc(sizeof(int32_t) * (size_t)ni, s));
    hipLaunchKernelGGL(k_pair_count, dim3((unsigned)((ni + 3) / 4)), dim3(256), 0, s, C,
                       (int32_t)ldc, ni, (int32_t)std::min<int64_t>(nmin, INT32_MAX),
                       (int32_t *)dCnt.p);
    FC_HIP(hipGetLastError());
    std::vector<int32_t> cnt((size_t)ni);
    FC_HIP(hipMemcpyAsync(cnt.data(), dCnt.p, sizeof(int32_t) * (size_t)ni,
                          hipMemcpyDeviceToHost, s));
    FC_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> off((size_t)ni + 1, 0);
    for (int32_t a = 0; a < ni; ++a) off[(size_t)a + 1] = off[(size_t)a] + cnt[(size_t)a];
    const int64_t total = off[(size_t)ni];
    *n_out = total;
    const int64_t nrec = std::min(total, cap);
    if (nrec > 0) {
        const bool odev = is_device_ptr(out);
        FC_HIP(dOff.alloc(sizeof(int64_t) * (size_t)ni, s));
        FC_HIP(hipMemcpyAsync(dOff.p, off.data(), sizeof(int64_t) * (size_t)ni,
                              hipMemcpyHostToDevice, s));
        fc_pair_rec *rec = out;
        if (!odev) {
            FC_HIP(dRec.alloc(sizeof(fc_pair_rec) * (size_t)nrec, s));
            rec = (fc_pair_rec *)dRec.p;
        }
        hipLaunchKernelGGL(k_pair_write, dim3((unsigned)((ni + 3) / 4)), dim3(256), 0, s, C,
                           (int32_t)ldc, ni, (int32_t)std::min<int64_t>(nmin, INT32_MAX),
                           (const int64_t *)dOff.p, nrec, (float)(1.0 / m), rec);
        FC_HIP(hipGetLastError());
        if (!odev)
            FC_HIP(hipMemcpyAsync(out, rec, sizeof(fc_pair_rec) * (size_t)nrec,
                                  hipMemcpyDeviceToHost, s));
    }
    if (gram) {
        const bool gdev = is_device_ptr(gram);
        int32_t *G = gram;
        if (!gdev) {
            FC_HIP(dG.alloc(sizeof(int32_t) * (size_t)ni * (size_t)ni, s));
            G = (int32_t *)dG.p;
        }
        const int64_t n2 = (int64_t)ni * ni;
        hipLaunchKernelGGL(k_mirror, dim3((unsigned)std::min<int64_t>((n2 + 255) / 256, 65536)),
                           dim3(256), 0, s, C, (int32_t)ldc, ni, G);
        FC_HIP(hipGetLastError());
        if (!gdev)
            FC_HIP(hipMemcpyAsync(gram, G, sizeof(int32_t) * (size_t)n2, hipMemcpyDeviceToHost, s));
    }
    FC_HIP(hipStreamSynchronize(s));
    return FC_OK;
}
