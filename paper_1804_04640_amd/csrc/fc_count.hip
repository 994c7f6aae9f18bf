// Counting kernels, the batch planner and the counting entry points.
//
// Three exact strategies produce identical tables (the numbers of the
// Section 2 definition):
//  * HIST: every instance's states form one mixed-radix key (the digits of
//    the MSD radix of Section 3.3, child least significant) and the key's
//    cell is incremented in an LDS histogram.  Each cell owns up to 64
//    consecutive words (one per lane slot, as many as the LDS allows), so
//    lanes of a wave add into different banks whatever their keys.  Keys of
//    tables up to 256 cells form as bytes (four instances per packed
//    multiply-add), up to 16,383 cells as 16-bit LDS addresses (two per
//    packed multiply-add); databases whose arities are all at most 16 are
//    also read from a 4-bit packed copy of the columns.
//  * BITMAP: the per-state bit-vectors of the query's variables are ANDed
//    down the configuration tree of Alg. 1 and the leaves are popcounted; a
//    subtree whose prefix is empty in every lane of the wave is pruned, as
//    Alg. 1 prunes a zero intersection.  The tree is walked on chip for a
//    few 64-row words per thread at a time, never stored.
//  * PARTITION: tables too large for LDS are split by their top key digits
//    into parts that fit (the MSD partition of Section 3.3): one pass over
//    the columns forms every key and histograms its part, the keys are moved
//    to their parts, and each part is an LDS histogram.  Tables beyond 2^25
//    cells (or whose scratch would not fit) fall back to key windows, each
//    an LDS histogram of a full scan that keeps the keys falling in it.
// Partial tables of row chunks are summed into the output with int32
// atomics, which is exact and order independent.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "fc_internal.h"

namespace fc {

constexpr int kHistMaxCells = 40000;  // generic kernel: odd row stride * 4 B <= 160 KiB
constexpr int32_t kPersistentLds = 64 * 64 * 4;  // groups up to this LDS share one launch
constexpr int64_t kGramBlock = 256;     // Gram rows come in whole column blocks
constexpr int64_t kGramMaxRows = 4096;  // state Gram at most 4096 x 4096 (64 MiB)

__device__ __forceinline__ void map_block(int64_t b, int32_t nd, int32_t chunks, int32_t &d,
                                          int32_t &c) {
    // XCD-aware order: blocks are dealt round-robin to the 8 XCDs, so block
    // b runs on XCD b % 8.  When chunks is a multiple of 8, XCD x works on
    // chunks x, x+8, ... of every descriptor in turn, keeping one row range
    // of all columns hot in its own L2.
    if (chunks % kXcds == 0) {
        int32_t x = (int32_t)(b % kXcds);
        int64_t t = b / kXcds;
        int32_t phase = (int32_t)(t / nd);
        d = (int32_t)(t % nd);
        c = phase * kXcds + x;
    } else {
        d = (int32_t)(b / chunks);
        c = (int32_t)(b % chunks);
    }
}

// A state column as a buffer resource: the loads of all K columns share one
// 32-bit vector offset (m_pad <= 2^31) and differ only in scalar registers,
// and a load past the column's end returns zeros instead of faulting.
typedef __amdgpu_buffer_rsrc_t Col;
__device__ __forceinline__ Col make_col(const uint8_t *p, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(p), (short)0, (int)bytes,
                                             0x00020000 /* 32-bit data format */);
}
__device__ __forceinline__ uint4 load16(Col c, uint32_t off) {
    return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(c, off, 0, 0));
}

__device__ __forceinline__ uint32_t byte_of(const uint4 &v, int i) {
    uint32_t w = (i < 4) ? v.x : (i < 8) ? v.y : (i < 12) ? v.z : v.w;
    return (w >> ((i & 3) * 8)) & 0xFFu;
}

// LDS histogram count of one descriptor over one row chunk.
// SMALL: every stride is below 2^24, so 24-bit multiplies suffice.
template <int K, bool SMALL>
__device__ __forceinline__ void hist_body(const uint8_t *__restrict__ cols, int64_t pitch,
                                          const uint8_t *__restrict__ arity, const QDesc &q,
                                          int32_t c, int32_t chunks, int32_t lds_words,
                                          int32_t pad_rows, int32_t *__restrict__ tables,
                                          uint32_t *lds) {
    const int32_t win_base = q.win_base;
    const uint32_t win = (uint32_t)q.win_cells;

    uint32_t stride[K];
    Col colp[K];
    {
        uint32_t s = 1;
#pragma unroll
        for (int t = K - 1; t >= 0; --t) {
            int32_t v = q.var[t];
            stride[t] = s;
            s *= arity[v];
            colp[t] = make_col(cols + (int64_t)v * pitch, pitch);
        }
    }
    const int32_t cs = (int32_t)(win | 1u);
    int32_t copies = lds_words / cs;
    copies = copies >= 64 ? 64 : copies >= 32 ? 32 : copies >= 16 ? 16 : copies >= 8 ? 8
           : copies >= 4 ? 4 : copies >= 2 ? 2 : 1;
    for (int32_t i = threadIdx.x; i < copies * cs; i += kBlock) lds[i] = 0;
    __syncthreads();

    const int64_t tiles = q.tiles;
    const int64_t r0 = (int64_t)c * tiles / chunks * kTileRows;
    const int64_t r1 = (int64_t)(c + 1) * tiles / chunks * kTileRows;
    uint32_t *h = lds + (threadIdx.x & (copies - 1)) * cs;

    for (uint32_t row = (uint32_t)r0 + threadIdx.x * 16u; row < (uint32_t)r1; row += kBlock * 16u) {
        uint4 v[K];
#pragma unroll
        for (int t = 0; t < K; ++t) v[t] = load16(colp[t], row);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            uint32_t key = 0;
#pragma unroll
            for (int t = 0; t < K; ++t) {
                uint32_t b = byte_of(v[t], i);
                key += SMALL ? __umul24(b, stride[t]) : b * stride[t];
            }
            key -= (uint32_t)win_base;
            if (key < win) atomicAdd(&h[key], 1u);
        }
    }
    __syncthreads();
    const bool has_pad = (r1 == tiles * kTileRows) && (r0 < r1) && win_base == 0;
    int32_t *out = tables + q.table_off + win_base;
    for (int32_t cell = threadIdx.x; cell < (int32_t)win; cell += kBlock) {
        uint32_t sum = 0;
        for (int32_t p = 0; p < copies; ++p) sum += lds[p * cs + cell];
        if (cell == 0 && has_pad) sum -= (uint32_t)pad_rows;  // padding rows are key 0
        if (chunks == 1) out[cell] = (int32_t)sum;  // the window's only workgroup
        else if (sum) atomicAdd(&out[cell], (int32_t)sum);
    }
}

template <int K, bool SMALL>
__global__ __launch_bounds__(kBlock) void k_hist(const uint8_t *__restrict__ cols, int64_t pitch,
                                                 const uint8_t *__restrict__ arity,
                                                 const QDesc *__restrict__ descs, int32_t nd,
                                                 int32_t chunks, int32_t lds_words,
                                                 int32_t pad_rows, int32_t *__restrict__ tables) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    int32_t di, c;
    map_block(blockIdx.x, nd, chunks, di, c);
    hist_body<K, SMALL>(cols, pitch, arity, descs[di], c, chunks, lds_words, pad_rows, tables, lds);
}

// One-pass partition (Section 3.3, Alg. 3's buckets) for tables beyond the
// LDS classes: the query's columns are read once to form every instance's
// key, which goes to a key buffer while its part (key >> kPartBits) is
// histogrammed; the parts are laid out by a scan, the keys moved to their
// part as 16-bit offsets within it, and each part is then counted in LDS,
// 2^kPartBits cells at a time.  Per query the scratch holds PartQ's arrays.
constexpr int kPartBits = 13;                  // cells per part (32 KiB of LDS counters)
constexpr int32_t kPartCells = 1 << kPartBits;
constexpr int32_t kPartMax = 4096;             // parts per query: tables up to 2^25 cells
constexpr int64_t kPartUnit = 65536;           // keys per counting work unit
constexpr int64_t kPartTile = kBlock * 16;     // rows per workgroup step (16 per thread)
constexpr size_t kPartBudget = size_t(512) << 20;  // scratch of one slice of queries

struct PartQ {
    uint32_t *cnt, *start, *cursor, *ustart;  // [kPartMax] each, ustart [kPartMax + 1]
    uint32_t *keys;                           // [m]
    uint16_t *low;                            // [m]
};

__host__ __device__ inline size_t part_qbytes(int64_t m) {
    const size_t head = sizeof(uint32_t) * (4 * (size_t)kPartMax + 4);
    return ((head + 4 * (size_t)m + 255) & ~(size_t)255) + ((2 * (size_t)m + 255) & ~(size_t)255);
}

__device__ __forceinline__ PartQ part_slots(char *q, int64_t m) {
    PartQ P;
    P.cnt = (uint32_t *)q;
    P.start = P.cnt + kPartMax;
    P.cursor = P.start + kPartMax;
    P.ustart = P.cursor + kPartMax;
    const size_t head = sizeof(uint32_t) * (4 * (size_t)kPartMax + 4);
    P.keys = (uint32_t *)(q + head);
    P.low = (uint16_t *)(q + ((head + 4 * (size_t)m + 255) & ~(size_t)255));
    return P;
}

// Keys of every instance (the query's columns read once) and the parts'
// sizes.  Grid: (workgroups per query, queries of the slice).
__global__ __launch_bounds__(kBlock) void k_part_keys(const uint8_t *__restrict__ cols,
                                                      int64_t pitch,
                                                      const uint8_t *__restrict__ arity,
                                                      const QDesc *__restrict__ descs, int64_t m,
                                                      char *__restrict__ scratch, size_t qstride) {
    __shared__ uint32_t h[kPartMax];
    const QDesc q = descs[blockIdx.y];
    const PartQ P = part_slots(scratch + blockIdx.y * qstride, m);
    const int32_t nparts = (q.cells + kPartCells - 1) >> kPartBits;
    uint32_t stride[FC_MAX_VARS];
    Col colp[FC_MAX_VARS];
    {
        uint32_t sacc = 1;
#pragma unroll
        for (int t = FC_MAX_VARS - 1; t >= 0; --t) {
            if (t < q.k) {
                const int32_t v = q.var[t];
                stride[t] = sacc;
                sacc *= arity[v];
                colp[t] = make_col(cols + (int64_t)v * pitch, pitch);
            } else {
                stride[t] = 0;
                colp[t] = make_col(cols, 0);
            }
        }
    }
    for (int32_t i = threadIdx.x; i < nparts; i += kBlock) h[i] = 0;
    __syncthreads();
    for (int64_t r0 = (int64_t)blockIdx.x * kPartTile + threadIdx.x * 16; r0 < m;
         r0 += (int64_t)gridDim.x * kPartTile) {
        uint32_t key[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) key[i] = 0;
#pragma unroll
        for (int t = 0; t < FC_MAX_VARS; ++t) {
            if (t < q.k) {
                const uint4 v = load16(colp[t], (uint32_t)r0);
#pragma unroll
                for (int i = 0; i < 16; ++i) key[i] += byte_of(v, i) * stride[t];
            }
        }
        if (r0 + 16 <= m) {
            uint4 *o = reinterpret_cast<uint4 *>(P.keys + r0);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                o[i] = make_uint4(key[4 * i], key[4 * i + 1], key[4 * i + 2], key[4 * i + 3]);
#pragma unroll
            for (int i = 0; i < 16; ++i) atomicAdd(&h[key[i] >> kPartBits], 1u);
        } else {
            for (int i = 0; i < 16; ++i)
                if (r0 + i < m) {
                    P.keys[r0 + i] = key[i];
                    atomicAdd(&h[key[i] >> kPartBits], 1u);
                }
        }
    }
    __syncthreads();
    for (int32_t i = threadIdx.x; i < nparts; i += kBlock)
        if (h[i]) atomicAdd(&P.cnt[i], h[i]);
}

// Per query (one workgroup): part starts, scatter cursors, and the first
// counting unit of every part (kPartUnit keys per unit).
__global__ __launch_bounds__(kBlock) void k_part_scan(const QDesc *__restrict__ descs, int64_t m,
                                                      char *__restrict__ scratch, size_t qstride) {
    __shared__ uint32_t sk[kBlock], su[kBlock];
    const QDesc q = descs[blockIdx.x];
    const PartQ P = part_slots(scratch + blockIdx.x * qstride, m);
    const int32_t nparts = (q.cells + kPartCells - 1) >> kPartBits;
    const int32_t per = (nparts + kBlock - 1) / kBlock;
    const int32_t a = min(nparts, (int32_t)threadIdx.x * per), b = min(nparts, a + per);
    uint32_t k = 0, u = 0;
    for (int32_t i = a; i < b; ++i) {
        k += P.cnt[i];
        u += (uint32_t)((P.cnt[i] + kPartUnit - 1) / kPartUnit);
    }
    sk[threadIdx.x] = k;
    su[threadIdx.x] = u;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        const uint32_t xk = threadIdx.x >= (unsigned)o ? sk[threadIdx.x - o] : 0u;
        const uint32_t xu = threadIdx.x >= (unsigned)o ? su[threadIdx.x - o] : 0u;
        __syncthreads();
        sk[threadIdx.x] += xk;
        su[threadIdx.x] += xu;
        __syncthreads();
    }
    k = sk[threadIdx.x] - k;
    u = su[threadIdx.x] - u;
    for (int32_t i = a; i < b; ++i) {
        const uint32_t c = P.cnt[i];
        P.start[i] = k;
        P.cursor[i] = k;
        P.ustart[i] = u;
        k += c;
        u += (uint32_t)((c + kPartUnit - 1) / kPartUnit);
    }
    if (threadIdx.x == kBlock - 1) P.ustart[nparts] = su[kBlock - 1];
}

// Every key to its part, as its offset within the part.  A workgroup step
// ranks its keys per part in LDS, stages them there in part order, takes one
// cursor atomic per part, and writes each part's keys as one contiguous run
// (neighbouring threads, neighbouring addresses).
__global__ __launch_bounds__(kBlock) void k_part_scatter(const QDesc *__restrict__ descs,
                                                         int64_t m, char *__restrict__ scratch,
                                                         size_t qstride) {
    __shared__ uint32_t h[kPartMax], tstart[kPartMax];
    __shared__ uint32_t stage[kPartTile];
    __shared__ uint32_t wsum[kBlock / 64];
    const QDesc q = descs[blockIdx.y];
    const PartQ P = part_slots(scratch + blockIdx.y * qstride, m);
    const int32_t nparts = (q.cells + kPartCells - 1) >> kPartBits;
    const int32_t per = (nparts + kBlock - 1) / kBlock;  // parts per thread in the scan
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t t0 = (int64_t)blockIdx.x * kPartTile; t0 < m; t0 += (int64_t)gridDim.x * kPartTile) {
        for (int32_t i = threadIdx.x; i < nparts; i += kBlock) h[i] = 0;
        __syncthreads();
        const int64_t r0 = t0 + threadIdx.x * 16;
        uint32_t key[16], rank[16];
        if (r0 + 16 <= m) {
            const uint4 *src = reinterpret_cast<const uint4 *>(P.keys + r0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint4 v = src[i];
                key[4 * i] = v.x;
                key[4 * i + 1] = v.y;
                key[4 * i + 2] = v.z;
                key[4 * i + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) key[i] = r0 + i < m ? P.keys[r0 + i] : 0u;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i)
            rank[i] = r0 + i < m ? atomicAdd(&h[key[i] >> kPartBits], 1u) : 0u;
        __syncthreads();
        // the tile's part starts (exclusive scan of h) and the global bases
        const int32_t a = min(nparts, (int32_t)threadIdx.x * per), b = min(nparts, a + per);
        uint32_t sum = 0;
        for (int32_t i = a; i < b; ++i) sum += h[i];
        uint32_t incl = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t x = __shfl_up(incl, o);
            if (lane >= o) incl += x;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        uint32_t run = incl - sum;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) run += w < wave ? wsum[w] : 0u;
        for (int32_t i = a; i < b; ++i) {
            const uint32_t c = h[i];
            tstart[i] = run;
            h[i] = c ? atomicAdd(&P.cursor[i], c) : 0u;  // becomes the part's global base
            run += c;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (r0 + i < m) stage[tstart[key[i] >> kPartBits] + rank[i]] = key[i];
        __syncthreads();
        const int32_t nt = (int32_t)min((int64_t)kPartTile, m - t0);
        for (int32_t j = threadIdx.x; j < nt; j += kBlock) {
            const uint32_t k = stage[j];
            const uint32_t p = k >> kPartBits;
            P.low[h[p] + (uint32_t)j - tstart[p]] = (uint16_t)(k & (kPartCells - 1));
        }
        __syncthreads();
    }
}

// Counts the parts in LDS: workgroups stride over the query's counting units
// (unit j of part p: its keys [j * kPartUnit, (j + 1) * kPartUnit)), and add
// each unit's non-zero cells to the (zeroed) table.
__global__ __launch_bounds__(kBlock) void k_part_count(const QDesc *__restrict__ descs, int64_t m,
                                                       char *__restrict__ scratch, size_t qstride,
                                                       int32_t *__restrict__ tables) {
    __shared__ uint32_t win[kPartCells];
    const QDesc q = descs[blockIdx.y];
    const PartQ P = part_slots(scratch + blockIdx.y * qstride, m);
    const int32_t nparts = (q.cells + kPartCells - 1) >> kPartBits;
    const uint32_t units = P.ustart[nparts];
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
        int32_t lo = 0, hi = nparts - 1;  // the last part whose first unit is <= u
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (P.ustart[mid] <= u) lo = mid; else hi = mid - 1;
        }
        const int32_t p = lo;
        const int64_t a = (int64_t)P.start[p] + (int64_t)(u - P.ustart[p]) * kPartUnit;
        const int64_t b = min((int64_t)P.start[p] + (int64_t)P.cnt[p], a + kPartUnit);
        for (int32_t i = threadIdx.x; i < kPartCells; i += kBlock) win[i] = 0;
        __syncthreads();
        for (int64_t i = a + threadIdx.x; i < b; i += kBlock) atomicAdd(&win[P.low[i]], 1u);
        __syncthreads();
        const int32_t c0 = p << kPartBits;
        const int32_t nc = min(kPartCells, q.cells - c0);
        int32_t *out = tables + q.table_off + c0;
        for (int32_t i = threadIdx.x; i < nc; i += kBlock) {
            const uint32_t v = win[i];
            if (v) atomicAdd(&out[i], (int32_t)v);
        }
        __syncthreads();
    }
}

// Lane-column histograms: every cell owns B consecutive LDS words (B a power
// of two).  Zeroing and the flush use all threads and 16-byte accesses when
// B >= 4: B/4 consecutive threads read one cell's words, combine their sums
// with lane shuffles, and the first adds the cell's count to the table.
__device__ __forceinline__ void zero_cols(uint32_t *lds, int32_t words) {
    if ((words & 3) == 0) {
        uint4 *l4 = reinterpret_cast<uint4 *>(lds);
        for (int32_t i = threadIdx.x; i < words / 4; i += kBlock) l4[i] = make_uint4(0u, 0u, 0u, 0u);
    } else {
        for (int32_t i = threadIdx.x; i < words; i += kBlock) lds[i] = 0;
    }
}

// direct: this workgroup is the only one counting these cells (one row
// chunk), so every cell is stored, zeros included, and the table needs no
// zeroing first; otherwise non-zero partial counts are added atomically.
__device__ __forceinline__ void flush_cols(const uint32_t *lds, int32_t cells, int32_t B,
                                           bool has_pad, int32_t pad_rows, bool direct,
                                           int32_t *out) {
    if (B >= 4) {
        const int32_t per = B / 4;  // threads per cell: 1, 2, 4, 8 or 16
        const int32_t total = cells * per;
        const uint4 *l4 = reinterpret_cast<const uint4 *>(lds);
        for (int32_t b0 = 0; b0 < total; b0 += kBlock) {  // uniform trip count
            const int32_t i = b0 + (int32_t)threadIdx.x;
            uint32_t sum = 0;
            if (i < total) {
                const uint4 v = l4[i];
                sum = (v.x + v.y) + (v.z + v.w);
            }
            for (int32_t off = per / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
            if (i < total && (i & (per - 1)) == 0) {
                const int32_t cell = i / per;
                if (cell == 0 && has_pad) sum -= (uint32_t)pad_rows;  // padding rows are key 0
                if (direct) out[cell] = (int32_t)sum;
                else if (sum) atomicAdd(&out[cell], (int32_t)sum);
            }
        }
    } else {
        for (int32_t cell = threadIdx.x; cell < cells; cell += kBlock) {
            uint32_t sum = 0;
            for (int32_t j = 0; j < B; ++j) sum += lds[cell * B + j];
            if (cell == 0 && has_pad) sum -= (uint32_t)pad_rows;
            if (direct) out[cell] = (int32_t)sum;
            else if (sum) atomicAdd(&out[cell], (int32_t)sum);
        }
    }
}

// LDS histogram for tables whose lane columns fit 64 KiB (no key window):
// the key of two instances at a time is formed in the 16-bit halves of one
// register with packed multiply-adds, directly as an LDS byte address
// (strides are pre-scaled by 4 B and the lane's word offset is the
// accumulator's start).
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pk_mad_u16(uint32_t a, uint32_t b, uint32_t c) {
    const u16x2 x = __builtin_bit_cast(u16x2, a), y = __builtin_bit_cast(u16x2, b),
                z = __builtin_bit_cast(u16x2, c);
    return __builtin_bit_cast(uint32_t, (u16x2)(x * y + z));
}

// Row order inside a chunk (a synchronized sweep): the chunk's steps are
// taken cyclically from step (seq * n / sweep) mod n, where seq is the
// workgroup's place in its XCD's dispatch order (blocks are dealt to the
// XCDs round-robin) and sweep the number of workgroups one XCD holds at a
// time.  A workgroup then starts where the one whose slot it takes ended,
// so the workgroups resident on an XCD read nearly the same rows of the
// columns at any moment and share them in that XCD's L2, instead of each
// reading a different part of the chunk.  The rows counted are the same in
// any order; sweep = 0 starts every workgroup at step 0.
__device__ __forceinline__ uint32_t sweep_start(int64_t seq, uint32_t n, int32_t sweep) {
    return sweep > 0 && n > 1 ? (uint32_t)(((uint64_t)seq * n / (uint32_t)sweep) % n) : 0u;
}

// Each 16-bit half shifted right by S (one packed shift).
template <int S>
__device__ __forceinline__ uint32_t pk_shr16(uint32_t a) {
    const u16x2 x = __builtin_bit_cast(u16x2, a);
    return __builtin_bit_cast(uint32_t, (u16x2)(x >> (unsigned short)S));
}

template <int K>
__device__ __forceinline__ void hist16_body(const uint8_t *__restrict__ cols, int64_t pitch,
                                            const uint8_t *__restrict__ arity, const QDesc &q,
                                            int32_t c, int32_t chunks, int32_t lds_words,
                                            int32_t pad_rows, int32_t *__restrict__ tables,
                                            uint32_t *lds, int64_t seq, int32_t sweep) {
    const int32_t cells = q.cells;
    uint32_t sb[K];
    Col colp[K];
    {
        uint32_t s = 1;
#pragma unroll
        for (int t = K - 1; t >= 0; --t) {
            const int32_t v = q.var[t];
            sb[t] = (s * 4u) * 0x00010001u;  // byte stride in both halves
            s *= arity[v];
            colp[t] = make_col(cols + (int64_t)v * pitch, pitch);
        }
    }
    // Lane columns: each cell owns B consecutive words (B = 64, 32, ..., 1,
    // as many as the LDS allows) and lane l adds into word x*B + l mod B, so
    // with B = 64 (or 32: a wave's halves go to the banks separately) no two
    // lanes of a ds_add share a bank whatever the keys, and smaller B only
    // ever shares a bank between lanes l and l + B.
    int32_t B = lds_words / cells;
    B = B >= 64 ? 64 : B >= 32 ? 32 : B >= 16 ? 16 : B >= 8 ? 8 : B >= 4 ? 4 : B >= 2 ? 2 : 1;
    zero_cols(lds, cells * B);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < K; ++t) sb[t] *= (uint32_t)B;
    const int64_t tiles = q.tiles;
    const int64_t r0 = (int64_t)c * tiles / chunks * kTileRows;
    const int64_t r1 = (int64_t)(c + 1) * tiles / chunks * kTileRows;
    const uint32_t init = ((threadIdx.x & (uint32_t)(B - 1)) * 4u) * 0x00010001u;
    char *base = reinterpret_cast<char *>(lds);

    const uint32_t nstep = (uint32_t)((r1 - r0 + kBlock * 16 - 1) / (kBlock * 16));
    uint32_t it = sweep_start(seq, nstep, sweep);
    for (uint32_t i = 0; i < nstep; ++i, it = it + 1 == nstep ? 0u : it + 1) {
        const uint32_t row = (uint32_t)r0 + it * (kBlock * 16u) + threadIdx.x * 16u;
        if (row >= (uint32_t)r1) continue;  // the chunk's ragged last step
        uint4 v[K];
#pragma unroll
        for (int t = 0; t < K; ++t) v[t] = load16(colp[t], row);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            uint32_t alo = init, ahi = init;  // instances (0,2) and (1,3) of this dword
#pragma unroll
            for (int t = 0; t < K; ++t) {
                const uint32_t w = d == 0 ? v[t].x : d == 1 ? v[t].y : d == 2 ? v[t].z : v[t].w;
                alo = pk_mad_u16(__builtin_amdgcn_perm(w, w, 0x0c020c00u), sb[t], alo);
                ahi = pk_mad_u16(__builtin_amdgcn_perm(w, w, 0x0c030c01u), sb[t], ahi);
            }
            atomicAdd(reinterpret_cast<uint32_t *>(base + (alo & 0xFFFFu)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + (ahi & 0xFFFFu)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + (alo >> 16)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + (ahi >> 16)), 1u);
        }
    }
    __syncthreads();
    flush_cols(lds, cells, B, (r1 == tiles * kTileRows) && (r0 < r1), pad_rows, chunks == 1,
               tables + q.table_off);
}

// LDS byte address of byte-key `i` of `key` (selector 0x0c0c0400 + i*256):
// B = 64: key*256 + slot with slot = lane*4; B = 32: (key*256 + slot) / 2
// with slot = (lane mod 32)*8.
template <int B>
__device__ __forceinline__ uint32_t lds_addr(uint32_t key, uint32_t slot, uint32_t sel) {
    const uint32_t a = __builtin_amdgcn_perm(key, slot, sel);
    return B == 64 ? a : a >> 1;
}

// LDS histogram for tables of at most 256 cells.  A column word holds four
// instances as bytes, so its low 16-bit half is b1*256 + b0; summed over the
// query's columns with packed multiply-adds, (b1*256 + b0) * stride gives
// key1*256 + key0 exactly, because every key is below 256 and no carry
// crosses the byte boundary (key3, key2 likewise in the high half).  One
// packed multiply-add per column thus forms four keys, and one byte permute
// per instance turns a key into the LDS byte address key*256 + lane*4: every
// cell owns 64 words, one per lane, so no ds_add of a wave has a bank
// conflict whatever the keys.  B = 32 (tables of up to 256 cells in 32 KiB):
// the permute builds key*256 + (lane mod 32)*8 and one shift halves it.
template <int K, int B>
__device__ __forceinline__ void hist8_body(const uint8_t *__restrict__ cols, int64_t pitch,
                                           const uint8_t *__restrict__ arity, const QDesc &q,
                                           int32_t c, int32_t chunks, int32_t pad_rows,
                                           int32_t *__restrict__ tables, uint32_t *lds,
                                           int64_t seq, int32_t sweep) {
    const int32_t cells = q.cells;
    uint32_t sb[K];
    Col colp[K];
    {
        uint32_t s = 1;
#pragma unroll
        for (int t = K - 1; t >= 0; --t) {
            const int32_t v = q.var[t];
            sb[t] = s * 0x00010001u;  // the stride in both halves
            s *= arity[v];
            colp[t] = make_col(cols + (int64_t)v * pitch, pitch);
        }
    }
    zero_cols(lds, cells * B);
    __syncthreads();
    const int64_t tiles = q.tiles;
    const int64_t r0 = (int64_t)c * tiles / chunks * kTileRows;
    const int64_t r1 = (int64_t)(c + 1) * tiles / chunks * kTileRows;
    const uint32_t slot = B == 64 ? (threadIdx.x & 63u) * 4u : (threadIdx.x & 31u) * 8u;
    char *base = reinterpret_cast<char *>(lds);

    const uint32_t nstep = (uint32_t)((r1 - r0 + kBlock * 16 - 1) / (kBlock * 16));
    uint32_t it = sweep_start(seq, nstep, sweep);
    for (uint32_t i = 0; i < nstep; ++i, it = it + 1 == nstep ? 0u : it + 1) {
        const uint32_t row = (uint32_t)r0 + it * (kBlock * 16u) + threadIdx.x * 16u;
        if (row >= (uint32_t)r1) continue;  // the chunk's ragged last step
        uint4 v[K];
#pragma unroll
        for (int t = 0; t < K; ++t) v[t] = load16(colp[t], row);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            uint32_t key = 0;  // bytes: keys of instances 0..3 of this word
#pragma unroll
            for (int t = 0; t < K; ++t) {
                const uint32_t w = d == 0 ? v[t].x : d == 1 ? v[t].y : d == 2 ? v[t].z : v[t].w;
                key = pk_mad_u16(w, sb[t], key);
            }
            // byte 0 of the address from `slot`, byte 1 from key byte i
            atomicAdd(reinterpret_cast<uint32_t *>(base + lds_addr<B>(key, slot, 0x0c0c0400u)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + lds_addr<B>(key, slot, 0x0c0c0500u)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + lds_addr<B>(key, slot, 0x0c0c0600u)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + lds_addr<B>(key, slot, 0x0c0c0700u)), 1u);
        }
    }
    __syncthreads();
    flush_cols(lds, cells, B, (r1 == tiles * kTileRows) && (r0 < r1), pad_rows, chunks == 1,
               tables + q.table_off);
}

// CAP: the launch group's largest table.  The histogram is a static LDS
// array so its address is a compile-time constant and no add is spent per
// instance on the LDS base.
template <int K, int CAP>
__global__ __launch_bounds__(kBlock) void k_hist8(const uint8_t *__restrict__ cols,
                                                  int64_t pitch,
                                                  const uint8_t *__restrict__ arity,
                                                  const QDesc *__restrict__ descs, int32_t nd,
                                                  int32_t chunks, int32_t pad_rows,
                                                  int32_t *__restrict__ tables, int32_t sweep) {
    constexpr int B = CAP <= 64 ? 64 : 32;
    __shared__ __attribute__((aligned(16))) uint32_t lds[CAP * B];
    int32_t di, c;
    map_block(blockIdx.x, nd, chunks, di, c);
    hist8_body<K, B>(cols, pitch, arity, descs[di], c, chunks, pad_rows, tables, lds,
                     (int64_t)blockIdx.x / kXcds, sweep);
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_hist16(const uint8_t *__restrict__ cols,
                                                   int64_t pitch,
                                                   const uint8_t *__restrict__ arity,
                                                   const QDesc *__restrict__ descs, int32_t nd,
                                                   int32_t chunks, int32_t lds_words,
                                                   int32_t pad_rows,
                                                   int32_t *__restrict__ tables, int32_t sweep) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    int32_t di, c;
    map_block(blockIdx.x, nd, chunks, di, c);
    hist16_body<K>(cols, pitch, arity, descs[di], c, chunks, lds_words, pad_rows, tables, lds,
                   (int64_t)blockIdx.x / kXcds, sweep);
}

// The same two histograms over the 4-bit packed columns (all arities at most
// 16): half the bytes per instance.  A packed word holds 8 instances, two
// per byte (low nibble first); each thread reads 32 instances per column.
//
// Byte keys (tables of at most 256 cells): the odd nibbles of a word, masked
// into bytes, give one chain of packed multiply-adds (four keys); the whole
// word gives another, P, whose halves hold even key + 16 x odd key (every
// key is below 256, so the difference P - 16 x odd is exact mod 2^16) and
// the even keys come from one more multiply-add per word.
template <int K, int B>
__device__ __forceinline__ void hist8n_body(const uint8_t *__restrict__ nib, int64_t pitch,
                                            const uint8_t *__restrict__ arity, const QDesc &q,
                                            int32_t c, int32_t chunks, int32_t pad_rows,
                                            int32_t *__restrict__ tables, uint32_t *lds,
                                            int64_t seq, int32_t sweep) {
    const int32_t cells = q.cells;
    uint32_t sb[K];
    Col colp[K];
    {
        uint32_t s = 1;
#pragma unroll
        for (int t = K - 1; t >= 0; --t) {
            const int32_t v = q.var[t];
            sb[t] = s * 0x00010001u;
            s *= arity[v];
            colp[t] = make_col(nib + (int64_t)v * (pitch / 2), pitch / 2);
        }
    }
    zero_cols(lds, cells * B);
    __syncthreads();
    const int64_t tiles = q.tiles;
    const int64_t r0 = (int64_t)c * tiles / chunks * kTileRows;
    const int64_t r1 = (int64_t)(c + 1) * tiles / chunks * kTileRows;
    const uint32_t slot = B == 64 ? (threadIdx.x & 63u) * 4u : (threadIdx.x & 31u) * 8u;
    char *base = reinterpret_cast<char *>(lds);
    uint32_t kMinus16 = 0xFFF0FFF0u;  // -16 in both halves, kept one multiply-add
    asm volatile("" : "+v"(kMinus16));

    const uint32_t nstep = (uint32_t)((r1 - r0 + kBlock * 32 - 1) / (kBlock * 32));
    uint32_t it = sweep_start(seq, nstep, sweep);
    for (uint32_t i = 0; i < nstep; ++i, it = it + 1 == nstep ? 0u : it + 1) {
        const uint32_t row = (uint32_t)r0 + it * (kBlock * 32u) + threadIdx.x * 32u;
        if (row >= (uint32_t)r1) continue;  // the chunk's ragged last step
        uint4 v[K];
#pragma unroll
        for (int t = 0; t < K; ++t) v[t] = load16(colp[t], row >> 1);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            uint32_t pw = 0, ko = 0;  // whole words / bytes: keys of the odd instances
#pragma unroll
            for (int t = 0; t < K; ++t) {
                const uint32_t w = d == 0 ? v[t].x : d == 1 ? v[t].y : d == 2 ? v[t].z : v[t].w;
                pw = pk_mad_u16(w, sb[t], pw);
                ko = pk_mad_u16((w >> 4) & 0x0F0F0F0Fu, sb[t], ko);
            }
            const uint32_t ke = pk_mad_u16(ko, kMinus16, pw);  // bytes: keys of the even instances
            atomicAdd(reinterpret_cast<uint32_t *>(base + lds_addr<B>(ke, slot, 0x0c0c0400u)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + lds_addr<B>(ke, slot, 0x0c0c0500u)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + lds_addr<B>(ke, slot, 0x0c0c0600u)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + lds_addr<B>(ke, slot, 0x0c0c0700u)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + lds_addr<B>(ko, slot, 0x0c0c0400u)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + lds_addr<B>(ko, slot, 0x0c0c0500u)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + lds_addr<B>(ko, slot, 0x0c0c0600u)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + lds_addr<B>(ko, slot, 0x0c0c0700u)), 1u);
        }
    }
    __syncthreads();
    flush_cols(lds, cells, B, (r1 == tiles * kTileRows) && (r0 < r1), pad_rows, chunks == 1,
               tables + q.table_off);
}

template <int K, int CAP>
__global__ __launch_bounds__(kBlock) void k_hist8n(const uint8_t *__restrict__ nib,
                                                   int64_t pitch,
                                                   const uint8_t *__restrict__ arity,
                                                   const QDesc *__restrict__ descs, int32_t nd,
                                                   int32_t chunks, int32_t pad_rows,
                                                   int32_t *__restrict__ tables, int32_t sweep) {
    constexpr int B = CAP <= 64 ? 64 : 32;
    __shared__ __attribute__((aligned(16))) uint32_t lds[CAP * B];
    int32_t di, c;
    map_block(blockIdx.x, nd, chunks, di, c);
    hist8n_body<K, B>(nib, pitch, arity, descs[di], c, chunks, pad_rows, tables, lds,
                      (int64_t)blockIdx.x / kXcds, sweep);
}

// Address keys (lane columns of B words per cell): the key of two instances
// (nibbles j and j + 4 of a word) forms in the 16-bit halves of a register.
// No nibble is masked out: with u_j the word's 16-bit halves each shifted
// right by 4j, the halves of u_j - 16 u_(j+1) are exactly nibbles j and
// j + 4 (and u_3 holds nibbles 3 and 7 alone), so the sums
// P_j = init_j + sum_t u_j(t) * stride_t give every key as
// P_j - 16 P_(j+1) (and P_3 itself) in one packed multiply-add per word:
// 3 shifts and 4 multiply-adds per column per 8 instances.  The starting
// values init_j are chosen so that each difference leaves the lane's word
// offset.
template <int K>
__device__ __forceinline__ void hist16n_body(const uint8_t *__restrict__ nib, int64_t pitch,
                                             const uint8_t *__restrict__ arity, const QDesc &q,
                                             int32_t c, int32_t chunks, int32_t lds_words,
                                             int32_t pad_rows, int32_t *__restrict__ tables,
                                             uint32_t *lds, int64_t seq, int32_t sweep) {
    const int32_t cells = q.cells;
    int32_t B = lds_words / cells;
    B = B >= 64 ? 64 : B >= 32 ? 32 : B >= 16 ? 16 : B >= 8 ? 8 : B >= 4 ? 4 : B >= 2 ? 2 : 1;
    uint32_t sa[K];
    Col colp[K];
    {
        uint32_t s = 1;
#pragma unroll
        for (int t = K - 1; t >= 0; --t) {
            const int32_t v = q.var[t];
            sa[t] = (s * 4u * (uint32_t)B) * 0x00010001u;  // byte stride of a state
            s *= arity[v];
            colp[t] = make_col(nib + (int64_t)v * (pitch / 2), pitch / 2);
        }
    }
    zero_cols(lds, cells * B);
    __syncthreads();
    const int64_t tiles = q.tiles;
    const int64_t r0 = (int64_t)c * tiles / chunks * kTileRows;
    const int64_t r1 = (int64_t)(c + 1) * tiles / chunks * kTileRows;
    // init_3 = o, init_j = o + 16 init_(j+1) (mod 2^16), o the lane's byte offset
    const uint32_t o = (threadIdx.x & (uint32_t)(B - 1)) * 4u;
    const uint32_t i3 = o * 0x00010001u, i2 = ((o * 17u) & 0xFFFFu) * 0x00010001u,
                   i1 = ((o * 273u) & 0xFFFFu) * 0x00010001u,
                   i0 = ((o * 4369u) & 0xFFFFu) * 0x00010001u;
    // -16 in both halves, hidden from the optimiser so that each difference
    // stays one multiply-add instead of a shift and a subtraction
    uint32_t kMinus16 = 0xFFF0FFF0u;
    asm volatile("" : "+v"(kMinus16));
    char *base = reinterpret_cast<char *>(lds);

    const uint32_t nstep = (uint32_t)((r1 - r0 + kBlock * 32 - 1) / (kBlock * 32));
    uint32_t it = sweep_start(seq, nstep, sweep);
    for (uint32_t i = 0; i < nstep; ++i, it = it + 1 == nstep ? 0u : it + 1) {
        const uint32_t row = (uint32_t)r0 + it * (kBlock * 32u) + threadIdx.x * 32u;
        if (row >= (uint32_t)r1) continue;  // the chunk's ragged last step
        uint4 v[K];
#pragma unroll
        for (int t = 0; t < K; ++t) v[t] = load16(colp[t], row >> 1);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            uint32_t p0 = i0, p1 = i1, p2 = i2, p3 = i3;
#pragma unroll
            for (int t = 0; t < K; ++t) {
                const uint32_t w = d == 0 ? v[t].x : d == 1 ? v[t].y : d == 2 ? v[t].z : v[t].w;
                p0 = pk_mad_u16(w, sa[t], p0);
                p1 = pk_mad_u16(pk_shr16<4>(w), sa[t], p1);
                p2 = pk_mad_u16(pk_shr16<8>(w), sa[t], p2);
                p3 = pk_mad_u16(pk_shr16<12>(w), sa[t], p3);
            }
            // instances (0,4) .. (3,7)
            const uint32_t a0 = pk_mad_u16(p1, kMinus16, p0), a1 = pk_mad_u16(p2, kMinus16, p1),
                           a2 = pk_mad_u16(p3, kMinus16, p2), a3 = p3;
            atomicAdd(reinterpret_cast<uint32_t *>(base + (a0 & 0xFFFFu)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + (a1 & 0xFFFFu)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + (a2 & 0xFFFFu)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + (a3 & 0xFFFFu)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + (a0 >> 16)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + (a1 >> 16)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + (a2 >> 16)), 1u);
            atomicAdd(reinterpret_cast<uint32_t *>(base + (a3 >> 16)), 1u);
        }
    }
    __syncthreads();
    flush_cols(lds, cells, B, (r1 == tiles * kTileRows) && (r0 < r1), pad_rows, chunks == 1,
               tables + q.table_off);
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_hist16n(const uint8_t *__restrict__ nib,
                                                    int64_t pitch,
                                                    const uint8_t *__restrict__ arity,
                                                    const QDesc *__restrict__ descs, int32_t nd,
                                                    int32_t chunks, int32_t lds_words,
                                                    int32_t pad_rows,
                                                    int32_t *__restrict__ tables, int32_t sweep) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    int32_t di, c;
    map_block(blockIdx.x, nd, chunks, di, c);
    hist16n_body<K>(nib, pitch, arity, descs[di], c, chunks, lds_words, pad_rows, tables, lds,
                    (int64_t)blockIdx.x / kXcds, sweep);
}

// Bitmap count (Alg. 1) of one descriptor over one chunk of 64-row words.
// Leaf rows (the last variable's states) of up to kLeafMax states are loaded
// once per word group into registers and reused under every prefix.
constexpr int kLeafMax = 8;

// Level L of the tree walks the variable at query position perm[L]; str[L]
// is that variable's cell stride in the table (the product of the arities
// after it in the query), so a leaf's cell is the same whatever the order.
template <int L, int K, int W>
struct Walk {
    __device__ __forceinline__ static void go(const uint64_t (&pre)[W], uint32_t cell,
                                              const uint64_t *__restrict__ bits, int64_t wpitch,
                                              int64_t w, const int32_t (&base)[K],
                                              const int32_t (&rad)[K], const uint32_t (&str)[K],
                                              bool cached, const uint64_t (&leaf)[kLeafMax][W],
                                              uint32_t *acc) {
        if constexpr (L == K - 1) {
            if (cached) {
#pragma unroll
                for (int s = 0; s < kLeafMax; ++s) {
                    if (s < rad[L]) {
                        uint32_t pc = 0;
#pragma unroll
                        for (int i = 0; i < W; ++i) pc += (uint32_t)__popcll(leaf[s][i] & pre[i]);
                        acc[(cell + (uint32_t)s * str[L]) * kBlock] += pc;
                    }
                }
                return;
            }
        }
        for (int32_t s = 0; s < rad[L]; ++s) {
            const uint64_t *row = bits + (int64_t)(base[L] + s) * wpitch + w;
            uint64_t x[W];
#pragma unroll
            for (int i = 0; i < W; ++i) x[i] = row[i] & pre[i];
            const uint32_t c2 = cell + (uint32_t)s * str[L];
            if constexpr (L == K - 1) {
                uint32_t pc = 0;
#pragma unroll
                for (int i = 0; i < W; ++i) pc += (uint32_t)__popcll(x[i]);
                acc[c2 * kBlock] += pc;
            } else {
                uint64_t any = 0;
#pragma unroll
                for (int i = 0; i < W; ++i) any |= x[i];
                if (__any(any != 0))
                    Walk<L + 1, K, W>::go(x, c2, bits, wpitch, w, base, rad, str, cached, leaf,
                                          acc);
            }
        }
    }
};

template <int K, int W>
__device__ __forceinline__ void bitmap_body(const uint64_t *__restrict__ bits, int64_t wpitch,
                                            const int32_t *__restrict__ soff,
                                            const uint8_t *__restrict__ arity, const QDesc &q,
                                            int32_t c, int32_t chunks,
                                            int32_t *__restrict__ tables,
                                            uint32_t *acc /* [cells][kBlock] */) {
    const int32_t cells = q.cells;
    // walk order: level L takes query position (win_base >> 3L) & 7
    int32_t ar[K];
    uint32_t st[K];
#pragma unroll
    for (int t = 0; t < K; ++t) ar[t] = arity[q.var[t]];
    st[K - 1] = 1;
#pragma unroll
    for (int t = K - 2; t >= 0; --t) st[t] = st[t + 1] * (uint32_t)ar[t + 1];
    int32_t base[K], rad[K];
    uint32_t str[K];
#pragma unroll
    for (int L = 0; L < K; ++L) {
        const int t = ((uint32_t)q.win_base >> (3 * L)) & 7u;
        base[L] = soff[q.var[t]];
        rad[L] = ar[t];
        str[L] = st[t];
    }
    for (int32_t i = threadIdx.x; i < cells * kBlock; i += kBlock) acc[i] = 0;
    __syncthreads();
    const int64_t tiles = q.tiles;
    const int64_t w0 = (int64_t)c * tiles / chunks * (kTileRows / 64);
    const int64_t w1 = (int64_t)(c + 1) * tiles / chunks * (kTileRows / 64);
    uint64_t ones[W];
#pragma unroll
    for (int i = 0; i < W; ++i) ones[i] = ~0ull;
    // K = 1: the root level is the leaf level and every row is read once
    const bool cached = K > 1 && rad[K - 1] <= kLeafMax;
    uint64_t leaf[kLeafMax][W];
    for (int64_t w = w0 + (int64_t)threadIdx.x * W; w < w1; w += kBlock * W) {
        if (cached) {
#pragma unroll
            for (int s = 0; s < kLeafMax; ++s) {
                if (s < rad[K - 1]) {  // uniform: no load for absent states
                    const uint64_t *row = bits + (int64_t)(base[K - 1] + s) * wpitch + w;
#pragma unroll
                    for (int i = 0; i < W; ++i) leaf[s][i] = row[i];
                } else {
#pragma unroll
                    for (int i = 0; i < W; ++i) leaf[s][i] = 0ull;
                }
            }
        }
        Walk<0, K, W>::go(ones, 0u, bits, wpitch, w, base, rad, str, cached, leaf,
                          acc + threadIdx.x);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t *out = tables + q.table_off;
    for (int32_t cell = wave; cell < cells; cell += kWaves) {
        uint32_t s = 0;
        for (int j = lane; j < kBlock; j += 64) s += acc[cell * kBlock + j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0 && s) atomicAdd(&out[cell], (int32_t)s);
    }
}

template <int K, int W>
__global__ __launch_bounds__(kBlock) void k_bitmap(const uint64_t *__restrict__ bits,
                                                   int64_t wpitch,
                                                   const int32_t *__restrict__ soff,
                                                   const uint8_t *__restrict__ arity,
                                                   const QDesc *__restrict__ descs, int32_t nd,
                                                   int32_t chunks, int32_t *__restrict__ tables) {
    extern __shared__ uint32_t acc[];  // [cells][kBlock], thread-private columns
    int32_t di, c;
    map_block(blockIdx.x, nd, chunks, di, c);
    bitmap_body<K, W>(bits, wpitch, soff, arity, descs[di], c, chunks, tables, acc);
}

// One persistent launch over many launch groups.  Each group is a set of
// descriptors counted with one strategy and one K; its (descriptor, chunk)
// blocks get virtual indices [vbase, vbase + nv), vbase a multiple of 8, and
// virtual block v belongs to XCD v % 8 (the same order map_block gives a
// normal launch).  A resident workgroup reads its XCD from HW_REG_XCC_ID,
// claims that XCD's virtual blocks through an atomic head, and steals from
// the other XCDs' sequences when its own runs dry; it exits when all eight
// are exhausted, so every wave reaches the exit.
struct PGroup {
    int64_t vbase;
    int64_t nv;       // padded to a multiple of 8
    int32_t first;    // first descriptor
    int32_t nd;
    int32_t chunks;
    int32_t kind;     // PK_* << 4 | K
};
enum { PK_HIST16 = 1, PK_HIST_S = 2, PK_HIST_B = 3, PK_BITMAP = 4, PK_HIST8 = 5, PK_HIST8N = 6 };

template <int K, int W>
__device__ __forceinline__ void persistent_case(int type, const uint8_t *cols, const uint8_t *nib,
                                                int64_t pitch, const uint64_t *bits,
                                                int64_t wpitch, const int32_t *soff,
                                                const uint8_t *arity, const QDesc &q, int32_t c,
                                                int32_t chunks, int32_t lds_words, int32_t pad,
                                                int32_t *tables, uint32_t *lds) {
    switch (type) {
        case PK_HIST8:
            hist8_body<K, 64>(cols, pitch, arity, q, c, chunks, pad, tables, lds, 0, 0);
            break;
        case PK_HIST8N:
            hist8n_body<K, 64>(nib, pitch, arity, q, c, chunks, pad, tables, lds, 0, 0);
            break;
        case PK_HIST16:
            hist16_body<K>(cols, pitch, arity, q, c, chunks, lds_words, pad, tables, lds, 0, 0);
            break;
        case PK_HIST_S:
            hist_body<K, true>(cols, pitch, arity, q, c, chunks, lds_words, pad, tables, lds);
            break;
        case PK_HIST_B:
            hist_body<K, false>(cols, pitch, arity, q, c, chunks, lds_words, pad, tables, lds);
            break;
        default:
            bitmap_body<K, W>(bits, wpitch, soff, arity, q, c, chunks, tables, lds);
            break;
    }
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_count_persistent(
    const uint8_t *__restrict__ cols, const uint8_t *__restrict__ nib, int64_t pitch,
    const uint64_t *__restrict__ bits, int64_t wpitch, const int32_t *__restrict__ soff,
    const uint8_t *__restrict__ arity, const QDesc *__restrict__ descs,
    const PGroup *__restrict__ groups, int32_t ngroups,
    int64_t total_v, uint32_t *__restrict__ heads, int32_t lds_words, int32_t pad_rows,
    int32_t *__restrict__ tables) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    __shared__ int64_t s_v;
    const uint32_t xcc = __builtin_amdgcn_s_getreg((3 << 11) | 20) & 7u;  // HW_REG_XCC_ID
    for (;;) {
        __syncthreads();  // the previous block is done with LDS and s_v
        if (threadIdx.x == 0) {
            int64_t v = -1;
            for (uint32_t s = 0; s < kXcds; ++s) {
                const uint32_t x = (xcc + s) & 7u;
                const int64_t cand = (int64_t)atomicAdd(&heads[x], 1u) * kXcds + x;
                if (cand < total_v) {
                    v = cand;
                    break;
                }
            }
            s_v = v;
        }
        __syncthreads();
        const int64_t v = s_v;
        if (v < 0) break;
        int32_t g = 0;
        while (g + 1 < ngroups && groups[g + 1].vbase <= v) ++g;
        const PGroup G = groups[g];
        const int64_t b = v - G.vbase;
        if (b >= (int64_t)G.nd * G.chunks) continue;  // padding block
        int32_t di, c;
        map_block(b, G.nd, G.chunks, di, c);
        const QDesc &q = descs[G.first + di];
        const int type = G.kind >> 4;
        switch (G.kind & 15) {
            case 1: persistent_case<1, W>(type, cols, nib, pitch, bits, wpitch, soff, arity, q, c, G.chunks, lds_words, pad_rows, tables, lds); break;
            case 2: persistent_case<2, W>(type, cols, nib, pitch, bits, wpitch, soff, arity, q, c, G.chunks, lds_words, pad_rows, tables, lds); break;
            case 3: persistent_case<3, W>(type, cols, nib, pitch, bits, wpitch, soff, arity, q, c, G.chunks, lds_words, pad_rows, tables, lds); break;
            case 4: persistent_case<4, W>(type, cols, nib, pitch, bits, wpitch, soff, arity, q, c, G.chunks, lds_words, pad_rows, tables, lds); break;
            case 5: persistent_case<5, W>(type, cols, nib, pitch, bits, wpitch, soff, arity, q, c, G.chunks, lds_words, pad_rows, tables, lds); break;
            case 6: persistent_case<6, W>(type, cols, nib, pitch, bits, wpitch, soff, arity, q, c, G.chunks, lds_words, pad_rows, tables, lds); break;
            case 7: persistent_case<7, W>(type, cols, nib, pitch, bits, wpitch, soff, arity, q, c, G.chunks, lds_words, pad_rows, tables, lds); break;
            default: persistent_case<8, W>(type, cols, nib, pitch, bits, wpitch, soff, arity, q, c, G.chunks, lds_words, pad_rows, tables, lds); break;
        }
    }
}

// Zero every descriptor's table (tables placed by the caller).
__global__ void k_zero_tables(const QDesc *__restrict__ descs, int32_t nd,
                              int32_t *__restrict__ tables) {
    for (int32_t d = blockIdx.x; d < nd; d += gridDim.x) {
        int32_t *t = tables + descs[d].table_off;
        for (int32_t i = threadIdx.x; i < descs[d].cells; i += blockDim.x) t[i] = 0;
    }
}

// Tables of one- and two-variable queries from the Gram C of their
// variables' state bit-vectors (valid on and above the diagonal): cell
// (s0, s1) of query (v0, v1) is Count(X_v0 = s0 AND X_v1 = s1), entry
// (pos[v0] + s0, pos[v1] + s1) read on its upper side; a one-variable table
// is the diagonal.  One workgroup per query.
__global__ void k_gram_tables(const QDesc *__restrict__ d, int64_t nd,
                              const int32_t *__restrict__ pos, const uint8_t *__restrict__ arity,
                              const int32_t *__restrict__ C, int64_t ldc,
                              int32_t *__restrict__ tables) {
    for (int64_t q = blockIdx.x; q < nd; q += gridDim.x) {
        const QDesc x = d[q];
        const int64_t p0 = pos[x.var[0]];
        const int64_t p1 = x.k == 2 ? pos[x.var[1]] : p0;
        const int32_t r1 = x.k == 2 ? arity[x.var[1]] : 1;
        for (int32_t c = threadIdx.x; c < x.cells; c += blockDim.x) {
            const int64_t i = x.k == 2 ? p0 + c / r1 : p0 + c;
            const int64_t j = x.k == 2 ? p1 + c % r1 : p0 + c;
            const int64_t a = i < j ? i : j, b = i < j ? j : i;
            tables[x.table_off + c] = C[a * ldc + b];
        }
    }
}

// Single-assignment count: one path of the Alg. 1 tree (bit-vector rows).
struct Rows8 {
    int32_t r[FC_MAX_VARS];
};
__global__ void k_assign_bits(const uint64_t *__restrict__ bits, int64_t words, int64_t wpitch,
                              Rows8 rows, int32_t k, unsigned long long *__restrict__ out) {
    unsigned long long cnt = 0;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words;
         w += (int64_t)gridDim.x * blockDim.x) {
        uint64_t x = ~0ull;
        for (int32_t t = 0; t < k; ++t) x &= bits[(int64_t)rows.r[t] * wpitch + w];
        cnt += (unsigned long long)__popcll(x);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(out, cnt);
}

// Same count from the state columns (no bit-vectors): one partition path.
struct Assign8 {
    int32_t var[FC_MAX_VARS];
    int32_t state[FC_MAX_VARS];
};
__global__ void k_assign_cols(const uint8_t *__restrict__ cols, int64_t m, int64_t pitch,
                              Assign8 a, int32_t k, unsigned long long *__restrict__ out) {
    unsigned long long cnt = 0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m;
         p += (int64_t)gridDim.x * blockDim.x) {
        bool ok = true;
        for (int32_t t = 0; t < k; ++t)
            ok = ok && cols[(int64_t)a.var[t] * pitch + p] == (uint8_t)a.state[t];
        cnt += ok ? 1ull : 0ull;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(out, cnt);
}

// Batched single-assignment counts: work unit (query, chunk of 64-instance
// words), XCD-ordered like the tables.  Each thread ANDs two words of the k
// bit-vector rows at a time and popcounts; one atomic per workgroup.
struct ADesc {
    int32_t row[FC_MAX_VARS];  // bit-vector rows (variable's first row + state)
    int32_t k;
    int32_t pad[3];
};

__global__ __launch_bounds__(kBlock) void k_assign_batch(const uint64_t *__restrict__ bits,
                                                         int64_t words, int64_t wpitch,
                                                         const ADesc *__restrict__ descs,
                                                         int32_t nd, int32_t chunks,
                                                         unsigned long long *__restrict__ out) {
    __shared__ unsigned long long part[kWaves];
    int32_t di, c;
    map_block(blockIdx.x, nd, chunks, di, c);
    const ADesc &q = descs[di];
    const int64_t tiles = words / (kTileRows / 64);
    const int64_t w0 = (int64_t)c * tiles / chunks * (kTileRows / 64);
    const int64_t w1 = (int64_t)(c + 1) * tiles / chunks * (kTileRows / 64);
    unsigned long long cnt = 0;
    for (int64_t w = w0 + 2 * (int64_t)threadIdx.x; w < w1; w += 2 * kBlock) {
        uint64_t x0 = ~0ull, x1 = ~0ull;
        for (int32_t t = 0; t < q.k; ++t) {
            const ulonglong2 v = *reinterpret_cast<const ulonglong2 *>(bits + (int64_t)q.row[t] * wpitch + w);
            x0 &= v.x;
            x1 &= v.y;
        }
        cnt += (unsigned long long)(__popcll(x0) + __popcll(x1));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int i = 0; i < kWaves; ++i) s += part[i];
        if (s) atomicAdd(&out[di], s);
    }
}

// The same counts from the state columns (no bit-vectors).
__global__ __launch_bounds__(kBlock) void k_assign_batch_cols(
    const uint8_t *__restrict__ cols, int64_t m, int64_t pitch, const int32_t *__restrict__ vflat,
    const int64_t *__restrict__ voff, const uint8_t *__restrict__ sflat, int32_t nd,
    int32_t chunks, unsigned long long *__restrict__ out) {
    __shared__ unsigned long long part[kWaves];
    int32_t di, c;
    map_block(blockIdx.x, nd, chunks, di, c);
    const int64_t o0 = voff[di], o1 = voff[di + 1];
    const int64_t tiles = (m + kTileRows - 1) / kTileRows;
    const int64_t r0 = (int64_t)c * tiles / chunks * kTileRows;
    const int64_t r1 = std::min<int64_t>(m, (int64_t)(c + 1) * tiles / chunks * kTileRows);
    unsigned long long cnt = 0;
    for (int64_t p = r0 + threadIdx.x; p < r1; p += kBlock) {
        bool ok = true;
        for (int64_t t = o0; t < o1; ++t) ok = ok && cols[(int64_t)vflat[t] * pitch + p] == sflat[t];
        cnt += ok ? 1ull : 0ull;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int i = 0; i < kWaves; ++i) s += part[i];
        if (s) atomicAdd(&out[di], s);
    }
}

// ------------------------------------------------------------------ planner
enum Strat { S_HIST = 1, S_BITMAP = 2, S_PART = 3 };

// A derived table: the table at dst_off (dst_cells cells) is the sum of the
// counted table at src_off over the axes the derived query lacks.  Axis a
// of the source (query order, last axis fastest) has src_rad[a] states and
// stride dst_str[a] in the derived table (0: summed out).
struct alignas(16) MDesc {
    int64_t dst_off, src_off;
    int32_t src_cells, dst_cells, src_k, pad;
    int32_t src_rad[FC_MAX_VARS];
    int32_t dst_str[FC_MAX_VARS];
};
static_assert(sizeof(MDesc) == 96, "MDesc layout");

// One workgroup per derived table: every non-zero source cell is decoded
// into its digits and added to the derived cell in LDS; the whole derived
// table is then stored (no zeroing of the output needed).
__global__ __launch_bounds__(kBlock) void k_marginal(const MDesc *__restrict__ md, int64_t nm,
                                                     int32_t *__restrict__ tables) {
    extern __shared__ uint32_t acc[];
    for (int64_t g = blockIdx.x; g < nm; g += gridDim.x) {
        const MDesc &d = md[g];
        const int32_t dc = d.dst_cells, sc = d.src_cells, k = d.src_k;
        for (int32_t j = threadIdx.x; j < dc; j += kBlock) acc[j] = 0;
        __syncthreads();
        const int32_t *src = tables + d.src_off;
        for (int32_t i = threadIdx.x; i < sc; i += kBlock) {
            const int32_t v = src[i];
            if (v == 0) continue;
            uint32_t rem = (uint32_t)i, idx = 0;
            for (int a = k - 1; a >= 0; --a) {
                const uint32_t r = (uint32_t)d.src_rad[a];
                const uint32_t q = rem / r;
                idx += (rem - q * r) * (uint32_t)d.dst_str[a];
                rem = q;
            }
            atomicAdd(&acc[idx], (uint32_t)v);
        }
        __syncthreads();
        int32_t *dst = tables + d.dst_off;
        for (int32_t j = threadIdx.x; j < dc; j += kBlock) dst[j] = (int32_t)acc[j];
        __syncthreads();
    }
}

struct Launch {
    char name[32];    // kernel instance (profiling)
    double alg_bytes; // k bytes per query and instance, summed
    int strat;
    int K;
    bool small;
    int32_t hk;       // histogram kernel: HK_HIST8(N), HK_HIST16(N) or HK_GENERIC
    int64_t first;    // first descriptor
    int32_t count;    // descriptors
    int32_t chunks;
    int32_t lds_bytes;
};

struct Plan {
    std::vector<QDesc> work;    // counting descriptors, grouped by launch
    std::vector<QDesc> query;   // one per query, in query order, when needed
    bool windows = false;       // some query is split into key windows
    int64_t nq = 0;
    std::vector<Launch> launches;
    int64_t total_cells = 0;    // table buffer size in cells
    bool packed = true;         // tables back to back in query order
    // one- and two-variable queries answered from the Gram of their
    // variables' state bit-vectors: descriptors work[gram_first, +gram_count)
    int64_t gram_first = 0, gram_count = 0;
    int32_t gram_np = 0;               // Gram rows, padded to whole blocks
    std::vector<int32_t> gram_rows;    // bit-vector row of each Gram row (-1: padding)
    std::vector<int32_t> gram_pos;     // [n] Gram row of a variable's state 0
    double gram_bytes = 0.0, gram_ops = 0.0;
    // every counting launch stores whole tables (or key windows) from one
    // workgroup each: the tables need no zeroing first
    bool direct = false;
    // tables summed out of a counted superset's table after counting
    std::vector<MDesc> marg;
    int32_t marg_max_cells = 0;
    // tables beyond the LDS classes counted by the one-pass partition:
    // descriptors work[part_first, +part_count), k bytes per instance each
    int64_t part_first = 0, part_count = 0;
    double part_bytes = 0.0;
};

// LDS size classes; every class but the last keeps its byte addresses below
// 2^16 (the packed 16-bit key path).
// Classes up to 256 cells use the byte-key kernels (64 words per cell up to
// 64 cells, 32 above, so that no class takes more than 32 KiB of LDS).
static const int32_t kClassCap[] = {16, 64, 256, 1024, 4096, 16383, kHistMaxCells};
static const int32_t kClassLds[] = {16 * 64 * 4, 64 * 64 * 4, 256 * 32 * 4, 1024 * 8 * 4,
                                    4096 * 2 * 4, 16383 * 4,  kHistMaxCells * 4 + 4};
constexpr int kHist8Classes = 3;
constexpr int kHist16Classes = 6;
enum { HK_GENERIC = 0, HK_HIST16 = 1, HK_HIST8 = 2, HK_HIST16N = 3, HK_HIST8N = 4 };

static int hist_class(int64_t cells) {
    for (int i = 0; i < 7; ++i)
        if (cells <= kClassCap[i]) return i;
    return -1;
}

static int validate(const fc_db *db, const int32_t *vars_flat, const int64_t *var_off,
                    int64_t nq, const int64_t *table_off, std::vector<int64_t> &cells) {
    if (!db) {
        set_error("NULL database handle");
        return FC_ERR_INVALID;
    }
    if (nq < 0 || (nq > 0 && (!vars_flat || !var_off))) {
        set_error("need nq >= 0, vars_flat and var_off");
        return FC_ERR_INVALID;
    }
    if (nq > (int64_t)INT32_MAX / 2) {
        set_error("batch of %lld queries is too large", (long long)nq);
        return FC_ERR_RANGE;
    }
    cells.resize((size_t)nq);
    if (nq > 0 && var_off[0] != 0) {
        set_error("var_off[0] must be 0");
        return FC_ERR_INVALID;
    }
    for (int64_t i = 0; i < nq; ++i) {
        int64_t k = var_off[i + 1] - var_off[i];
        if (k < 1 || k > FC_MAX_VARS) {
            set_error("query %lld has %lld variables (need 1..%d)", (long long)i, (long long)k,
                      FC_MAX_VARS);
            return FC_ERR_INVALID;
        }
        const int32_t *v = vars_flat + var_off[i];
        int64_t c = 1;
        for (int64_t t = 0; t < k; ++t) {
            if (v[t] < 0 || v[t] >= db->n) {
                set_error("query %lld: variable %d out of range [0, %d)", (long long)i, v[t],
                          db->n);
                return FC_ERR_INVALID;
            }
            for (int64_t u = 0; u < t; ++u)
                if (v[u] == v[t]) {
                    set_error("query %lld: variable %d appears twice", (long long)i, v[t]);
                    return FC_ERR_INVALID;
                }
            c *= db->arity[v[t]];
        }
        if (c > INT32_MAX) {
            set_error("query %lld: table of %lld cells exceeds int32 indexing", (long long)i,
                      (long long)c);
            return FC_ERR_RANGE;
        }
        cells[(size_t)i] = c;
    }
    if (table_off) {
        int64_t total = table_off[nq];
        for (int64_t i = 0; i < nq; ++i)
            if (table_off[i] < 0 || table_off[i] + cells[(size_t)i] > total) {
                set_error("query %lld: table_off places its %lld cells outside [0, %lld)",
                          (long long)i, (long long)cells[(size_t)i], (long long)total);
                return FC_ERR_INVALID;
            }
    }
    return FC_OK;
}

// Row chunks per descriptor.  Small chunks keep one row range of every
// column of the batch inside an XCD's L2 (the XCD-aware block order deals
// chunk x, x+8, ... of every descriptor to XCD x); each chunk costs one flush
// of the partial table, so chunks never get shorter than 8 cells per row.
static int32_t pick_chunks(const fc_db *db, int64_t nd, int64_t cells, int strat) {
    const int64_t tiles = db->m_pad / kTileRows;
    int64_t rows = strat == S_BITMAP ? db->tune.bitmap_chunk_rows : db->tune.chunk_rows;
    if (rows <= 0) rows = 65536;
    rows = std::max<int64_t>(rows, 8 * cells);
    int64_t ch = (db->m_pad + rows - 1) / rows;
    // enough workgroups for a small batch (4 per CU)
    const int64_t want = (4 * (int64_t)db->cu_count + nd - 1) / nd;
    if (ch < want) ch = std::min<int64_t>(want, std::max<int64_t>(1, db->m_pad / (8 * cells)));
    ch = std::min(ch, tiles);
    if (ch >= kXcds) ch -= ch % kXcds;
    if (ch < 1) ch = 1;
    return (int32_t)ch;
}

// Planning: validation, cells, table offsets, strategy per query shape, and
// the grouping of descriptors into launches, in two passes over contiguous
// query ranges (several host threads for large batches): pass 1 validates and
// counts the descriptors of every launch bucket, pass 2 writes each
// descriptor straight into its final slot.  The order inside a bucket is the
// query order, whatever the number of threads.
constexpr int kBuckets = 3 * 8 * 7 * 2;  // strategy x K x LDS class x 24-bit strides

static inline int bucket_of(int st, int K, int cls, bool small) {
    return (((st - 1) * 8 + (K - 1)) * 7 + cls) * 2 + (small ? 1 : 0);
}

namespace {
struct RangeStat {
    int64_t lo = 0, hi = 0;
    int64_t err_q = -1;
    int err_code = FC_OK;
    std::string err;
    int64_t cells_sum = 0;
    bool windows = false;
    std::vector<int64_t> cnt, cur;
    std::vector<double> bytes;
    std::vector<int32_t> maxc;
    int64_t nsmall = 0, gcur = 0;   // one- and two-variable queries; their cursor
    std::vector<uint8_t> used;      // [n] variables of those queries
    int64_t npart = 0, pcur = 0;    // one-pass partition queries; their cursor
    double pbytes = 0.0;
};

// Whether a partitioned query takes the one-pass partition (its parts fit
// the part table and one query's scratch fits the slice budget); else key
// windows, each a scan of the columns.
inline bool one_pass(const fc_db *db, int64_t c) {
    return db->tune.one_pass && db->m > 0 && c <= (int64_t)kPartMax * kPartCells &&
           part_qbytes(db->m) <= kPartBudget;
}

// Strategy of one query (validated), and its window size for partitions.
inline int choose(const fc_db *db, uint32_t forced, int64_t k, int64_t c, int64_t &win) {
    int st;
    if (forced == FC_STRAT_BITMAP)
        st = c <= 128 ? S_BITMAP : (c <= kHistMaxCells ? S_HIST : S_PART);
    else if (forced == FC_STRAT_HIST)
        st = c <= kHistMaxCells ? S_HIST : S_PART;
    else if (forced == FC_STRAT_PARTITION)
        st = S_PART;
    else if (db->d_bits && db->tune.bitmap_for((int)k, c))
        st = S_BITMAP;
    else
        st = c <= kHistMaxCells ? S_HIST : S_PART;
    win = c;
    if (st == S_PART) {
        // windows over the top key digits: at least two when forced
        win = kHistMaxCells;
        if (forced == FC_STRAT_PARTITION && c <= kHistMaxCells) win = (c + 1) / 2;
        if (win < 1) win = 1;
    }
    return st;
}

// Validates query i; returns its cells (> 0) or 0 with the error filled in.
inline int64_t check_one(const fc_db *db, const int32_t *vars_flat, const int64_t *var_off,
                         int64_t i, RangeStat &R) {
    const int64_t k = var_off[i + 1] - var_off[i];
    char buf[160];
    if (k < 1 || k > FC_MAX_VARS) {
        snprintf(buf, sizeof buf, "query %lld has %lld variables (need 1..%d)", (long long)i,
                 (long long)k, FC_MAX_VARS);
        R.err = buf;
        R.err_code = FC_ERR_INVALID;
        return 0;
    }
    const int32_t *v = vars_flat + var_off[i];
    int64_t c = 1;
    for (int64_t t = 0; t < k; ++t) {
        if (v[t] < 0 || v[t] >= db->n) {
            snprintf(buf, sizeof buf, "query %lld: variable %d out of range [0, %d)", (long long)i,
                     v[t], db->n);
            R.err = buf;
            R.err_code = FC_ERR_INVALID;
            return 0;
        }
        for (int64_t u = 0; u < t; ++u)
            if (v[u] == v[t]) {
                snprintf(buf, sizeof buf, "query %lld: variable %d appears twice", (long long)i,
                         v[t]);
                R.err = buf;
                R.err_code = FC_ERR_INVALID;
                return 0;
            }
        c *= db->arity[v[t]];
        if (c > INT32_MAX) {
            snprintf(buf, sizeof buf, "query %lld: table exceeds int32 indexing (use the sparse "
                     "path)", (long long)i);
            R.err = buf;
            R.err_code = FC_ERR_RANGE;
            return 0;
        }
    }
    return c;
}

// ------------------------------------------------------- derived tables
// A table is exactly the marginal of the table of any query whose variable
// set contains its own (the count over a set of variables is the sum of the
// counts of its extensions; Section 2).  In an automatic plan, a query of
// three or four variables whose set lies inside another query of the batch
// (or repeats one) is not counted from the instances: its table is summed
// out of a counted superset's table after the counting launches.  Sources
// are always counted queries: `src[i]` of a derived query resolves through
// subset links and repeats to a query that no other query of the batch
// contains (or one too costly to derive).
constexpr int64_t kMargMaxCells = 16384;  // derived tables accumulate in 64 KiB of LDS

namespace {
inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// One partition of an open-addressing map from a variable-set key (never
// 0) to a query index, keeping the entry that `better` prefers.  Key and
// value share a 16-byte slot, so a probe touches one cache line.
struct SetMap {
    struct Slot {
        uint64_t key;
        int32_t val;
        int32_t pad;
    };
    std::vector<Slot> slots;
    uint64_t mask = 0;
    void init(size_t entries) {
        size_t cap = 16;
        while (cap < 2 * entries) cap <<= 1;
        slots.assign(cap, Slot{0, -1, 0});
        mask = cap - 1;
    }
    template <typename Better>
    void put(uint64_t key, uint64_t h, int32_t v, Better better) {
        for (uint64_t i = h & mask;; i = (i + 1) & mask) {
            Slot &e = slots[i];
            if (e.key == 0) {
                e.key = key;
                e.val = v;
                return;
            }
            if (e.key == key) {
                if (better(v, e.val)) e.val = v;
                return;
            }
        }
    }
    int32_t get(uint64_t key, uint64_t h) const {
        if (slots.empty()) return -1;
        for (uint64_t i = h & mask;; i = (i + 1) & mask) {
            const Slot &e = slots[i];
            if (e.key == key) return e.val;
            if (e.key == 0) return -1;
        }
    }
};
}  // namespace

// Fills src[i] (-1: counted from the instances) and returns the number of
// derived queries.  Needs at most 255 variables (a key packs the sorted
// variables + 1 as bytes); any malformed query disables derivation, and
// validation reports it.
// The planner's working arrays, kept per host thread between calls so that
// a steady stream of batches reuses their pages instead of faulting in new
// ones on every call.
struct DeriveScratch {
    static constexpr int kFiltBits = 20;
    std::vector<uint64_t> key;
    std::vector<int64_t> cells;
    std::vector<uint8_t> kk;
    std::vector<int32_t> rep;
    std::vector<std::vector<std::pair<uint64_t, int32_t>>> own;
    std::vector<SetMap> m0;
    std::unique_ptr<std::atomic<uint64_t>[]> filt{new std::atomic<uint64_t>[(size_t)1 << (kFiltBits - 6)]};
    std::unique_ptr<std::atomic<uint64_t>[]> best;
    size_t best_cap = 0;
};

static int64_t derive_plan(const fc_db *db, const int32_t *vars_flat, const int64_t *var_off,
                           int64_t nq, std::vector<int32_t> &src) {
    src.clear();
    if (nq < 2 || db->n > 255 || db->m <= 0) return 0;
    unsigned hw = std::thread::hardware_concurrency();
    const int T = (int)std::min<int64_t>(std::max<unsigned>(1u, std::min(16u, hw ? hw : 1u)),
                                         std::max<int64_t>(1, nq / 2048));
    static thread_local DeriveScratch W;
    W.key.resize((size_t)nq);
    W.cells.resize((size_t)nq);
    W.kk.resize((size_t)nq);
    W.rep.resize((size_t)nq);
    if (W.best_cap < (size_t)nq) {
        W.best.reset(new std::atomic<uint64_t>[(size_t)nq]);
        W.best_cap = (size_t)nq;
    }
    uint64_t *key = W.key.data();
    int64_t *cells = W.cells.data();
    uint8_t *kk = W.kk.data();
    int32_t *rep = W.rep.data();  // query of 3+ variables -> its representative
    std::atomic<uint64_t> *best = W.best.get();
    // per (range, owner partition): (own key, query) of queries of 3+ variables
    auto &own = W.own;
    own.resize((size_t)T * T);
    for (auto &v : own) v.clear();
    std::atomic<bool> bad(false);
    // a bit per hashed variable set of 3 or 4 variables present in the batch
    // (2^20 bits): most subsets of the larger queries are absent and are
    // turned away here without a probe of the map
    constexpr int kFiltBits = DeriveScratch::kFiltBits;
    std::atomic<uint64_t> *filt = W.filt.get();
    for (size_t i = 0; i < ((size_t)1 << (kFiltBits - 6)); ++i) filt[i].store(0, std::memory_order_relaxed);
    auto filt_bit = [](uint64_t h) { return h >> (64 - kFiltBits); };
    // owner partition of a hashed key: its high half scaled to [0, T), no division
    auto part_of = [T](uint64_t h) { return (size_t)(((h >> 32) * (uint64_t)T) >> 32); };
    auto run = [&](auto f) { parallel_for(T, [&](int t) { f(t); }); };
    // keys (sorted variables + 1 as bytes), cells
    run([&](int t) {
        const int64_t lo = nq * t / T, hi = nq * (t + 1) / T;
        for (int o = 0; o < T; ++o) own[(size_t)t * T + o].reserve((size_t)((hi - lo) / T + 16));
        for (int64_t i = lo; i < hi; ++i) best[i].store(~0ull, std::memory_order_relaxed);
        for (int64_t i = lo; i < hi; ++i) {
            const int64_t k = var_off[i + 1] - var_off[i];
            if (k < 1 || k > FC_MAX_VARS) {
                bad = true;
                return;
            }
            uint8_t v[FC_MAX_VARS];
            int64_t c = 1;
            for (int64_t a = 0; a < k; ++a) {
                const int32_t x = vars_flat[var_off[i] + a];
                if (x < 0 || x >= db->n) {
                    bad = true;
                    return;
                }
                v[a] = (uint8_t)(x + 1);
                c *= db->arity[x];
                if (c > INT32_MAX) c = INT32_MAX;
            }
            for (int64_t a = 1; a < k; ++a)  // insertion sort of at most 8 bytes
                for (int64_t b = a; b > 0 && v[b - 1] > v[b]; --b) std::swap(v[b - 1], v[b]);
            uint64_t kv = 0;
            for (int64_t a = 0; a < k; ++a) kv = (kv << 8) | v[a];
            key[(size_t)i] = kv;
            cells[(size_t)i] = c;
            kk[(size_t)i] = (uint8_t)k;
            if (k >= 3) {
                const uint64_t h = mix64(kv);
                own[(size_t)t * T + part_of(h)].push_back({kv, (int32_t)i});
            }
        }
    });
    if (bad) return 0;
    // representatives: every variable set of 3+ variables to its lowest
    // query; the filter bits of the sets of 3 or 4 variables are set here,
    // by the partition's owner (a partition's keys share the hash's high
    // bits, so its filter words are a range of their own: few contended
    // cache lines)
    auto &m0 = W.m0;
    m0.resize((size_t)T);
    run([&](int o) {
        size_t n0 = 0;
        for (int t = 0; t < T; ++t) n0 += own[(size_t)t * T + o].size();
        m0[(size_t)o].init(n0);
        for (int t = 0; t < T; ++t)
            for (auto &e : own[(size_t)t * T + o]) {
                const uint64_t h = mix64(e.first);
                m0[(size_t)o].put(e.first, h >> 8, e.second,
                                  [](int32_t a, int32_t b) { return a < b; });
                if (e.first < (1ull << 32)) {  // 3 or 4 variables, a byte each
                    const uint64_t b = filt_bit(h);
                    filt[(size_t)(b >> 6)].fetch_or(1ull << (b & 63), std::memory_order_relaxed);
                }
            }
    });
    // every query of 3+ variables to its representative, looked up by the
    // partition's owner while that map is in its thread's cache
    run([&](int o) {
        for (int t = 0; t < T; ++t)
            for (auto &e : own[(size_t)t * T + o])
                rep[(size_t)e.second] = m0[(size_t)o].get(e.first, mix64(e.first) >> 8);
    });
    // the smallest superset (fewest cells, then lowest index) of every
    // represented set of 3 or 4 variables: each query of 4+ variables looks
    // its sorted 3- and 4-variable subsets up and offers itself to those
    // that some query has.  A query's subsets that pass the filter are
    // staged with their map slots prefetched, then probed, so the probes'
    // memory latencies overlap.
    run([&](int t) {
        const int64_t lo = nq * t / T, hi = nq * (t + 1) / T;
        uint64_t skb[126], hb[126];  // C(8,3) + C(8,4) subsets at most
        int32_t rb[126];
        for (int64_t i = lo; i < hi; ++i) {
            const int k = kk[(size_t)i];
            if (k < 4) continue;
            uint8_t v[FC_MAX_VARS];
            for (int a = 0; a < k; ++a) v[a] = (uint8_t)(key[(size_t)i] >> (8 * (k - 1 - a)));
            const uint64_t mine = ((uint64_t)cells[(size_t)i] << 32) | (uint64_t)i;
            int ns = 0;
            auto stage = [&](uint64_t sk) {
                const uint64_t h = mix64(sk);
                const uint64_t bit = filt_bit(h);
                if (!((filt[(size_t)(bit >> 6)].load(std::memory_order_relaxed) >> (bit & 63)) & 1))
                    return;
                const SetMap &mp = m0[part_of(h)];
                __builtin_prefetch(&mp.slots[(h >> 8) & mp.mask]);
                skb[ns] = sk;
                hb[ns] = h;
                ++ns;
            };
            for (int a = 0; a < k; ++a)
                for (int b = a + 1; b < k; ++b)
                    for (int d = b + 1; d < k; ++d) {
                        const uint64_t s3 = ((uint64_t)v[a] << 16) | ((uint64_t)v[b] << 8) | v[d];
                        stage(s3);
                        if (k < 5) continue;
                        for (int e = d + 1; e < k; ++e) stage((s3 << 8) | v[e]);
                    }
            int nr = 0;
            for (int j = 0; j < ns; ++j) {
                const int32_t r = m0[part_of(hb[j])].get(skb[j], hb[j] >> 8);
                if (r < 0) continue;
                __builtin_prefetch(&best[(size_t)r]);
                rb[nr++] = r;
            }
            for (int j = 0; j < nr; ++j) {
                std::atomic<uint64_t> &slot = best[(size_t)rb[j]];
                uint64_t cur = slot.load(std::memory_order_relaxed);
                while (mine < cur &&
                       !slot.compare_exchange_weak(cur, mine, std::memory_order_relaxed)) {
                }
            }
        }
    });
    src.assign((size_t)nq, -1);
    // The chain of query i: its representative (lowest index with the same
    // variable set), then the representatives of successive smallest
    // supersets while the set has 3 or 4 variables.  The top of a chain is
    // counted; a member below it is derived when a counted member above can
    // serve it (at most kMargMaxCells cells to accumulate, and the source's
    // cells cheap against the instances), else counted.  Every query of a
    // chain computes the same decisions, so sources are always counted.
    const int64_t m = db->m;
    auto serves = [&](int32_t from, int32_t to) {
        return cells[(size_t)to] <= kMargMaxCells && cells[(size_t)from] * 32 <= m * kk[(size_t)to];
    };
    run([&](int t) {
        const int64_t lo = nq * t / T, hi = nq * (t + 1) / T;
        for (int64_t i = lo; i < hi; ++i) {
            if (kk[(size_t)i] < 3 || cells[(size_t)i] > kMargMaxCells) continue;
            int32_t ch[FC_MAX_VARS + 1];
            int L = 0;
            ch[L++] = rep[(size_t)i];
            while (L < FC_MAX_VARS + 1) {
                const int32_t r = ch[L - 1];
                const int kr = kk[(size_t)r];
                const uint64_t bu = (kr == 3 || kr == 4) ? best[(size_t)r].load(std::memory_order_relaxed)
                                                         : ~0ull;
                if (bu == ~0ull) break;
                const int32_t up = (int32_t)(bu & 0xFFFFFFFFull);
                ch[L++] = rep[(size_t)up];
            }
            bool counted[FC_MAX_VARS + 1];
            counted[L - 1] = true;
            for (int j = L - 2; j >= 0; --j) {
                counted[j] = true;
                for (int l = j + 1; l < L && counted[j]; ++l)
                    if (counted[l] && serves(ch[l], ch[j])) counted[j] = false;
            }
            // the lowest counted member (other than i) that serves i
            for (int l = 0; l < L; ++l)
                if (ch[l] != (int32_t)i && counted[l] && serves(ch[l], (int32_t)i)) {
                    src[(size_t)i] = ch[l];
                    break;
                }
        }
    });
    // a source must itself be counted: one that is derived by the rule above
    // (only possible through the cost bound) makes its dependants counted
    int64_t n = 0;
    for (int64_t i = 0; i < nq; ++i) {
        const int32_t r = src[(size_t)i];
        if (r >= 0 && src[(size_t)r] >= 0) src[(size_t)i] = -1;
        if (src[(size_t)i] >= 0) ++n;
    }
    return n;
}

// Order in which a Bitmap tree walks the variables of descriptor d, three
// bits per level (level L walks query position (code >> 3L) & 7): ascending
// marginal entropy, ties by lower variable index (Section 3.2: a
// low-entropy variable first leaves fewer non-empty prefixes to extend), or
// the query's own order when the tuning says so.
static uint32_t walk_order(const fc_db *db, const QDesc &d) {
    int32_t perm[FC_MAX_VARS];
    for (int32_t t = 0; t < d.k; ++t) perm[t] = t;
    if (db->tune.bitmap_order)
        std::stable_sort(perm, perm + d.k, [&](int32_t a, int32_t b) {
            const float ea = db->entropy[(size_t)d.var[a]], eb = db->entropy[(size_t)d.var[b]];
            return ea != eb ? ea < eb : d.var[a] < d.var[b];
        });
    uint32_t code = 0;
    for (int32_t L = 0; L < d.k; ++L) code |= (uint32_t)perm[L] << (3 * L);
    return code;
}

template <typename F>
void parallel_ranges(std::vector<RangeStat> &R, F f) {
    parallel_for((int)R.size(), [&](int t) { f(R[(size_t)t]); });
}
}  // namespace

static int build_plan(const fc_db *db, const int32_t *vars_flat, const int64_t *var_off,
                      int64_t nq, const int64_t *table_off, uint32_t flags, bool reducers,
                      Plan &P) {
    if (!db) {
        set_error("NULL database handle");
        return FC_ERR_INVALID;
    }
    if (nq < 0 || (nq > 0 && (!vars_flat || !var_off))) {
        set_error("need nq >= 0, vars_flat and var_off");
        return FC_ERR_INVALID;
    }
    if (nq > (int64_t)INT32_MAX / 2) {
        set_error("batch of %lld queries is too large", (long long)nq);
        return FC_ERR_RANGE;
    }
    if (nq > 0 && var_off[0] != 0) {
        set_error("var_off[0] must be 0");
        return FC_ERR_INVALID;
    }
    const uint32_t forced = flags & FC_STRAT_MASK;
    if (forced > FC_STRAT_PARTITION) {
        set_error("unknown strategy %u", forced);
        return FC_ERR_INVALID;
    }
    if (forced == FC_STRAT_BITMAP && !db->d_bits) {
        set_error("FC_STRAT_BITMAP needs a database created with FC_DB_BITVECTORS");
        return FC_ERR_INVALID;
    }
    P.packed = table_off == nullptr;
    P.nq = nq;
    const int64_t total_cells_in = table_off ? table_off[nq] : 0;
    const bool gram_allowed = forced == FC_STRAT_AUTO && db->d_bits && db->m > 0;
    unsigned hw = std::thread::hardware_concurrency();
    int64_t T = std::min<int64_t>(std::max<unsigned>(1u, std::min(16u, hw ? hw : 1u)),
                                  std::max<int64_t>(1, nq / 4096));  // workers persist: cheap
    std::vector<RangeStat> R((size_t)T);
    for (int64_t t = 0; t < T; ++t) {
        R[(size_t)t].lo = nq * t / T;
        R[(size_t)t].hi = nq * (t + 1) / T;
        R[(size_t)t].cnt.assign(kBuckets, 0);
        R[(size_t)t].bytes.assign(kBuckets, 0.0);
        R[(size_t)t].maxc.assign(kBuckets, 0);
        if (gram_allowed) R[(size_t)t].used.assign((size_t)db->n, 0);
    }
    // tables derivable from a counted superset's table (automatic plans)
    std::vector<int32_t> dsrc;
    const bool derive = forced == FC_STRAT_AUTO && db->tune.derive &&
                        derive_plan(db, vars_flat, var_off, nq, dsrc) > 0;
    // pass 1: validate, count descriptors per bucket
    parallel_ranges(R, [&](RangeStat &r) {
        for (int64_t i = r.lo; i < r.hi; ++i) {
            const int64_t c = check_one(db, vars_flat, var_off, i, r);
            if (!c) {
                r.err_q = i;
                return;
            }
            if (table_off && (table_off[i] < 0 || table_off[i] + c > total_cells_in)) {
                char buf[160];
                snprintf(buf, sizeof buf, "query %lld: table_off places its %lld cells outside "
                         "[0, %lld)", (long long)i, (long long)c, (long long)total_cells_in);
                r.err = buf;
                r.err_code = FC_ERR_INVALID;
                r.err_q = i;
                return;
            }
            const int64_t k = var_off[i + 1] - var_off[i];
            int64_t win;
            const int st = choose(db, forced, k, c, win);
            const bool small = c < (int64_t(1) << 24);
            r.cells_sum += c;
            if (derive && dsrc[(size_t)i] >= 0) continue;  // summed out of another table
            if (k <= 2 && gram_allowed) {
                ++r.nsmall;
                for (int64_t t = 0; t < k; ++t) r.used[(size_t)vars_flat[var_off[i] + t]] = 1;
            } else if (st == S_PART && one_pass(db, c)) {
                ++r.npart;
                r.pbytes += (double)k * (double)db->m;
                continue;
            }
            for (int64_t b0 = 0; b0 < c; b0 += win) {
                const int64_t wc = std::min<int64_t>(win, c - b0);
                const int b = st == S_BITMAP ? bucket_of(S_BITMAP, (int)k, 0, false)
                                             : bucket_of(st, (int)k, hist_class(wc), small);
                r.cnt[(size_t)b] += 1;
                r.bytes[(size_t)b] += (double)k * (double)db->m * ((double)wc / (double)c);
                r.maxc[(size_t)b] = std::max<int32_t>(r.maxc[(size_t)b], (int32_t)wc);
                if (st == S_PART) r.windows = true;
            }
        }
    });
    for (auto &r : R)
        if (r.err_q >= 0) {
            set_error("%s", r.err.c_str());
            return r.err_code;
        }
    P.windows = false;
    for (auto &r : R) P.windows = P.windows || r.windows;
    // Gram of the small queries' state bit-vectors instead of their own
    // launches, when estimated at most half their cost: about 2e15 useful
    // operations/s on the matrix cores plus a launch, against about 3e13
    // query-instances/s for one- and two-variable counts
    bool use_gram = false;
    if (gram_allowed) {
        int64_t nsmall = 0;
        for (auto &r : R) nsmall += r.nsmall;
        std::vector<uint8_t> used((size_t)db->n, 0);
        for (auto &r : R)
            for (int32_t v = 0; v < db->n; ++v) used[(size_t)v] |= r.used[(size_t)v];
        int64_t states = 0;
        for (int32_t v = 0; v < db->n; ++v)
            if (used[(size_t)v]) states += db->arity[(size_t)v];
        const int64_t np = (states + kGramBlock - 1) / kGramBlock * kGramBlock;
        const double t_gram = (double)np * (double)np * (double)db->m / 2e15 + 20e-6;
        const double t_small = (double)nsmall * (double)db->m * 3e-14;
        if (nsmall > 0 && np <= kGramMaxRows && t_gram < 0.5 * t_small) {
            use_gram = true;
            P.gram_np = (int32_t)np;
            P.gram_rows.assign((size_t)np, -1);
            P.gram_pos.assign((size_t)db->n, -1);
            int32_t row = 0;
            for (int32_t v = 0; v < db->n; ++v)
                if (used[(size_t)v]) {
                    P.gram_pos[(size_t)v] = row;
                    for (int32_t st = 0; st < db->arity[(size_t)v]; ++st)
                        P.gram_rows[(size_t)row++] = db->state_off[(size_t)v] + st;
                }
            P.gram_ops = (double)db->m * (double)states * (double)(states + 1);
            // their buckets (K = 1, 2) empty out: every such query is here
            for (auto &r : R)
                for (int st = 1; st <= 3; ++st)
                    for (int K = 1; K <= 2; ++K)
                        for (int cls = 0; cls < 7; ++cls)
                            for (int sm = 0; sm < 2; ++sm) {
                                const int b = bucket_of(st, K, cls, sm != 0);
                                P.gram_bytes += r.bytes[(size_t)b];
                                r.cnt[(size_t)b] = 0;
                                r.bytes[(size_t)b] = 0.0;
                            }
        }
    }
    // bucket starts (launch order) and per-range cursors
    std::vector<int64_t> start(kBuckets + 1, 0);
    for (int b = 0; b < kBuckets; ++b) {
        int64_t tot = 0;
        for (auto &r : R) tot += r.cnt[(size_t)b];
        start[(size_t)b + 1] = start[(size_t)b] + tot;
    }
    {
        std::vector<int64_t> run(start.begin(), start.end() - 1);
        for (auto &r : R) {
            r.cur.assign(kBuckets, 0);
            for (int b = 0; b < kBuckets; ++b) {
                r.cur[(size_t)b] = run[(size_t)b];
                run[(size_t)b] += r.cnt[(size_t)b];
            }
        }
    }
    const bool need_query = !P.packed || (reducers && P.windows) || derive;
    P.gram_first = start[kBuckets];
    P.gram_count = 0;
    if (use_gram)
        for (auto &r : R) {
            r.gcur = P.gram_first + P.gram_count;
            P.gram_count += r.nsmall;
        }
    P.part_first = start[kBuckets] + P.gram_count;
    P.part_count = 0;
    P.part_bytes = 0.0;
    for (auto &r : R) {
        r.pcur = P.part_first + P.part_count;
        P.part_count += r.npart;
        P.part_bytes += r.pbytes;
    }
    P.work.resize((size_t)(P.part_first + P.part_count));
    if (need_query) P.query.resize((size_t)nq);
    std::vector<int64_t> base((size_t)T, 0);
    for (int64_t t = 1; t < T; ++t) base[(size_t)t] = base[(size_t)t - 1] + R[(size_t)t - 1].cells_sum;
    P.total_cells = table_off ? total_cells_in : (T ? base[(size_t)T - 1] + R[(size_t)T - 1].cells_sum : 0);
    // pass 2: write every descriptor into its slot
    for (int64_t t = 0; t < T; ++t) R[(size_t)t].cells_sum = base[(size_t)t];  // reuse as offset
    parallel_ranges(R, [&](RangeStat &r) {
        int64_t off = r.cells_sum;
        for (int64_t i = r.lo; i < r.hi; ++i) {
            const int64_t k = var_off[i + 1] - var_off[i];
            int64_t c = 1;
            QDesc d;
            std::memset(&d, 0, sizeof d);
            for (int64_t t = 0; t < k; ++t) {
                d.var[t] = vars_flat[var_off[i] + t];
                c *= db->arity[d.var[t]];
            }
            d.k = (int32_t)k;
            d.cells = (int32_t)c;
            d.qid = (int32_t)i;
            d.table_off = table_off ? table_off[i] : off;
            off += c;
            d.win_base = 0;
            d.win_cells = (int32_t)c;
            d.tiles = (int32_t)(db->m_pad / kTileRows);
            if (need_query) P.query[(size_t)i] = d;
            if (derive && dsrc[(size_t)i] >= 0) continue;
            if (use_gram && k <= 2) {
                P.work[(size_t)r.gcur++] = d;
                continue;
            }
            int64_t win;
            const int st = choose(db, forced, k, c, win);
            const bool small = c < (int64_t(1) << 24);
            if (st == S_PART && one_pass(db, c) && !(k <= 2 && gram_allowed)) {
                P.work[(size_t)r.pcur++] = d;  // as counted in pass 1
                continue;
            }
            for (int64_t b0 = 0; b0 < c; b0 += win) {
                const int64_t wc = std::min<int64_t>(win, c - b0);
                const int b = st == S_BITMAP ? bucket_of(S_BITMAP, (int)k, 0, false)
                                             : bucket_of(st, (int)k, hist_class(wc), small);
                QDesc w = d;
                w.win_base = (int32_t)b0;
                w.win_cells = (int32_t)wc;
                if (st == S_BITMAP) w.win_base = (int32_t)walk_order(db, d);
                P.work[(size_t)r.cur[(size_t)b]++] = w;
            }
        }
    });
    for (int st = 1; st <= 3; ++st)
        for (int K = 1; K <= 8; ++K)
            for (int cls = 0; cls < 7; ++cls)
                for (int sm = 0; sm < 2; ++sm) {
                    const int b = bucket_of(st, K, cls, sm != 0);
                    const int64_t cnt = start[(size_t)b + 1] - start[(size_t)b];
                    if (!cnt) continue;
                    Launch L;
                    L.strat = st;
                    L.K = K;
                    L.small = sm != 0;
                    L.first = start[(size_t)b];
                    L.count = (int32_t)cnt;
                    int64_t maxc = 0;
                    double bytes = 0.0;
                    for (auto &r : R) {
                        maxc = std::max<int64_t>(maxc, r.maxc[(size_t)b]);
                        bytes += r.bytes[(size_t)b];
                    }
                    L.chunks = pick_chunks(db, L.count, maxc, st);
                    const bool nib = db->d_nib && db->tune.packed_columns;
                    L.hk = st != S_HIST                    ? HK_GENERIC
                           : cls < kHist8Classes            ? (nib ? HK_HIST8N : HK_HIST8)
                           : nib && cls < kHist16Classes    ? HK_HIST16N
                           : cls < kHist16Classes           ? HK_HIST16
                                                            : HK_GENERIC;
                    // algorithmic bytes: k per (query, instance) whichever
                    // column store or strategy the launch reads
                    L.lds_bytes = st == S_BITMAP ? (int32_t)(maxc * kBlock * 4) : kClassLds[cls];
                    L.alg_bytes = bytes;
                    if (st == S_BITMAP)
                        snprintf(L.name, sizeof L.name, "k_bitmap<%d,%d>", K,
                                 db->tune.bitmap_words >= 4 ? 4 : db->tune.bitmap_words == 2 ? 2 : 1);
                    else if (L.hk == HK_HIST8 || L.hk == HK_HIST8N)  // <K, LDS cells>
                        snprintf(L.name, sizeof L.name, "k_hist8%s<%d,%d>",
                                 L.hk == HK_HIST8N ? "n" : "", K,
                                 L.lds_bytes <= 16 * 64 * 4   ? 16
                                 : L.lds_bytes <= 64 * 64 * 4 ? 64
                                                              : 256);
                    else if (L.hk == HK_HIST16N)
                        snprintf(L.name, sizeof L.name, "k_hist16n<%d>", K);
                    else if (L.hk == HK_HIST16)
                        snprintf(L.name, sizeof L.name, "k_hist16<%d>", K);
                    else
                        snprintf(L.name, sizeof L.name, "k_hist<%d,%d>", K, sm);
                    P.launches.push_back(L);
                }
    P.direct = db->m > 0;  // the partition zeroes its own tables
    for (const Launch &L : P.launches)
        if (L.strat == S_BITMAP || L.chunks != 1) P.direct = false;
    if (derive) {
        for (int64_t i = 0; i < nq; ++i) {
            const int32_t j = dsrc[(size_t)i];
            if (j < 0) continue;
            const QDesc &dq = P.query[(size_t)i], &sq = P.query[(size_t)j];
            MDesc m;
            std::memset(&m, 0, sizeof m);
            m.dst_off = dq.table_off;
            m.src_off = sq.table_off;
            m.dst_cells = dq.cells;
            m.src_cells = sq.cells;
            m.src_k = sq.k;
            for (int32_t a = 0; a < sq.k; ++a) {
                m.src_rad[a] = db->arity[(size_t)sq.var[a]];
                int32_t stride = 1;
                for (int32_t t = dq.k - 1; t >= 0; --t) {
                    if (dq.var[t] == sq.var[a]) {
                        m.dst_str[a] = stride;
                        break;
                    }
                    stride *= db->arity[(size_t)dq.var[t]];
                }
            }
            P.marg.push_back(m);
            P.marg_max_cells = std::max(P.marg_max_cells, dq.cells);
        }
    }
    return FC_OK;
}

// ------------------------------------------------------------------ launch
// Workgroups of kernel f (dyn bytes of dynamic LDS) one XCD holds at a time:
// the sweep argument of the histogram kernels (0 with row_sweep off).
static int32_t sweep_of(const fc_db *db, const void *f, int32_t dyn) {
    if (!db->tune.row_sweep) return 0;
    static std::mutex mu;
    static std::map<std::pair<const void *, int32_t>, int32_t> per_cu;
    int32_t nb = 0;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = per_cu.find({f, dyn});
        if (it != per_cu.end()) {
            nb = it->second;
        } else {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kBlock, (size_t)dyn) !=
                hipSuccess) {
                (void)hipGetLastError();
                nb = 0;
            }
            per_cu[{f, dyn}] = nb;
        }
    }
    return nb > 0 ? (int32_t)((int64_t)nb * db->cu_count / kXcds) : 0;
}

template <int K>
static hipError_t launch_hist_k(const fc_db *db, const Launch &L, const QDesc *d,
                                int32_t *tables, hipStream_t s) {
    const int64_t blocks = (int64_t)L.count * L.chunks;
    const int32_t pad = (int32_t)(db->m_pad - db->m);
    const dim3 grid((unsigned)blocks), block(kBlock);
    if (L.hk == HK_HIST8N && L.lds_bytes <= 16 * 64 * 4)
        hipLaunchKernelGGL((k_hist8n<K, 16>), grid, block, 0, s, db->d_nib, db->pitch,
                           db->d_arity, d, L.count, L.chunks, pad, tables,
                           sweep_of(db, (const void *)k_hist8n<K, 16>, 0));
    else if (L.hk == HK_HIST8N && L.lds_bytes <= 64 * 64 * 4)
        hipLaunchKernelGGL((k_hist8n<K, 64>), grid, block, 0, s, db->d_nib, db->pitch,
                           db->d_arity, d, L.count, L.chunks, pad, tables,
                           sweep_of(db, (const void *)k_hist8n<K, 64>, 0));
    else if (L.hk == HK_HIST8N)
        hipLaunchKernelGGL((k_hist8n<K, 256>), grid, block, 0, s, db->d_nib, db->pitch,
                           db->d_arity, d, L.count, L.chunks, pad, tables,
                           sweep_of(db, (const void *)k_hist8n<K, 256>, 0));
    else if (L.hk == HK_HIST16N)
        hipLaunchKernelGGL((k_hist16n<K>), grid, block, L.lds_bytes, s, db->d_nib, db->pitch,
                           db->d_arity, d, L.count, L.chunks, L.lds_bytes / 4, pad, tables,
                           sweep_of(db, (const void *)k_hist16n<K>, L.lds_bytes));
    else if (L.hk == HK_HIST8 && L.lds_bytes <= 16 * 64 * 4)
        hipLaunchKernelGGL((k_hist8<K, 16>), grid, block, 0, s, db->d_cols, db->pitch,
                           db->d_arity, d, L.count, L.chunks, pad, tables,
                           sweep_of(db, (const void *)k_hist8<K, 16>, 0));
    else if (L.hk == HK_HIST8 && L.lds_bytes <= 64 * 64 * 4)
        hipLaunchKernelGGL((k_hist8<K, 64>), grid, block, 0, s, db->d_cols, db->pitch,
                           db->d_arity, d, L.count, L.chunks, pad, tables,
                           sweep_of(db, (const void *)k_hist8<K, 64>, 0));
    else if (L.hk == HK_HIST8)
        hipLaunchKernelGGL((k_hist8<K, 256>), grid, block, 0, s, db->d_cols, db->pitch,
                           db->d_arity, d, L.count, L.chunks, pad, tables,
                           sweep_of(db, (const void *)k_hist8<K, 256>, 0));
    else if (L.hk == HK_HIST16)
        hipLaunchKernelGGL((k_hist16<K>), grid, block, L.lds_bytes, s, db->d_cols, db->pitch,
                           db->d_arity, d, L.count, L.chunks, L.lds_bytes / 4, pad, tables,
                           sweep_of(db, (const void *)k_hist16<K>, L.lds_bytes));
    else if (L.small)
        hipLaunchKernelGGL((k_hist<K, true>), dim3((unsigned)blocks), dim3(kBlock), L.lds_bytes,
                           s, db->d_cols, db->pitch, db->d_arity, d, L.count, L.chunks,
                           L.lds_bytes / 4, pad, tables);
    else
        hipLaunchKernelGGL((k_hist<K, false>), dim3((unsigned)blocks), dim3(kBlock), L.lds_bytes,
                           s, db->d_cols, db->pitch, db->d_arity, d, L.count, L.chunks,
                           L.lds_bytes / 4, pad, tables);
    return hipGetLastError();
}

template <int K>
static hipError_t launch_bitmap_k(const fc_db *db, const Launch &L, const QDesc *d,
                                  int32_t *tables, hipStream_t s) {
    const int64_t blocks = (int64_t)L.count * L.chunks;
    if (db->tune.bitmap_words >= 4)
        hipLaunchKernelGGL((k_bitmap<K, 4>), dim3((unsigned)blocks), dim3(kBlock), L.lds_bytes,
                           s, db->d_bits, db->pitch / 64, db->d_soff, db->d_arity, d, L.count,
                           L.chunks, tables);
    else if (db->tune.bitmap_words == 2)
        hipLaunchKernelGGL((k_bitmap<K, 2>), dim3((unsigned)blocks), dim3(kBlock), L.lds_bytes,
                           s, db->d_bits, db->pitch / 64, db->d_soff, db->d_arity, d, L.count,
                           L.chunks, tables);
    else
        hipLaunchKernelGGL((k_bitmap<K, 1>), dim3((unsigned)blocks), dim3(kBlock), L.lds_bytes,
                           s, db->d_bits, db->pitch / 64, db->d_soff, db->d_arity, d, L.count,
                           L.chunks, tables);
    return hipGetLastError();
}

template <int K>
static hipError_t launch_one(const fc_db *db, const Launch &L, const QDesc *d, int32_t *t,
                             hipStream_t s) {
    return L.strat == S_BITMAP ? launch_bitmap_k<K>(db, L, d, t, s)
                               : launch_hist_k<K>(db, L, d, t, s);
}

static hipError_t launch_count(const fc_db *db, const Launch &L, const QDesc *d_work,
                               int32_t *tables, hipStream_t s) {
    const QDesc *d = d_work + L.first;
    switch (L.K) {
        case 1: return launch_one<1>(db, L, d, tables, s);
        case 2: return launch_one<2>(db, L, d, tables, s);
        case 3: return launch_one<3>(db, L, d, tables, s);
        case 4: return launch_one<4>(db, L, d, tables, s);
        case 5: return launch_one<5>(db, L, d, tables, s);
        case 6: return launch_one<6>(db, L, d, tables, s);
        case 7: return launch_one<7>(db, L, d, tables, s);
        default: return launch_one<8>(db, L, d, tables, s);
    }
}

static bool g_lds_attr_set = false;
static std::mutex g_attr_mu;

template <int K>
static void set_attrs_k() {
    (void)hipFuncSetAttribute((const void *)k_hist<K, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytesMax);
    (void)hipFuncSetAttribute((const void *)k_hist<K, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytesMax);
    (void)hipFuncSetAttribute((const void *)k_hist16<K>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytesMax);
    (void)hipFuncSetAttribute((const void *)k_hist16n<K>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytesMax);
    (void)hipFuncSetAttribute((const void *)k_bitmap<K, 1>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytesMax);
    (void)hipFuncSetAttribute((const void *)k_bitmap<K, 2>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytesMax);
    (void)hipFuncSetAttribute((const void *)k_bitmap<K, 4>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytesMax);
}

static void ensure_attrs() {
    std::lock_guard<std::mutex> lk(g_attr_mu);
    if (g_lds_attr_set) return;
    set_attrs_k<1>(); set_attrs_k<2>(); set_attrs_k<3>(); set_attrs_k<4>();
    set_attrs_k<5>(); set_attrs_k<6>(); set_attrs_k<7>(); set_attrs_k<8>();
    for (const void *f : {(const void *)k_count_persistent<1>, (const void *)k_count_persistent<2>,
                          (const void *)k_count_persistent<4>})
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kPersistentLds);
    (void)hipGetLastError();
    g_lds_attr_set = true;
}


template <int W>
static hipError_t launch_persistent_w(const fc_db *db, const PGroup *d_groups, int32_t ngroups,
                                      int64_t vtotal, uint32_t *heads, int32_t lds,
                                      const QDesc *dw, int32_t *tables, hipStream_t s) {
    static std::atomic<int> per_cu{0};  // resident workgroups per CU (one value per W)
    int nb = per_cu.load(std::memory_order_relaxed);
    if (!nb) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_count_persistent<W>, kBlock,
                                                         kPersistentLds) != hipSuccess || nb < 1) {
            (void)hipGetLastError();
            nb = 2;
        }
        per_cu.store(nb, std::memory_order_relaxed);
    }
    int64_t grid = (int64_t)nb * db->cu_count;
    grid = std::min<int64_t>(grid, vtotal);
    grid = std::max<int64_t>(grid, 1);
    hipLaunchKernelGGL((k_count_persistent<W>), dim3((unsigned)grid), dim3(kBlock), lds, s,
                       db->d_cols, db->d_nib, db->pitch, db->d_bits, db->pitch / 64, db->d_soff,
                       db->d_arity, dw,
                       d_groups, ngroups, vtotal, heads, lds / 4, (int32_t)(db->m_pad - db->m),
                       tables);
    return hipGetLastError();
}

// Device image of a planned batch: one buffer with the counting descriptors,
// the per-query descriptors (reducers, zeroing of caller-placed tables), the
// persistent group table and the eight queue heads.
struct Image {
    std::vector<PGroup> groups;
    std::vector<const Launch *> solo;
    int64_t vtotal = 0;
    int32_t plds = 0;
    double pbytes = 0.0;
    bool with_query = false;
    size_t off_query = 0, off_groups = 0, off_heads = 0, bytes = 0;
    size_t off_gram_rows = 0, off_gram_pos = 0, off_gram_c = 0, off_marg = 0;
    size_t dev_bytes = 0;  // bytes plus the device-only state Gram and partition scratch
    size_t off_part = 0, part_qstride = 0;
    int64_t part_slice = 0;  // partition queries per slice (they share the scratch)
};

static void make_image(const fc_db *db, const Plan &P, uint32_t reducers, Image &I) {
    // Groups of the persistent launch in decreasing cost of one work unit
    // (longest processing time first: the dearest units are claimed first
    // and the cheap ones fill in at the end): rows scanned per unit times
    // the key digits per row, plus the zeroing and flush of the table.
    std::vector<const Launch *> order;
    for (const Launch &L : P.launches) order.push_back(&L);
    if (P.nq <= db->tune.persistent_max_queries) {
        auto unit_cost = [&](const Launch *L) {
            const double rows = (double)db->m_pad / (double)std::max<int32_t>(L->chunks, 1);
            return rows * (double)(L->K + 1) + (double)L->lds_bytes;
        };
        std::stable_sort(order.begin(), order.end(), [&](const Launch *a, const Launch *b) {
            return unit_cost(a) > unit_cost(b);
        });
    }
    for (const Launch *Lp : order) {
        const Launch &L = *Lp;
        if (P.nq <= db->tune.persistent_max_queries &&
            L.lds_bytes <= kPersistentLds) {
            PGroup g;
            g.vbase = I.vtotal;
            g.nv = ((int64_t)L.count * L.chunks + kXcds - 1) / kXcds * kXcds;
            g.first = (int32_t)L.first;
            g.nd = L.count;
            g.chunks = L.chunks;
            // tables of these groups fit 16 KiB of LDS: the byte-key classes
            // (packed columns or bytes), Bitmap walks, or generic keys
            const int type = L.strat == S_BITMAP ? PK_BITMAP
                           : L.hk == HK_HIST8N ? PK_HIST8N
                           : L.hk == HK_HIST8 ? PK_HIST8
                           : (L.hk == HK_HIST16 || L.hk == HK_HIST16N) ? PK_HIST16
                           : L.small ? PK_HIST_S : PK_HIST_B;
            g.kind = (type << 4) | L.K;
            I.vtotal += g.nv;
            I.groups.push_back(g);
            I.pbytes += L.alg_bytes;
            I.plds = std::max(I.plds, L.lds_bytes);
        } else {
            I.solo.push_back(&L);
        }
    }
    I.with_query = !P.query.empty();
    size_t b = sizeof(QDesc) * P.work.size();
    I.off_query = b;
    if (I.with_query) b += sizeof(QDesc) * P.query.size();
    I.off_groups = b;
    b += sizeof(PGroup) * I.groups.size();
    I.off_heads = b;
    b += 64;
    I.off_gram_rows = b;
    b += sizeof(int32_t) * P.gram_rows.size();
    I.off_gram_pos = b;
    b += sizeof(int32_t) * P.gram_pos.size();
    b = (b + 15) & ~(size_t)15;
    I.off_marg = b;
    b += sizeof(MDesc) * P.marg.size();
    I.bytes = b;
    I.off_gram_c = (b + 255) & ~(size_t)255;
    I.dev_bytes = P.gram_count ? I.off_gram_c + sizeof(int32_t) * (size_t)P.gram_np *
                                                    (size_t)P.gram_np
                               : I.bytes;
    if (P.part_count) {
        I.part_qstride = part_qbytes(db->m);
        I.part_slice = std::max<int64_t>(
            1, std::min<int64_t>(P.part_count, (int64_t)(kPartBudget / I.part_qstride)));
        I.off_part = (I.dev_bytes + 255) & ~(size_t)255;
        I.dev_bytes = I.off_part + I.part_qstride * (size_t)I.part_slice;
    }
}

// memcpy split over host threads for large plans (pinned destination).
static void parallel_copy(void *dst, const void *src, size_t bytes) {
    const size_t kPiece = size_t(4) << 20;
    unsigned hw = std::thread::hardware_concurrency();
    const size_t T = std::min<size_t>(std::min(16u, hw ? hw : 1u), bytes / kPiece);
    if (T <= 1) {
        std::memcpy(dst, src, bytes);
        return;
    }
    parallel_for((int)T, [&](int t) {
        const size_t lo = bytes * (size_t)t / T, hi = bytes * (size_t)(t + 1) / T;
        std::memcpy((char *)dst + lo, (const char *)src + lo, hi - lo);
    });
}

static void fill_image(const Plan &P, const Image &I, void *host) {
    char *h = (char *)host;
    parallel_copy(h, P.work.data(), sizeof(QDesc) * P.work.size());
    if (I.with_query) std::memcpy(h + I.off_query, P.query.data(), sizeof(QDesc) * P.query.size());
    std::memcpy(h + I.off_groups, I.groups.data(), sizeof(PGroup) * I.groups.size());
    std::memset(h + I.off_heads, 0, 64);
    if (!P.gram_rows.empty())
        std::memcpy(h + I.off_gram_rows, P.gram_rows.data(), sizeof(int32_t) * P.gram_rows.size());
    if (!P.gram_pos.empty())
        std::memcpy(h + I.off_gram_pos, P.gram_pos.data(), sizeof(int32_t) * P.gram_pos.size());
    if (!P.marg.empty())
        std::memcpy(h + I.off_marg, P.marg.data(), sizeof(MDesc) * P.marg.size());
}

// The one-pass partition queries, a slice at a time (a slice's queries
// share the scratch; the slices follow each other on the stream).
__global__ void k_part_zero(char *scratch, size_t qstride) {
    uint32_t *cnt = (uint32_t *)(scratch + blockIdx.x * qstride);
    for (int32_t i = threadIdx.x; i < kPartMax; i += blockDim.x) cnt[i] = 0u;
}

static hipError_t enqueue_partition(const fc_db *db, const Plan &P, const Image &I,
                                    const QDesc *dw, char *scratch, int32_t *tables,
                                    hipStream_t s) {
    const int64_t m = db->m;
    const int cus = db->cu_count > 0 ? db->cu_count : 256;
    for (int64_t s0 = 0; s0 < P.part_count; s0 += I.part_slice) {
        const int64_t n = std::min<int64_t>(I.part_slice, P.part_count - s0);
        const QDesc *d = dw + P.part_first + s0;
        double bytes = 0.0;
        for (int64_t i = 0; i < n; ++i)
            bytes += (double)P.work[(size_t)(P.part_first + s0 + i)].k * (double)m;
        const int64_t tiles = (m + kPartTile - 1) / kPartTile;
        const unsigned gx = (unsigned)std::max<int64_t>(
            1, std::min<int64_t>(tiles, (8 * (int64_t)cus + n - 1) / n));
        const int64_t units_max = (m + kPartUnit - 1) / kPartUnit + kPartMax;
        const unsigned gc = (unsigned)std::max<int64_t>(
            1, std::min<int64_t>(units_max, (8 * (int64_t)cus + n - 1) / n));
        hipLaunchKernelGGL(k_part_zero, dim3((unsigned)n), dim3(256), 0, s, scratch,
                           I.part_qstride);
        if (P.direct)  // the other tables are stored whole; these are added to
            hipLaunchKernelGGL(k_zero_tables, dim3((unsigned)n), dim3(256), 0, s, d, (int32_t)n,
                               tables);
        {
            // algorithmic bytes: k per (query, instance), the columns read once
            ProfScope ps("k_part_keys", s, bytes, 0.0);
            hipLaunchKernelGGL(k_part_keys, dim3(gx, (unsigned)n), dim3(kBlock), 0, s, db->d_cols,
                               db->pitch, db->d_arity, d, m, scratch, I.part_qstride);
            ps.end(s);
        }
        hipLaunchKernelGGL(k_part_scan, dim3((unsigned)n), dim3(kBlock), 0, s, d, m, scratch,
                           I.part_qstride);
        {
            ProfScope ps("k_part_scatter", s, 0.0, 0.0);
            hipLaunchKernelGGL(k_part_scatter, dim3(gx, (unsigned)n), dim3(kBlock), 0, s, d, m,
                               scratch, I.part_qstride);
            ps.end(s);
        }
        {
            ProfScope ps("k_part_count", s, 0.0, 0.0);
            hipLaunchKernelGGL(k_part_count, dim3(gc, (unsigned)n), dim3(kBlock), 0, s, d, m,
                               scratch, I.part_qstride, tables);
            ps.end(s);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Every device step of a batch whose image is resident at `dimg`: zero the
// tables and queue heads (kernels, no memset nodes), count, reduce.  Safe to
// record into a hipGraph.
static int enqueue_batch(fc_db *db, const Plan &P, const Image &I, void *dimg, int32_t *tables,
                         uint32_t reducers, double ess, float *scores, float *err,
                         hipStream_t s) {
    const QDesc *dw = (const QDesc *)dimg;
    const QDesc *dq = (const QDesc *)((char *)dimg + I.off_query);
    if (P.direct) {
        // every cell is stored by its counting launch
    } else if (P.packed) {
        FC_HIP(fill_zero_i32(tables, P.total_cells, s));
    } else if (!P.query.empty()) {
        const int32_t nd = (int32_t)P.query.size();
        hipLaunchKernelGGL(k_zero_tables, dim3((unsigned)std::min<int32_t>(nd, 65536)), dim3(256),
                           0, s, dq, nd, tables);
        FC_HIP(hipGetLastError());
    }
    if (db->m > 0 && P.gram_count > 0) {
        const int32_t np = P.gram_np;
        int32_t *C = (int32_t *)((char *)dimg + I.off_gram_c);
        const int32_t *rows = (const int32_t *)((char *)dimg + I.off_gram_rows);
        const int32_t *pos = (const int32_t *)((char *)dimg + I.off_gram_pos);
        FC_HIP(fill_zero_i32(C, (int64_t)np * np, s));
        FC_HIP(launch_gram(db, rows, np, C, np, "k_gram_states", P.gram_bytes, P.gram_ops, s));
        const int64_t nd = P.gram_count;
        ProfScope ps("k_gram_tables", s, 0.0, 0.0);
        hipLaunchKernelGGL(k_gram_tables, dim3((unsigned)std::min<int64_t>(nd, 65536)), dim3(64),
                           0, s, dw + P.gram_first, nd, pos, db->d_arity, C, (int64_t)np, tables);
        ps.end(s);
        FC_HIP(hipGetLastError());
    }
    if (db->m > 0) {
        if (!I.groups.empty()) {
            uint32_t *heads = (uint32_t *)((char *)dimg + I.off_heads);
            FC_HIP(fill_zero_i32((int32_t *)heads, 16, s));
            const int W = db->tune.bitmap_words >= 4 ? 4 : db->tune.bitmap_words == 2 ? 2 : 1;
            char name[32];
            snprintf(name, sizeof name, "k_count_persistent<%d>", W);
            const PGroup *g = (const PGroup *)((char *)dimg + I.off_groups);
            const int32_t ng = (int32_t)I.groups.size();
            ProfScope ps(name, s, I.pbytes, 0.0);
            hipError_t e;
            if (W == 4)
                e = launch_persistent_w<4>(db, g, ng, I.vtotal, heads, I.plds, dw, tables, s);
            else if (W == 2)
                e = launch_persistent_w<2>(db, g, ng, I.vtotal, heads, I.plds, dw, tables, s);
            else
                e = launch_persistent_w<1>(db, g, ng, I.vtotal, heads, I.plds, dw, tables, s);
            ps.end(s);
            FC_HIP(e);
        }
        for (const Launch *L : I.solo) {
            ProfScope ps(L->name, s, L->alg_bytes, 0.0);
            FC_HIP(launch_count(db, *L, dw, tables, s));
            ps.end(s);
        }
        if (P.part_count) FC_HIP(enqueue_partition(db, P, I, dw, (char *)dimg + I.off_part, tables, s));
        if (!P.marg.empty()) {
            const MDesc *md = (const MDesc *)((char *)dimg + I.off_marg);
            const int64_t nm = (int64_t)P.marg.size();
            ProfScope ps("k_marginal", s, 0.0, 0.0);
            hipLaunchKernelGGL(k_marginal, dim3((unsigned)std::min<int64_t>(nm, 65536)),
                               dim3(kBlock), sizeof(uint32_t) * (size_t)P.marg_max_cells, s, md,
                               nm, tables);
            ps.end(s);
            FC_HIP(hipGetLastError());
        }
    }
    if (reducers && P.nq > 0) {
        // one descriptor per query: the per-query list when windows split a
        // query, else the counting descriptors themselves (scores go by qid)
        const QDesc *rd = I.with_query ? dq : dw;
        const int64_t nrd = I.with_query ? (int64_t)P.query.size() : (int64_t)P.work.size();
        ProfScope ps("k_reduce", s, 0.0, 0.0);
        FC_HIP(launch_reduce(db, rd, nrd, P.nq, tables, reducers, ess, scores, err, s));
        ps.end(s);
    }
    return FC_OK;
}

// Runs a whole batch: one plan upload, then the device steps.
// tables: device buffer of P.total_cells cells.
// The plan image, and the tables when `tables` is NULL (consumed by the
// reducers), live in a device workspace of the handle: released in stream
// order after the last launch that reads them.
static int run_batch(fc_db *db, Plan &P, int32_t *tables, uint32_t reducers, double ess,
                     float *scores, float *err, hipStream_t s) {
    ensure_attrs();
    Image I;
    make_image(db, P, reducers, I);
    const size_t img = (I.dev_bytes + 255) & ~(size_t)255;
    const size_t tbytes = tables ? 0 : sizeof(int32_t) * (size_t)std::max<int64_t>(P.total_cells, 1);
    Workspace *w = workspace_acquire(db, img + tbytes, s);
    if (!w) {
        set_error("device workspace of %zu bytes could not be allocated", img + tbytes);
        return FC_ERR_NOMEM;
    }
    struct Release {
        fc_db *db;
        Workspace *w;
        hipStream_t s;
        ~Release() { workspace_release(db, w, s); }
    } release{db, w, s};
    void *dimg = w->p;
    if (!tables) tables = (int32_t *)((char *)w->p + img);
    Staging *st = staging_acquire(I.bytes);
    if (!st) {
        set_error("pinned staging allocation of %zu bytes failed", I.bytes);
        return FC_ERR_NOMEM;
    }
    fill_image(P, I, st->host);
    hipError_t e = hipMemcpyAsync(dimg, st->host, I.bytes, hipMemcpyHostToDevice, s);
    staging_release(st, s);
    if (e != hipSuccess) {
        set_error("plan upload failed: %s", hipGetErrorString(e));
        return FC_ERR_DEVICE;
    }
    return enqueue_batch(db, P, I, dimg, tables, reducers, ess, scores, err, s);
}

// Counts and reduces a validated-on-entry batch into device score buffers
// ([slot][nq], slot = set bits of `reducers` in ascending order); the tables
// live in a workspace of the handle.  Used by the native drivers.
int count_reduce_device(fc_db *db, const int32_t *vars_flat, const int64_t *var_off, int64_t nq,
                        uint32_t reducers, double ess, float *scores, hipStream_t s) {
    Plan P;
    int rc = build_plan(db, vars_flat, var_off, nq, nullptr, FC_STRAT_AUTO, true, P);
    if (rc || nq == 0) return rc;
    return run_batch(db, P, nullptr, reducers, ess, scores, nullptr, s);
}

}  // namespace fc

using namespace fc;

extern "C" int64_t fc_table_cells(const fc_db *db, const int32_t *vars, int32_t k) {
    clear_error();
    if (!vars) {
        set_error("fc_table_cells: vars is NULL");
        return FC_ERR_INVALID;
    }
    std::vector<int64_t> cells;
    int64_t off[2] = {0, k};
    int rc = validate(db, vars, off, 1, nullptr, cells);
    return rc ? rc : cells[0];
}

extern "C" int fc_count_batch(fc_db *db, const int32_t *vars_flat, const int64_t *var_off,
                              int64_t nq, int32_t *tables, const int64_t *table_off,
                              uint32_t flags, void *stream) {
    clear_error();
    int rc = FC_OK;
    if (nq > 0 && !tables) {
        set_error("fc_count_batch: tables is NULL");
        return FC_ERR_INVALID;
    }
    Plan P;
    if ((rc = build_plan(db, vars_flat, var_off, nq, table_off, flags, false, P))) return rc;
    if (nq == 0) return FC_OK;
    hipStream_t s = (hipStream_t)stream;
    FC_HIP(hipSetDevice(db->device));
    if (is_device_ptr(tables)) return run_batch(db, P, tables, 0, 0.0, nullptr, nullptr, s);
    DevBuf dt;
    FC_HIP(dt.alloc(sizeof(int32_t) * (size_t)P.total_cells, s));
    if (!P.packed) {  // keep the caller's cells outside the tables intact
        FC_HIP(hipMemcpyAsync(dt.p, tables, sizeof(int32_t) * (size_t)P.total_cells,
                              hipMemcpyHostToDevice, s));
    }
    if ((rc = run_batch(db, P, (int32_t *)dt.p, 0, 0.0, nullptr, nullptr, s))) return rc;
    FC_HIP(hipMemcpyAsync(tables, dt.p, sizeof(int32_t) * (size_t)P.total_cells,
                          hipMemcpyDeviceToHost, s));
    FC_HIP(hipStreamSynchronize(s));
    return FC_OK;
}

extern "C" int fc_count(fc_db *db, const int32_t *vars, int32_t k, int32_t *table, int64_t cells,
                        void *stream) {
    clear_error();
    if (!vars || !table) {
        set_error("fc_count: vars and table must not be NULL");
        return FC_ERR_INVALID;
    }
    int64_t off[2] = {0, k};
    std::vector<int64_t> c;
    int rc = validate(db, vars, off, 1, nullptr, c);
    if (rc) return rc;
    if (c[0] != cells) {
        set_error("fc_count: cells=%lld but the query's table has %lld cells", (long long)cells,
                  (long long)c[0]);
        return FC_ERR_INVALID;
    }
    return fc_count_batch(db, vars, off, 1, table, nullptr, FC_STRAT_AUTO, stream);
}

extern "C" int fc_count_reduce(fc_db *db, const int32_t *vars_flat, const int64_t *var_off,
                               int64_t nq, uint32_t reducers, const fc_reduce_params *p,
                               float *scores, float *err, int32_t *tables,
                               const int64_t *table_off, uint32_t flags, void *stream) {
    clear_error();
    int rc = FC_OK;
    if (reducers == 0 || (reducers & ~(uint32_t)(FC_RED_LL | FC_RED_MDL | FC_RED_BDEU | FC_RED_MI))) {
        set_error("fc_count_reduce: reducer mask %#x is empty or unknown", reducers);
        return FC_ERR_INVALID;
    }
    const double ess = p ? p->ess : 1.0;
    if (!(ess > 0.0)) {
        set_error("fc_count_reduce: ess must be > 0");
        return FC_ERR_INVALID;
    }
    if (nq > 0 && !scores) {
        set_error("fc_count_reduce: scores is NULL");
        return FC_ERR_INVALID;
    }
    if (!tables && table_off) {
        set_error("fc_count_reduce: table_off given without tables");
        return FC_ERR_INVALID;
    }
    Plan P;
    if ((rc = build_plan(db, vars_flat, var_off, nq, table_off, flags, true, P))) return rc;
    if (nq == 0) return FC_OK;
    hipStream_t s = (hipStream_t)stream;
    FC_HIP(hipSetDevice(db->device));
    const int nred = __builtin_popcount(reducers);
    const size_t sbytes = sizeof(float) * (size_t)nred * (size_t)nq;
    const bool tdev = tables && is_device_ptr(tables);
    const bool sdev = is_device_ptr(scores);
    const bool edev = err && is_device_ptr(err);
    DevBuf dt, ds, de;
    int32_t *t = tables;  // NULL: the tables live in run_batch's workspace
    if (tables && !tdev) {
        FC_HIP(dt.alloc(sizeof(int32_t) * (size_t)P.total_cells, s));
        t = (int32_t *)dt.p;
        if (!P.packed)
            FC_HIP(hipMemcpyAsync(t, tables, sizeof(int32_t) * (size_t)P.total_cells,
                                  hipMemcpyHostToDevice, s));
    }
    float *sc = scores, *er = err;
    if (!sdev) {
        FC_HIP(ds.alloc(sbytes, s));
        sc = (float *)ds.p;
    }
    if (err && !edev) {
        FC_HIP(de.alloc(sbytes, s));
        er = (float *)de.p;
    }
    if ((rc = run_batch(db, P, t, reducers, ess, sc, er, s))) return rc;
    bool sync = false;
    if (tables && !tdev) {
        FC_HIP(hipMemcpyAsync(tables, t, sizeof(int32_t) * (size_t)P.total_cells,
                              hipMemcpyDeviceToHost, s));
        sync = true;
    }
    if (!sdev) {
        FC_HIP(hipMemcpyAsync(scores, sc, sbytes, hipMemcpyDeviceToHost, s));
        sync = true;
    }
    if (err && !edev) {
        FC_HIP(hipMemcpyAsync(err, er, sbytes, hipMemcpyDeviceToHost, s));
        sync = true;
    }
    if (sync) FC_HIP(hipStreamSynchronize(s));
    return FC_OK;
}

// ------------------------------------------------- no-allocation variant
// One statically sized device array per GPU holds the plan image and the
// consumed tables of fc_count_reduce_noalloc.  The array's name is a host
// stand-in in host code; its device address comes from hipGetSymbolAddress,
// taken once per device with that device current, and only that address is
// passed to copies and kernels.
namespace fc {
static __device__ __align__(256) unsigned char scratch[FC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of this device's scratch array (the device must be
// current), or NULL with the error set.
static void *scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("fc_count_reduce_noalloc: device %d out of range", device);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error("fc_count_reduce_noalloc: scratch address of device %d: %s", device,
                      hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[device] = ptr;
    }
    return g_scratch_ptr[device];
}
}  // namespace fc

extern "C" int fc_count_reduce_noalloc(fc_db *db, const int32_t *vars_flat,
                                       const int64_t *var_off, int64_t nq, uint32_t reducers,
                                       const fc_reduce_params *p, float *scores, float *err,
                                       uint32_t flags, void *stream) {
    clear_error();
    if (reducers == 0 || (reducers & ~(uint32_t)(FC_RED_LL | FC_RED_MDL | FC_RED_BDEU | FC_RED_MI))) {
        set_error("fc_count_reduce_noalloc: reducer mask %#x is empty or unknown", reducers);
        return FC_ERR_INVALID;
    }
    const double ess = p ? p->ess : 1.0;
    if (!(ess > 0.0)) {
        set_error("fc_count_reduce_noalloc: ess must be > 0");
        return FC_ERR_INVALID;
    }
    Plan P;
    int rc = build_plan(db, vars_flat, var_off, nq, nullptr, flags, true, P);
    if (rc) return rc;
    if (nq == 0) return FC_OK;
    if (!scores || !is_device_ptr(scores) || (err && !is_device_ptr(err))) {
        set_error("fc_count_reduce_noalloc: scores (and err, when given) must be device memory");
        return FC_ERR_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    FC_HIP(hipSetDevice(db->device));
    ensure_attrs();
    Image I;
    make_image(db, P, reducers, I);
    const size_t img = (I.dev_bytes + 255) & ~(size_t)255;
    const size_t need = img + sizeof(int32_t) * (size_t)std::max<int64_t>(P.total_cells, 1);
    if (need > (size_t)FC_NOALLOC_SCRATCH_BYTES) {
        set_error("fc_count_reduce_noalloc: the batch needs %zu bytes of scratch (plan %zu + "
                  "tables of %lld cells), more than the %lld the library holds; split the batch",
                  need, img, (long long)P.total_cells, (long long)FC_NOALLOC_SCRATCH_BYTES);
        return FC_ERR_RANGE;
    }
    char *base = (char *)scratch_address(db->device);
    if (!base) return FC_ERR_DEVICE;
    // the plan image goes through pageable host memory: the copy has read it
    // when hipMemcpyAsync returns, so the buffer is reused by the next call
    static thread_local std::vector<char> host;
    if (host.size() < I.bytes) host.resize(I.bytes);
    fill_image(P, I, host.data());
    hipError_t e = hipMemcpyAsync(base, host.data(), I.bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        set_error("fc_count_reduce_noalloc: plan upload failed: %s", hipGetErrorString(e));
        return FC_ERR_DEVICE;
    }
    return enqueue_batch(db, P, I, base, (int32_t *)(base + img), reducers, ess, scores, err, s);
}

extern "C" int fc_count_assignment(fc_db *db, const int32_t *vars, const uint8_t *states,
                                   int32_t k, int64_t *count, void *stream) {
    clear_error();
    if (!vars || !states || !count) {
        set_error("fc_count_assignment: vars, states and count must not be NULL");
        return FC_ERR_INVALID;
    }
    int64_t off[2] = {0, k};
    std::vector<int64_t> c;
    int rc = validate(db, vars, off, 1, nullptr, c);
    if (rc) return rc;
    for (int32_t t = 0; t < k; ++t)
        if (states[t] >= db->arity[vars[t]]) {
            set_error("fc_count_assignment: state %u of variable %d is not below its arity %u",
                      states[t], vars[t], db->arity[vars[t]]);
            return FC_ERR_INVALID;
        }
    hipStream_t s = (hipStream_t)stream;
    FC_HIP(hipSetDevice(db->device));
    DevBuf d;
    FC_HIP(d.alloc(sizeof(unsigned long long), s));
    FC_HIP(fill_zero_i32((int32_t *)d.p, 2, s));
    if (db->m > 0) {
        if (db->d_bits) {
            Rows8 rows;
            for (int32_t t = 0; t < FC_MAX_VARS; ++t)
                rows.r[t] = t < k ? db->state_off[vars[t]] + states[t] : 0;
            int64_t blocks = std::min<int64_t>((db->words + 255) / 256, 4 * db->cu_count);
            hipLaunchKernelGGL(k_assign_bits, dim3((unsigned)blocks), dim3(256), 0, s, db->d_bits,
                               db->words, db->pitch / 64, rows, k, (unsigned long long *)d.p);
        } else {
            Assign8 a;
            for (int32_t t = 0; t < FC_MAX_VARS; ++t) {
                a.var[t] = t < k ? vars[t] : 0;
                a.state[t] = t < k ? states[t] : 0;
            }
            int64_t blocks = std::min<int64_t>((db->m + 255) / 256, 4 * db->cu_count);
            hipLaunchKernelGGL(k_assign_cols, dim3((unsigned)blocks), dim3(256), 0, s, db->d_cols,
                               db->m, db->pitch, a, k, (unsigned long long *)d.p);
        }
        FC_HIP(hipGetLastError());
    }
    unsigned long long h = 0;
    FC_HIP(hipMemcpyAsync(&h, d.p, sizeof h, hipMemcpyDeviceToHost, s));
    FC_HIP(hipStreamSynchronize(s));
    *count = (int64_t)h;
    return FC_OK;
}

extern "C" int fc_batch_footprint(const fc_db *db, const int32_t *vars_flat,
                                  const int64_t *var_off, int64_t nq, uint32_t flags,
                                  int64_t *bytes) {
    clear_error();
    if (!bytes) {
        set_error("fc_batch_footprint: bytes is NULL");
        return FC_ERR_INVALID;
    }
    int rc = FC_OK;
    Plan P;
    if ((rc = build_plan(db, vars_flat, var_off, nq, nullptr, flags, true, P))) return rc;
    *bytes = (int64_t)sizeof(int32_t) * P.total_cells +
             (int64_t)sizeof(QDesc) * (int64_t)(P.work.size() + P.query.size()) +
             (int64_t)sizeof(int32_t) * ((int64_t)P.gram_np * P.gram_np + P.gram_np +
                                         (int64_t)P.gram_pos.size()) +
             (int64_t)sizeof(float) * 2 * 4 * nq;
    return FC_OK;
}

// ------------------------------------------------------------------ tuning
extern "C" int fc_plan_summary(const fc_db *db, const int32_t *vars_flat, const int64_t *var_off,
                               int64_t nq, uint32_t flags, int64_t *out) {
    clear_error();
    if (!out) {
        set_error("fc_plan_summary: out is NULL");
        return FC_ERR_INVALID;
    }
    Plan P;
    const int rc = build_plan(db, vars_flat, var_off, nq, nullptr, flags, false, P);
    if (rc) return rc;
    std::vector<uint8_t> seen((size_t)nq, 0);
    int64_t hist = 0, bitmap = 0;
    for (const Launch &L : P.launches)
        for (int64_t d = L.first; d < L.first + L.count; ++d) {
            const int32_t q = P.work[(size_t)d].qid;
            if (seen[(size_t)q]) continue;  // key windows of one query
            seen[(size_t)q] = 1;
            if (L.strat == S_BITMAP) ++bitmap; else ++hist;
        }
    out[0] = hist + P.part_count;
    out[1] = bitmap;
    out[2] = P.gram_count;
    out[3] = (int64_t)P.marg.size();
    return FC_OK;
}

extern "C" int fc_db_get_tuning(const fc_db *db, fc_tuning *t) {
    clear_error();
    if (!db || !t) {
        set_error("fc_db_get_tuning: NULL argument");
        return FC_ERR_INVALID;
    }
    t->chunk_rows = db->tune.chunk_rows;
    t->bitmap_chunk_rows = db->tune.bitmap_chunk_rows;
    t->bitmap_words = db->tune.bitmap_words;
    t->persistent_max_queries = db->tune.persistent_max_queries;
    std::memcpy(t->bitmap_cells, db->tune.bitmap_cells, sizeof t->bitmap_cells);
    t->packed_columns = db->tune.packed_columns;
    t->bitmap_order = db->tune.bitmap_order;
    t->derive_tables = db->tune.derive;
    t->one_pass_partition = db->tune.one_pass;
    t->row_sweep = db->tune.row_sweep;
    return FC_OK;
}

extern "C" int fc_db_set_tuning(fc_db *db, const fc_tuning *t) {
    clear_error();
    if (!db || !t) {
        set_error("fc_db_set_tuning: NULL argument");
        return FC_ERR_INVALID;
    }
    if (t->chunk_rows < kTileRows || t->bitmap_chunk_rows < kTileRows ||
        (t->bitmap_words != 1 && t->bitmap_words != 2 && t->bitmap_words != 4) ||
        (t->packed_columns != 0 && t->packed_columns != 1) ||
        (t->bitmap_order != 0 && t->bitmap_order != 1) ||
        (t->derive_tables != 0 && t->derive_tables != 1) ||
        (t->one_pass_partition != 0 && t->one_pass_partition != 1) ||
        (t->row_sweep != 0 && t->row_sweep != 1)) {
        set_error("fc_db_set_tuning: chunk rows must be >= %lld, bitmap_words 1, 2 or 4, "
                  "packed_columns, bitmap_order, derive_tables, one_pass_partition and "
                  "row_sweep 0 or 1",
                  (long long)kTileRows);
        return FC_ERR_INVALID;
    }
    db->tune.chunk_rows = t->chunk_rows;
    db->tune.bitmap_chunk_rows = t->bitmap_chunk_rows;
    db->tune.bitmap_words = t->bitmap_words;
    db->tune.persistent_max_queries = t->persistent_max_queries < 0 ? 0 : t->persistent_max_queries;
    std::memcpy(db->tune.bitmap_cells, t->bitmap_cells, sizeof t->bitmap_cells);
    db->tune.packed_columns = t->packed_columns;
    db->tune.bitmap_order = t->bitmap_order;
    db->tune.derive = t->derive_tables;
    db->tune.one_pass = t->one_pass_partition;
    db->tune.row_sweep = t->row_sweep;
    return FC_OK;
}

namespace fc {

// Time per batch under the current tuning: one warm-up call, then `reps`
// calls back to back between two events, so the host's planning of a call
// overlaps the device work of the one before it.
// With device = true, the time is instead the summed event-timed duration
// of the batch's kernel launches: the measure for choices that only change
// device work (column store, chunk sizes, row order, per-shape strategy),
// which on a batch bound by host planning the wall time would hide.
static int time_batch(fc_db *db, const std::vector<int32_t> &flat,
                      const std::vector<int64_t> &off, uint32_t flags, int32_t *tables,
                      hipStream_t s, int reps, float &ms_out, bool device = false) {
    const int64_t nq = (int64_t)off.size() - 1;
    int rc = fc_count_batch(db, flat.data(), off.data(), nq, tables, nullptr, flags, s);
    if (rc) return rc;
    FC_HIP(hipStreamSynchronize(s));
    if (device) {
        double dev = 0.0;
        device_time_begin(&dev);
        for (int r = 0; r < reps && rc == FC_OK; ++r)
            rc = fc_count_batch(db, flat.data(), off.data(), nq, tables, nullptr, flags, s);
        device_time_end();
        if (rc) return rc;
        ms_out = (float)(dev / reps);
        return FC_OK;
    }
    hipEvent_t a, b;
    FC_HIP(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        set_error("hipEventCreate failed");
        return FC_ERR_DEVICE;
    }
    (void)hipEventRecord(a, s);
    for (int r = 0; r < reps && rc == FC_OK; ++r)
        rc = fc_count_batch(db, flat.data(), off.data(), nq, tables, nullptr, flags, s);
    (void)hipEventRecord(b, s);
    float ms = 0.f;
    const hipError_t e = rc == FC_OK ? hipEventSynchronize(b) : hipSuccess;
    if (rc == FC_OK && e == hipSuccess) (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    if (e != hipSuccess) {
        set_error("hipEventSynchronize: %s", hipGetErrorString(e));
        return FC_ERR_DEVICE;
    }
    ms_out = ms / (float)reps;
    return FC_OK;
}

// The queries of a batch whose automatic plan counts them with bitmaps
// (bitmap = true) or with histograms and partitions (false), in batch order.
static int plan_subset(fc_db *db, const int32_t *vars_flat, const int64_t *var_off, int64_t nq,
                       bool bitmap, std::vector<int32_t> &f, std::vector<int64_t> &o) {
    Plan P;
    const int rc = build_plan(db, vars_flat, var_off, nq, nullptr, FC_STRAT_AUTO, false, P);
    if (rc) return rc;
    std::vector<uint8_t> sel((size_t)nq, 0);
    for (const Launch &L : P.launches)
        if ((L.strat == S_BITMAP) == bitmap)
            for (int64_t d = L.first; d < L.first + L.count; ++d)
                sel[(size_t)P.work[(size_t)d].qid] = 1;
    f.clear();
    o.assign(1, 0);
    for (int64_t i = 0; i < nq; ++i)
        if (sel[(size_t)i]) {
            f.insert(f.end(), vars_flat + var_off[i], vars_flat + var_off[i + 1]);
            o.push_back((int64_t)f.size());
        }
    return FC_OK;
}

}  // namespace fc

extern "C" int fc_autotune(fc_db *db, const int32_t *vars_flat, const int64_t *var_off,
                           int64_t nq, void *stream) {
    clear_error();
    std::vector<int64_t> cells;
    int rc = validate(db, vars_flat, var_off, nq, nullptr, cells);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    FC_HIP(hipSetDevice(db->device));
    int64_t total = 1024 * 128;  // room for a replicated bucket (<= 128 cells each)
    {
        int64_t sum = 0;
        for (int64_t c : cells) sum += c;
        total = std::max(total, sum);
    }
    DevBuf dt;
    FC_HIP(dt.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(total, 1), s));
    int32_t *tables = (int32_t *)dt.p;
    std::vector<int32_t> flat(vars_flat, vars_flat + var_off[nq]);
    std::vector<int64_t> off(var_off, var_off + nq + 1);
    const int64_t cand[] = {16384, 32768, 65536, 131072, 262144, 524288};
    auto sweep_chunks = [&](int which) -> int {
        // timed on the queries the setting affects (those the automatic plan
        // counts with histograms, or with bitmaps); the current value is kept
        // unless another is at least 3% faster
        std::vector<int32_t> sf;
        std::vector<int64_t> so;
        int r = plan_subset(db, vars_flat, var_off, nq, which == 1, sf, so);
        if (r) return r;
        if (so.size() < 2) return FC_OK;
        const int64_t cur = which == 0 ? db->tune.chunk_rows : db->tune.bitmap_chunk_rows;
        int64_t best = cur;
        float best_ms = 1e30f, cur_ms = 1e30f;
        for (int64_t c : cand) {
            if (which == 0) db->tune.chunk_rows = c; else db->tune.bitmap_chunk_rows = c;
            float ms = 0.f;
            r = time_batch(db, sf, so, FC_STRAT_AUTO, tables, s, 5, ms, true);
            if (r) return r;
            if (c == cur) cur_ms = ms;
            if (ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
        if (!(best_ms < 0.97f * cur_ms)) best = cur;
        if (which == 0) db->tune.chunk_rows = best; else db->tune.bitmap_chunk_rows = best;
        return FC_OK;
    };
    // 0. Batch size up to which one persistent launch beats one launch per
    //    group: prefixes of the sample of growing size, stop at the first loss.
    auto tune_persistent = [&]() -> int {
        int32_t thr = 0;
        for (int64_t nsub : {16, 64, 256, 1024, 4096}) {
            if (nsub > nq) break;
            std::vector<int32_t> f(vars_flat, vars_flat + var_off[nsub]);
            std::vector<int64_t> o(var_off, var_off + nsub + 1);
            float ms_p = 0.f, ms_s = 0.f;
            db->tune.persistent_max_queries = (int32_t)nsub;
            if ((rc = time_batch(db, f, o, FC_STRAT_AUTO, tables, s, 5, ms_p)))
                return rc;
            db->tune.persistent_max_queries = 0;
            if ((rc = time_batch(db, f, o, FC_STRAT_AUTO, tables, s, 5, ms_s)))
                return rc;
            if (ms_p < ms_s) thr = (int32_t)nsub; else break;
        }
        db->tune.persistent_max_queries = thr;
        return FC_OK;
    };
    if ((rc = tune_persistent())) return rc;
    // 1. Packed 4-bit columns against byte columns for the histograms (when
    //    the database has them), then the histogram chunk size.
    if (db->d_nib) {
        const int cur = db->tune.packed_columns;
        float ms_cur = 0.f, ms_alt = 0.f;
        if ((rc = time_batch(db, flat, off, FC_STRAT_AUTO, tables, s, 5, ms_cur, true))) return rc;
        db->tune.packed_columns = 1 - cur;
        if ((rc = time_batch(db, flat, off, FC_STRAT_AUTO, tables, s, 5, ms_alt, true))) return rc;
        db->tune.packed_columns = ms_alt < 0.97f * ms_cur ? 1 - cur : cur;
    }
    if ((rc = sweep_chunks(0))) return rc;
    // 2. Bitmap against histogram per (k, size bucket), on the sample's own
    //    queries of that shape, repeated to at least 1024 queries so the
    //    timing is not dominated by launch latency.
    if (db->d_bits) {
        for (int k = 1; k <= FC_MAX_VARS; ++k)
            for (int bkt = 0; bkt < 6; ++bkt) {
                const int64_t lo = bkt == 0 ? 0 : (int64_t(4) << (bkt - 1)), hi = int64_t(4) << bkt;
                std::vector<int32_t> f;
                std::vector<int64_t> o(1, 0);
                for (int64_t i = 0; i < nq; ++i)
                    if (var_off[i + 1] - var_off[i] == k && cells[(size_t)i] > lo &&
                        cells[(size_t)i] <= hi) {
                        f.insert(f.end(), vars_flat + var_off[i], vars_flat + var_off[i + 1]);
                        o.push_back((int64_t)f.size());
                    }
                if (o.size() < 2) continue;
                const size_t nb = o.size() - 1, fl = f.size();
                while (o.size() - 1 < 1024)
                    for (size_t i = 0; i < nb && o.size() - 1 < 1024; ++i) {
                        f.insert(f.end(), f.begin() + o[i], f.begin() + o[i + 1]);
                        o.push_back((int64_t)f.size());
                    }
                (void)fl;
                int64_t need = 0;
                for (size_t i = 0; i + 1 < o.size(); ++i) {
                    int64_t c = 1;
                    for (int64_t t = o[i]; t < o[i + 1]; ++t) c *= db->arity[f[(size_t)t]];
                    need += c;
                }
                if (need > total) continue;  // the scratch table is sized for the sample
                float tb = 0.f, th = 0.f;
                if ((rc = time_batch(db, f, o, FC_STRAT_BITMAP, tables, s, 5, tb, true)))
                    return rc;
                if ((rc = time_batch(db, f, o, FC_STRAT_HIST, tables, s, 5, th, true)))
                    return rc;
                // switch away from the current choice only on a clear win
                const bool cur_bitmap = db->tune.bitmap_cells[k - 1][bkt] != 0;
                if (cur_bitmap && th < 0.97f * tb) db->tune.bitmap_cells[k - 1][bkt] = 0;
                if (!cur_bitmap && tb < 0.97f * th) db->tune.bitmap_cells[k - 1][bkt] = 1;
            }
    }
    // 3. Chunk sizes again, for the strategy mix just chosen.
    if ((rc = sweep_chunks(0))) return rc;
    if (db->d_bits && (rc = sweep_chunks(1))) return rc;
    // 4. Words per bitmap tree walk.
    if (db->d_bits) {
        const int curw = db->tune.bitmap_words;
        int bestw = curw;
        float best_ms = 1e30f, cur_ms = 1e30f;
        for (int wv : {1, 2, 4}) {
            db->tune.bitmap_words = wv;
            float ms = 0.f;
            if ((rc = time_batch(db, flat, off, FC_STRAT_AUTO, tables, s, 5, ms, true)))
                return rc;
            if (wv == curw) cur_ms = ms;
            if (ms < best_ms) {
                best_ms = ms;
                bestw = wv;
            }
        }
        db->tune.bitmap_words = best_ms < 0.97f * cur_ms ? bestw : curw;
    }
    // 5. The per-shape bitmap choices against none at all, on the whole
    //    batch: on a small, launch-bound batch the extra launch groups of the
    //    mixed strategies can cost more than the bitmap walks save.  After a
    //    switch the persistent threshold and chunk size are tuned again.
    if (db->d_bits) {
        uint8_t saved[FC_MAX_VARS][6];
        std::memcpy(saved, db->tune.bitmap_cells, sizeof saved);
        float ms_mix = 0.f, ms_hist = 0.f;
        if ((rc = time_batch(db, flat, off, FC_STRAT_AUTO, tables, s, 5, ms_mix))) return rc;
        std::memset(db->tune.bitmap_cells, 0, sizeof saved);
        if ((rc = time_batch(db, flat, off, FC_STRAT_AUTO, tables, s, 5, ms_hist))) return rc;
        if (!(ms_hist < 0.97f * ms_mix)) {
            std::memcpy(db->tune.bitmap_cells, saved, sizeof saved);
        } else {
            if ((rc = tune_persistent())) return rc;
            if ((rc = sweep_chunks(0))) return rc;
        }
    }
    // 6. Synchronized row sweeps against every workgroup starting at its
    //    chunk's first row.
    {
        const int cur = db->tune.row_sweep;
        float ms_cur = 0.f, ms_alt = 0.f;
        if ((rc = time_batch(db, flat, off, FC_STRAT_AUTO, tables, s, 5, ms_cur, true))) return rc;
        db->tune.row_sweep = 1 - cur;
        if ((rc = time_batch(db, flat, off, FC_STRAT_AUTO, tables, s, 5, ms_alt, true))) return rc;
        db->tune.row_sweep = ms_alt < 0.97f * ms_cur ? 1 - cur : cur;
    }
    return FC_OK;
}

// ------------------------------------------------------------------ graphs
struct fc_graph {
    fc_db *db = nullptr;
    uint64_t epoch = 0;  // database epoch at capture
    fc::Plan P;
    fc::Image I;
    void *dimg = nullptr;
    int32_t *scratch = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" void fc_graph_destroy(fc_graph *g) {
    if (!g) return;
    if (g->cap) (void)hipStreamSynchronize(g->cap);
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    if (g->dimg) (void)hipFree(g->dimg);
    if (g->scratch) (void)hipFree(g->scratch);
    (void)hipGetLastError();
    delete g;
}

extern "C" int fc_graph_create(fc_db *db, const int32_t *vars_flat, const int64_t *var_off,
                               int64_t nq, uint32_t reducers, const fc_reduce_params *p,
                               float *scores, float *err, int32_t *tables,
                               const int64_t *table_off, uint32_t flags, void *stream,
                               fc_graph **out) {
    clear_error();
    if (!out) {
        set_error("fc_graph_create: out is NULL");
        return FC_ERR_INVALID;
    }
    *out = nullptr;
    int rc = FC_OK;
    if (nq < 1) {
        set_error("fc_graph_create: empty batch");
        return FC_ERR_INVALID;
    }
    if (reducers & ~(uint32_t)(FC_RED_LL | FC_RED_MDL | FC_RED_BDEU | FC_RED_MI)) {
        set_error("fc_graph_create: unknown reducer mask %#x", reducers);
        return FC_ERR_INVALID;
    }
    if (!reducers && !tables) {
        set_error("fc_graph_create: counts only (no reducer) needs tables");
        return FC_ERR_INVALID;
    }
    if ((tables && !is_device_ptr(tables)) || (reducers && !is_device_ptr(scores)) ||
        (err && !is_device_ptr(err))) {
        set_error("fc_graph_create: every output must be device memory");
        return FC_ERR_INVALID;
    }
    if (!tables && table_off) {
        set_error("fc_graph_create: table_off given without tables");
        return FC_ERR_INVALID;
    }
    const double ess = p ? p->ess : 1.0;
    if (!(ess > 0.0)) {
        set_error("fc_graph_create: ess must be > 0");
        return FC_ERR_INVALID;
    }
    FC_HIP(hipSetDevice(db->device));
    ensure_attrs();
    fc_graph *g = new (std::nothrow) fc_graph();
    if (!g) {
        set_error("fc_graph_create: host allocation failed");
        return FC_ERR_NOMEM;
    }
    g->db = db;
    g->epoch = db->epoch;
    struct Guard {
        fc_graph *g;
        ~Guard() { if (g) fc_graph_destroy(g); }
    } guard{g};
    if ((rc = build_plan(db, vars_flat, var_off, nq, table_off, flags, reducers != 0, g->P))) return rc;
    make_image(db, g->P, reducers, g->I);
    FC_HIP(hipMalloc(&g->dimg, g->I.dev_bytes));
    std::vector<char> host(g->I.bytes);
    fill_image(g->P, g->I, host.data());
    FC_HIP(hipMemcpy(g->dimg, host.data(), g->I.bytes, hipMemcpyHostToDevice));
    int32_t *t = tables;
    if (!t) {
        FC_HIP(hipMalloc(&g->scratch, sizeof(int32_t) * (size_t)std::max<int64_t>(g->P.total_cells, 1)));
        t = g->scratch;
    }
    FC_HIP(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
    FC_HIP(hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
    set_capturing(true);
    rc = enqueue_batch(db, g->P, g->I, g->dimg, t, reducers, ess, scores, err, g->cap);
    set_capturing(false);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(g->cap, &graph);
    g->graph = graph;
    if (rc) return rc;
    FC_HIP(e);
    FC_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    (void)stream;
    *out = g;
    guard.g = nullptr;
    return FC_OK;
}

extern "C" int fc_graph_launch(fc_graph *g, void *stream) {
    clear_error();
    if (!g || !g->exec) {
        set_error("fc_graph_launch: NULL graph");
        return FC_ERR_INVALID;
    }
    if (g->epoch != g->db->epoch) {
        set_error("fc_graph_launch: the database changed since the batch was captured");
        return FC_ERR_INVALID;
    }
    FC_HIP(hipSetDevice(g->db->device));
    ProfScope ps("graph", (hipStream_t)stream, 0.0, 0.0);
    FC_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    ps.end((hipStream_t)stream);
    return FC_OK;
}

extern "C" int fc_count_assignments(fc_db *db, const int32_t *vars_flat, const int64_t *var_off,
                                    const uint8_t *states_flat, int64_t nq, int64_t *counts,
                                    void *stream) {
    clear_error();
    std::vector<int64_t> cells;
    int rc = validate(db, vars_flat, var_off, nq, nullptr, cells);
    if (rc) return rc;
    if (nq > 0 && (!states_flat || !counts)) {
        set_error("fc_count_assignments: states_flat and counts must not be NULL");
        return FC_ERR_INVALID;
    }
    for (int64_t i = 0; i < nq; ++i)
        for (int64_t t = var_off[i]; t < var_off[i + 1]; ++t)
            if (states_flat[t] >= db->arity[vars_flat[t]]) {
                set_error("fc_count_assignments: query %lld: state %u of variable %d is not below "
                          "its arity %u", (long long)i, states_flat[t], vars_flat[t],
                          db->arity[vars_flat[t]]);
                return FC_ERR_INVALID;
            }
    if (nq == 0) return FC_OK;
    hipStream_t s = (hipStream_t)stream;
    FC_HIP(hipSetDevice(db->device));
    const bool cdev = is_device_ptr(counts);
    // one workspace of the handle: host-bound counts, then the descriptors
    const size_t nv = (size_t)var_off[nq];
    const size_t obytes = cdev ? 0 : ((sizeof(int64_t) * (size_t)nq + 255) & ~(size_t)255);
    const size_t qbytes = db->d_bits ? sizeof(ADesc) * (size_t)nq
                                     : sizeof(int32_t) * nv + sizeof(int64_t) * ((size_t)nq + 1) + nv;
    Workspace *w = workspace_acquire(db, obytes + qbytes, s);
    if (!w) {
        set_error("fc_count_assignments: device workspace could not be allocated");
        return FC_ERR_NOMEM;
    }
    struct Release {
        fc_db *db;
        Workspace *w;
        hipStream_t s;
        ~Release() { workspace_release(db, w, s); }
    } release{db, w, s};
    void *dq = (char *)w->p + obytes;
    unsigned long long *out = (unsigned long long *)counts;
    if (!cdev) out = (unsigned long long *)w->p;
    FC_HIP(fill_zero_i32((int32_t *)out, 2 * nq, s));
    // enough workgroups, chunks a multiple of 8 (XCD order), >= 64K instances each
    const int64_t tiles = db->m_pad / kTileRows;
    int64_t ch = std::max<int64_t>(1, db->m_pad / 65536);
    ch = std::min(ch, tiles);
    if (ch >= kXcds) ch -= ch % kXcds;
    if (db->m > 0) {
        const double alg = (double)var_off[nq] * (double)db->m / 8.0;  // k bits per instance
        ProfScope ps("k_assign_batch", s, alg, 0.0);
        if (db->d_bits) {
            std::vector<ADesc> h((size_t)nq);
            for (int64_t i = 0; i < nq; ++i) {
                ADesc &d = h[(size_t)i];
                std::memset(&d, 0, sizeof d);
                d.k = (int32_t)(var_off[i + 1] - var_off[i]);
                for (int32_t t = 0; t < d.k; ++t) {
                    const int32_t v = vars_flat[var_off[i] + t];
                    d.row[t] = db->state_off[v] + states_flat[var_off[i] + t];
                }
            }
            Staging *st = staging_acquire(sizeof(ADesc) * (size_t)nq);
            if (!st) {
                set_error("pinned staging allocation failed");
                return FC_ERR_NOMEM;
            }
            std::memcpy(st->host, h.data(), sizeof(ADesc) * (size_t)nq);
            hipError_t e = hipMemcpyAsync(dq, st->host, sizeof(ADesc) * (size_t)nq,
                                          hipMemcpyHostToDevice, s);
            staging_release(st, s);
            FC_HIP(e);
            hipLaunchKernelGGL(k_assign_batch, dim3((unsigned)(nq * ch)), dim3(kBlock), 0, s,
                               db->d_bits, db->words, db->pitch / 64, (const ADesc *)dq, (int32_t)nq,
                               (int32_t)ch, out);
        } else {
            const size_t bytes = qbytes;
            Staging *st = staging_acquire(bytes);
            if (!st) {
                set_error("pinned staging allocation failed");
                return FC_ERR_NOMEM;
            }
            // var_off first (8-byte aligned), then the variables, then the states
            const size_t ob = sizeof(int64_t) * ((size_t)nq + 1), vb = sizeof(int32_t) * nv;
            char *hp = (char *)st->host;
            std::memcpy(hp, var_off, ob);
            std::memcpy(hp + ob, vars_flat, vb);
            std::memcpy(hp + ob + vb, states_flat, nv);
            hipError_t e = hipMemcpyAsync(dq, st->host, bytes, hipMemcpyHostToDevice, s);
            staging_release(st, s);
            FC_HIP(e);
            char *dp = (char *)dq;
            hipLaunchKernelGGL(k_assign_batch_cols, dim3((unsigned)(nq * ch)), dim3(kBlock), 0, s,
                               db->d_cols, db->m, db->pitch, (const int32_t *)(dp + ob),
                               (const int64_t *)dp, (const uint8_t *)(dp + ob + vb), (int32_t)nq,
                               (int32_t)ch, out);
        }
        FC_HIP(hipGetLastError());
        ps.end(s);
    }
    if (!cdev) {
        FC_HIP(hipMemcpyAsync(counts, out, sizeof(int64_t) * (size_t)nq, hipMemcpyDeviceToHost, s));
        FC_HIP(hipStreamSynchronize(s));
    }
    return FC_OK;
}
