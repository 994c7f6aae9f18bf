// All-pairs co-occurrence counts of binary items and association-rule pair
// records (Section 4.3: support and confidence of rules between two items).
//
// The count of every pair Count(X_a = 1 AND X_b = 1) is one entry of the
// Gram matrix A^T A of the m x n one-hot {0,1} instance-by-item matrix, a
// dense contraction over the instances.  It runs on the matrix cores with
// e2m1 (FP4) operands: 0 and 1 are exact e2m1 values, so every product is
// exact, and the fp32 accumulators stay exact while a sum is at most 2^24,
// which holds because one workgroup covers at most 2^24 instances.  The
// item bit-vectors of state 1 are expanded to one nibble per instance in
// registers, never materialised.
//  * a workgroup of 4 waves owns a 128 x 128 block of items (the blocks
//    that reach the upper triangle; the matrix is symmetric) over one range
//    of instances (split K); each wave holds a 128 x 32 part as an 8 x 2 grid
//    of 16x16x128 scaled-MFMA accumulators (e2m1 operands, unit scales),
//    which leaves registers for four resident workgroups per CU;
//    partial blocks are converted to int32 and summed into the output with
//    int32 atomics;
//  * the instances are taken 512 at a time (8 words of every item): a lane
//    of K group g loads words 2g and 2g+1 of each of its items with one
//    16-byte load (the 4 groups of an item read 64 contiguous bytes), and
//    MFMA step h of the 4 feeds it dword h of those two words (32
//    instances).  Every instance is used exactly once, and A and B
//    fragments come from the same function over the same instance groups,
//    so their K order agrees whatever the hardware's order is;
//  * a lane expands its 32 bits of an item to 32 nibbles (16 bytes), the
//    operand layout of the MFMA: bit 4k + t goes to nibble k of dword t.
//    The 128 row items are shared by the 4 waves: each expands 2 of the 8
//    row fragments into an LDS panel two steps ahead (four panels in
//    rotation, one barrier per two steps); the 32 column items of a wave
//    stay in registers, expanded one step ahead;
//  * the words of the next 512 instances load during the current ones.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fc_internal.h"

namespace fc {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kGT = 128;  // row items per block
constexpr int kGK = 2;         // column fragments per wave
constexpr int kGC = 4 * kGK * 16;  // column items per block (kGK * 16 per wave)
constexpr int kGR = kGT / 16;  // row fragments
constexpr int kGS = 8;         // words per load step

// 32 instance bits -> 32 e2m1 values of 0 or 1.0 (0x2): bit 4k + t of b
// becomes nibble k of dword t (a shift and a mask per 8 instances).
__device__ __forceinline__ v4i expand32(uint32_t b) {
    v4i r;
    r[0] = (int)((b << 1) & 0x22222222u);
    r[1] = (int)(b & 0x22222222u);
    r[2] = (int)((b >> 1) & 0x22222222u);
    r[3] = (int)((b >> 2) & 0x22222222u);
    return r;
}

// The 32 bits of MFMA step h: dword h of a lane's two words.
template <int H>
__device__ __forceinline__ uint32_t bits_of(const uint4 &v) {
    return H == 0 ? v.x : H == 1 ? v.y : H == 2 ? v.z : v.w;
}

__device__ __forceinline__ v4f mfma_fp4(const v4i &a, const v4i &b, const v4f &c) {
    const v8i a8 = {a[0], a[1], a[2], a[3], 0, 0, 0, 0};
    const v8i b8 = {b[0], b[1], b[2], b[3], 0, 0, 0, 0};
    // formats 4/4: e2m1 operands; scales 127: 2^0
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a8, b8, c, 4, 4, 0, 127, 0, 127);
}

// A lane's 2 row items (its share of the panel) and 4 column items.
struct Words {
    uint4 a[2], b[kGK];
};

__device__ __forceinline__ Words load_words(const uint64_t *const (&pa)[2],
                                            const uint64_t *const (&pb)[kGK], int64_t w) {
    Words x;
#pragma unroll
    for (int i = 0; i < 2; ++i) x.a[i] = *reinterpret_cast<const uint4 *>(pa[i] + w);
#pragma unroll
    for (int j = 0; j < kGK; ++j) x.b[j] = *reinterpret_cast<const uint4 *>(pb[j] + w);
    return x;
}

// One step: the 8 x kGK MFMAs of the current operands (row fragments from
// `cur_panel`, column fragments `b`) with expansions interleaved between the
// MFMA rows, so a wave's VALU work overlaps its own matrix-core work: this
// wave's row fragments of the step two ahead (words `xr`, dword HR) into
// `far_panel`, its column fragments of the next step (words `xc`, dword HC)
// into `nb`.  Four panels rotate, so a barrier is needed after every
// second step only (SYNC): the panel a step reads was written two steps
// earlier, before the previous barrier, and the one it writes was last
// read two steps earlier, also before it.
template <int HR, int HC, bool SYNC>
__device__ __forceinline__ void gram_step(const Words &xr, const Words &xc, const uint4 (&ma)[2],
                                          const uint4 (&mb)[kGK], v4i (*cur_panel)[64],
                                          v4i (*far_panel)[64], int wave, int lane,
                                          bool active, const v4i (&b)[kGK], v4i (&nb)[kGK],
                                          v4f (&acc)[kGR][kGK]) {
    if (active) {
#pragma unroll
        for (int i = 0; i < kGR; ++i) {
            const v4i a = cur_panel[i][lane];
#pragma unroll
            for (int j = 0; j < kGK; ++j)
                acc[i][j] = mfma_fp4(a, b[j], acc[i][j]);
            if (i < 2)
                far_panel[2 * wave + i][lane] =
                    expand32(bits_of<HR>(xr.a[i]) & bits_of<HR>(ma[i]));
            else if (i < 2 + kGK)
                nb[i - 2] = expand32(bits_of<HC>(xc.b[i - 2]) & bits_of<HC>(mb[i - 2]));
        }
    } else {
#pragma unroll
        for (int i = 0; i < 2; ++i)
            far_panel[2 * wave + i][lane] = expand32(bits_of<HR>(xr.a[i]) & bits_of<HR>(ma[i]));
#pragma unroll
        for (int j = 0; j < kGK; ++j) nb[j] = expand32(bits_of<HC>(xc.b[j]) & bits_of<HC>(mb[j]));
    }
    if (SYNC) __syncthreads();
}

__global__ __launch_bounds__(256, 2) void k_gram(const uint64_t *__restrict__ bits, int64_t words,
                                                 int64_t wpitch,
                                                 const int32_t *__restrict__ rowidx, int32_t nrb,
                                                 int32_t ncb, int32_t npairs, int32_t splits,
                                                 int32_t *__restrict__ C, int32_t ldc) {
    __shared__ v4i panel[4][kGR][64];  // row fragments of four steps, lane-major
    const int32_t p = (int32_t)(blockIdx.x % (uint32_t)npairs);
    const int32_t sp = (int32_t)(blockIdx.x / (uint32_t)npairs);
    // pair index -> (I, J): row block I meets the upper triangle from column
    // block I * kGT / kGC on
    int32_t I = 0, rem = p;
    while (rem >= ncb - I * kGT / kGC) {
        rem -= ncb - I * kGT / kGC;
        ++I;
    }
    const int32_t J = I * kGT / kGC + rem;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, grp = lane >> 4, col = lane & 15;
    const int32_t col0 = J * kGC + wave * kGK * 16;  // this wave's first column item
    // a wave whose columns all lie left of the block's first row adds nothing
    const bool active = col0 + kGK * 16 - 1 >= I * kGT;
    // this lane's words 2g, 2g + 1 of every 8; padding items read row 0, masked
    const uint64_t *pa[2], *pb[kGK];
    uint4 ma[2], mb[kGK];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int32_t r = rowidx[I * kGT + (2 * wave + i) * 16 + col];
        pa[i] = bits + (int64_t)(r < 0 ? 0 : r) * wpitch + 2 * grp;
        const uint32_t m = r < 0 ? 0u : 0xFFFFFFFFu;
        ma[i] = make_uint4(m, m, m, m);
    }
#pragma unroll
    for (int j = 0; j < kGK; ++j) {
        const int32_t r = rowidx[col0 + j * 16 + col];
        pb[j] = bits + (int64_t)(r < 0 ? 0 : r) * wpitch + 2 * grp;
        const uint32_t m = r < 0 ? 0u : 0xFFFFFFFFu;
        mb[j] = make_uint4(m, m, m, m);
    }
    const int64_t tiles = words / (kTileRows / 64);
    const int64_t w0 = (int64_t)sp * tiles / splits * (kTileRows / 64);
    const int64_t w1 = (int64_t)(sp + 1) * tiles / splits * (kTileRows / 64);

    v4f acc[kGR][kGK];
#pragma unroll
    for (int i = 0; i < kGR; ++i)
#pragma unroll
        for (int j = 0; j < kGK; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    if (w0 < w1) {
        // (w1 - w0) is a multiple of 64 words; past the range the loads
        // repeat the last step's words (expanded, never multiplied)
        const int64_t last = w1 - kGS;
        Words cur = load_words(pa, pb, w0);
        v4i b[kGK], nb[kGK];
        // the row fragments of steps 0 and 1, the column fragments of step 0
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            panel[0][2 * wave + i][lane] = expand32(bits_of<0>(cur.a[i]) & bits_of<0>(ma[i]));
            panel[1][2 * wave + i][lane] = expand32(bits_of<1>(cur.a[i]) & bits_of<1>(ma[i]));
        }
#pragma unroll
        for (int j = 0; j < kGK; ++j) b[j] = expand32(bits_of<0>(cur.b[j]) & bits_of<0>(mb[j]));
        __syncthreads();
        for (int64_t w = w0; w < w1; w += kGS) {
            const Words nxt = load_words(pa, pb, w + kGS < last ? w + kGS : last);
            gram_step<2, 1, false>(cur, cur, ma, mb, panel[0], panel[2], wave, lane, active, b, nb, acc);
            gram_step<3, 2, true>(cur, cur, ma, mb, panel[1], panel[3], wave, lane, active, nb, b, acc);
            gram_step<0, 3, false>(nxt, cur, ma, mb, panel[2], panel[0], wave, lane, active, b, nb, acc);
            gram_step<1, 0, true>(nxt, nxt, ma, mb, panel[3], panel[1], wave, lane, active, nb, b, acc);
            cur = nxt;
        }
    }
    if (!active) return;
    // D layout of a 16x16 MFMA tile: lane l, element e -> row 4*(l/16)+e, column l%16
#pragma unroll
    for (int i = 0; i < kGR; ++i)
#pragma unroll
        for (int j = 0; j < kGK; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int32_t v = (int32_t)acc[i][j][e];
                if (v) {
                    const int64_t row = (int64_t)I * kGT + i * 16 + 4 * grp + e;
                    const int64_t cc = (int64_t)col0 + j * 16 + col;
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

hipError_t launch_gram(const fc_db *db, const int32_t *rowidx, int32_t np, int32_t *C,
                       int64_t ldc, const char *name, double alg_bytes, double alg_ops,
                       hipStream_t s) {
    if (db->m == 0 || np == 0) return hipSuccess;
    const int32_t ncb = np / kGC, nrb = np / kGT;
    int32_t npairs = 0;  // (row block, column block) pairs reaching the upper triangle
    for (int32_t I = 0; I < nrb; ++I) npairs += ncb - I * kGT / kGC;
    const int64_t tiles = db->words / (kTileRows / 64);
    // as many splits as fill the resident workgroups once, whole 64-word
    // tiles each
    static const int per_cu = [] {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)k_gram, 256, 0) !=
                hipSuccess || nb < 1) {
            (void)hipGetLastError();
            nb = 2;
        }
        return nb;
    }();
    int64_t splits = (int64_t)per_cu * db->cu_count / npairs;
    splits = std::min<int64_t>(splits, tiles);
    // at most 4096 tiles (2^24 instances) per workgroup keeps the fp32 sums exact
    splits = std::max<int64_t>(splits, (tiles + 4095) / 4096);
    if (splits < 1) splits = 1;
    ProfScope ps(name, s, alg_bytes, alg_ops);
    hipLaunchKernelGGL(k_gram, dim3((unsigned)(npairs * splits)), dim3(256), 0, s, db->d_bits,
                       db->words, db->pitch / 64, rowidx, nrb, ncb, npairs, (int32_t)splits, C,
                       (int32_t)ldc);
    const hipError_t e = hipGetLastError();
    ps.end(s);
    return e;
}

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
    const int32_t ncb = (ni + kGC - 1) / kGC;  // column blocks
    const int32_t np = ncb * kGC;              // items padded to whole blocks
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
    // no support exceeds 1: minsup >= 1 (however large) admits no pair, and
    // the product below then stays within int64
    const double start = std::floor(std::min(minsup, 1.0) * m) - 2.0;
    int64_t nmin = start > 0.0 ? (int64_t)start : 0;
    while (!((double)nmin / m > minsup) && nmin <= db->m) ++nmin;
    if (db->m == 0) nmin = 1;  // no instance: no pair has support
    hipStream_t s = (hipStream_t)stream;
    FC_HIP(hipSetDevice(db->device));
    // the Gram, the row items, the per-row counts and offsets in one
    // workspace of the handle; device copies of host outputs separately
    DevBuf dRec, dG;
    const int64_t ldc = np;
    const size_t cb = (sizeof(int32_t) * (size_t)np * (size_t)np + 255) & ~(size_t)255;
    const size_t rb = (sizeof(int32_t) * (size_t)np + 255) & ~(size_t)255;
    const size_t nb = (sizeof(int32_t) * (size_t)ni + 255) & ~(size_t)255;
    Workspace *w = workspace_acquire(db, cb + rb + nb + sizeof(int64_t) * (size_t)ni, s);
    if (!w) {
        set_error("fc_pairs: device workspace could not be allocated");
        return FC_ERR_NOMEM;
    }
    struct Release {
        fc_db *db;
        Workspace *w;
        hipStream_t s;
        ~Release() { workspace_release(db, w, s); }
    } release{db, w, s};
    int32_t *C = (int32_t *)w->p;
    int32_t *d_row = (int32_t *)((char *)w->p + cb);
    int32_t *d_cnt = (int32_t *)((char *)w->p + cb + rb);
    int64_t *d_off = (int64_t *)((char *)w->p + cb + rb + nb);
    FC_HIP(hipMemcpyAsync(d_row, rowidx.data(), sizeof(int32_t) * (size_t)np,
                          hipMemcpyHostToDevice, s));
    FC_HIP(fill_zero_i32(C, (int64_t)np * np, s));
    // algorithmic work: the upper triangle with the diagonal, 2 ops per pair and instance
    const double ops = (double)db->m * (double)ni * (double)(ni + 1);
    FC_HIP(launch_gram(db, d_row, np, C, ldc, "k_gram", 0.0, ops, s));
    // records: per-row counts -> offsets (host) -> ordered writes
    hipLaunchKernelGGL(k_pair_count, dim3((unsigned)((ni + 3) / 4)), dim3(256), 0, s, C,
                       (int32_t)ldc, ni, (int32_t)std::min<int64_t>(nmin, INT32_MAX),
                       d_cnt);
    FC_HIP(hipGetLastError());
    std::vector<int32_t> cnt((size_t)ni);
    FC_HIP(hipMemcpyAsync(cnt.data(), d_cnt, sizeof(int32_t) * (size_t)ni,
                          hipMemcpyDeviceToHost, s));
    FC_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> off((size_t)ni + 1, 0);
    for (int32_t a = 0; a < ni; ++a) off[(size_t)a + 1] = off[(size_t)a] + cnt[(size_t)a];
    const int64_t total = off[(size_t)ni];
    *n_out = total;
    const int64_t nrec = std::min(total, cap);
    if (nrec > 0) {
        const bool odev = is_device_ptr(out);
        FC_HIP(hipMemcpyAsync(d_off, off.data(), sizeof(int64_t) * (size_t)ni,
                              hipMemcpyHostToDevice, s));
        fc_pair_rec *rec = out;
        if (!odev) {
            FC_HIP(dRec.alloc(sizeof(fc_pair_rec) * (size_t)nrec, s));
            rec = (fc_pair_rec *)dRec.p;
        }
        hipLaunchKernelGGL(k_pair_write, dim3((unsigned)((ni + 3) / 4)), dim3(256), 0, s, C,
                           (int32_t)ldc, ni, (int32_t)std::min<int64_t>(nmin, INT32_MAX),
                           (const int64_t *)d_off, nrec, (float)(1.0 / m), rec);
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
