// Fused score reducers over finished contingency tables, in float32.
//
// The stream interface of Section 3.1 hands a function object (N_ijk, N_ij)
// pairs; here a fixed set of reducers reads each finished table once (row
// sums N_ij from the contiguous child slice, child marginals N_.k from the
// database marginals) and accumulates with Neumaier compensated summation.
// One wave owns one table and the order of every addition depends only on
// that table, so a score is bit-identical whether its query ran alone or in
// any batch.
//
// The plain formulas lose most of their float32 digits to cancellation
// (lnGamma terms of size N log N whose difference is small; mutual
// information terms of both signs around zero), so each reducer is evaluated
// in a form whose summands share one sign or are small:
//  * LL (Eq. (1)): N log(N/N_j) with log1p(-(N_j-N)/N_j) when N > N_j/2.
//  * BDeu: lnGamma(z) = f(z) + ln(2 pi)/2 + R(z), f(z) = (z-1/2) ln z - z.
//    Per parent configuration j with Z = N_j + a_j, z_k = N_jk + a_jk and
//    K = {k : N_jk > 0} the exact identity
//      sum_K f(z_k) - f(Z) = sum_K (z_k - 1/2) ln(z_k/Z)
//                            - [(r-|K|) a_jk + (|K|-1)/2] ln Z + (r-|K|) a_jk
//    removes the N ln N parts; R is the Stirling series for z >= 8 and
//    lgamma - f - ln(2 pi)/2 below.
//  * MI: with e = N_j N_k / m and d = (m N - N_j N_k)/(N_j N_k) (exact
//    integers), m MI = sum over all cells with N_j, N_k > 0 of e g(d),
//    g(d) = (1+d) ln(1+d) - d >= 0, because sum e d = 0; g uses an atanh
//    series near 0.
// Each summand's magnitude (of its largest intermediate) is accumulated to
// give a per-result absolute error estimate.
#include <cmath>

#include "fc_internal.h"

namespace fc {

namespace {

constexpr float kHalfLn2Pi = 0.918938533204672742f;
constexpr float kInvLn2 = 1.44269504088896341f;
constexpr float kEps = 5.9604644775390625e-8f;  // 2^-24

struct Acc {
    float s = 0.f, c = 0.f, mag = 0.f;
    __device__ __forceinline__ void add(float x, float m) {
        float t = s + x;
        if (fabsf(s) >= fabsf(x))
            c += (s - t) + x;
        else
            c += (x - t) + s;
        s = t;
        mag += m;
    }
    __device__ __forceinline__ void add(float x) { add(x, fabsf(x)); }
};

// Exact error-free combination of two lanes' accumulators (TwoSum), so the
// butterfly gives the same bits in every lane.
__device__ __forceinline__ void combine(Acc &a, const Acc &b) {
    float s = a.s + b.s;
    float bb = s - a.s;
    float e = (a.s - (s - bb)) + (b.s - bb);
    a.c = (a.c + b.c) + e;
    a.s = s;
    a.mag = a.mag + b.mag;
}

__device__ __forceinline__ void wave_reduce(Acc &a) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        Acc o;
        o.s = __shfl_xor(a.s, off);
        o.c = __shfl_xor(a.c, off);
        o.mag = __shfl_xor(a.mag, off);
        combine(a, o);
    }
}

// ln(N / Nj) for 0 < N <= Nj, accurate when the ratio is close to 1.
__device__ __forceinline__ float log_ratio(int64_t n, int64_t nj) {
    if (2 * n > nj) return log1pf(-(float)(nj - n) / (float)nj);
    return logf((float)n / (float)nj);
}

// R(z) = lnGamma(z) - (z - 1/2) ln z + z - ln(2 pi)/2, and the magnitude of
// the values it is formed from.
__device__ __forceinline__ float stirling_rem(float z, float &mag) {
    if (z >= 8.0f) {
        float w = 1.0f / z, w2 = w * w;
        float r = w * (1.0f / 12.0f - w2 * (1.0f / 360.0f - w2 * (1.0f / 1260.0f - w2 * (1.0f / 1680.0f))));
        mag = r;
        return r;
    }
    float lg = lgammaf(z);
    float f = (z - 0.5f) * logf(z) - z;
    mag = fabsf(lg) + fabsf(f) + kHalfLn2Pi;
    return (lg - f) - kHalfLn2Pi;
}

// g(d) = (1 + d) ln(1 + d) - d for d >= -1.
__device__ __forceinline__ float g_fun(float d) {
    if (d > -0.6f && d < 2.0f) {
        float u = d / (2.0f + d), u2 = u * u;
        // sum_{i>=0} u^(2i) / (2i+3), 14 terms (u^2 < 0.25)
        float sser = 1.0f / 29.0f;
        sser = 1.0f / 27.0f + u2 * sser;
        sser = 1.0f / 25.0f + u2 * sser;
        sser = 1.0f / 23.0f + u2 * sser;
        sser = 1.0f / 21.0f + u2 * sser;
        sser = 1.0f / 19.0f + u2 * sser;
        sser = 1.0f / 17.0f + u2 * sser;
        sser = 1.0f / 15.0f + u2 * sser;
        sser = 1.0f / 13.0f + u2 * sser;
        sser = 1.0f / 11.0f + u2 * sser;
        sser = 1.0f / 9.0f + u2 * sser;
        sser = 1.0f / 7.0f + u2 * sser;
        sser = 1.0f / 5.0f + u2 * sser;
        sser = 1.0f / 3.0f + u2 * sser;
        return d * d / (2.0f + d) + 2.0f * (1.0f + d) * u * u2 * sser;
    }
    return (1.0f + d) * log1pf(d) - d;
}

__global__ __launch_bounds__(256) void k_reduce(const QDesc *__restrict__ descs, int64_t nd,
                                                int64_t nq,
                                                const int32_t *__restrict__ tables,
                                                const uint8_t *__restrict__ arity,
                                                const int32_t *__restrict__ soff,
                                                const int32_t *__restrict__ marg, int64_t m,
                                                uint32_t reducers, float ess,
                                                float *__restrict__ scores,
                                                float *__restrict__ err) {
    // R(z) of BDeu's small arguments, per wave: z = n + a_jk and z = n + a_j
    // for n = 0..7, each computed once by one lane exactly as a cell would
    __shared__ float rtab[4][2][8], mtab[4][2][8];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t di = (int64_t)blockIdx.x * 4 + wv;
    if (di >= nd) return;
    const QDesc &d = descs[di];
    const int32_t child = d.var[d.k - 1];
    const int32_t r = arity[child];
    const int64_t q = (int64_t)d.cells / r;
    const int32_t *T = tables + d.table_off;
    const int32_t *nk = marg + soff[child];

    const bool want_ll = reducers & (FC_RED_LL | FC_RED_MDL);
    const bool want_bd = reducers & FC_RED_BDEU;
    const bool want_mi = reducers & FC_RED_MI;

    // BDeu constants: a_j = ess/q, a_jk = ess/(r q); G2 = lnGamma(a_jk),
    // D0 = lnGamma(a_j) - lnGamma(a_jk), both without cancellation.
    const float a1 = ess / (float)q;
    const float a2 = a1 / (float)r;
    const float da = a1 - a2;
    float G2, D0;
    if (a2 < 1.0f)
        G2 = lgammaf(1.0f + a2) - logf(a2);
    else
        G2 = lgammaf(a2);
    if (a1 < 1.0f)
        D0 = -logf((float)r) + (lgammaf(1.0f + a1) - lgammaf(1.0f + a2));
    else
        D0 = lgammaf(a1) - G2;
    if (want_bd && lane < 16) {
        const float z = (float)(lane & 7) + ((lane < 8) ? a2 : a1);
        float rm;
        const float rz = stirling_rem(z, rm);
        rtab[wv][lane >> 3][lane & 7] = rz;
        mtab[wv][lane >> 3][lane & 7] = rm;
    }
    // the 64 lanes of a wave run in lockstep: the tables are complete here
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const float c3 = kHalfLn2Pi - G2;
    const float c3mag = kHalfLn2Pi + fabsf(G2);
    const float fm = (float)m;
    const float inv_m = 1.0f / fm;

    Acc ll, bd, mi;
    for (int64_t j = lane; j < q; j += 64) {
        const int32_t *row = T + j * r;
        int64_t nj = 0;
        int32_t kc = 0;
        for (int32_t k = 0; k < r; ++k) {
            int32_t v = row[k];
            nj += v;
            kc += v > 0;
        }
        if (nj == 0) continue;
        float Z = 0.f, lnZ = 0.f, invZ = 0.f;
        if (want_bd) {
            Z = (float)nj + a1;
            lnZ = logf(Z);
            invZ = 1.0f / Z;
            float t1 = -((float)(r - kc) * a2 + 0.5f * (float)(kc - 1)) * lnZ;
            bd.add(t1);
            bd.add((float)(r - kc) * a2);
            bd.add((float)(kc - 1) * c3, (float)(kc - 1) * c3mag);
            bd.add(D0, fabsf(D0) + 2.0f);
            float rm, rZ;
            if (nj < 8) {
                rZ = rtab[wv][1][nj];
                rm = mtab[wv][1][nj];
            } else {
                rZ = stirling_rem(Z, rm);
            }
            bd.add(-rZ, rm);
        }
        for (int32_t k = 0; k < r; ++k) {
            const int64_t n = row[k];
            if (want_mi && nk[k] > 0) {
                const int64_t den = nj * (int64_t)nk[k];
                const float e = (float)den * inv_m;
                if (n == 0) {
                    mi.add(e);
                } else {
                    const int64_t num = m * n - den;
                    const float dd = (float)num / (float)den;
                    mi.add(e * g_fun(dd));
                }
            }
            if (n == 0) continue;
            if (want_ll) {
                float t = (float)n * log_ratio(n, nj);
                ll.add(t);
            }
            if (want_bd) {
                const float zk = (float)n + a2;
                const float dz = (float)(nj - n) + da;  // Z - z_k
                const float lr = (dz < 0.5f * Z) ? log1pf(-dz * invZ) : logf(zk * invZ);
                bd.add(((float)n + (a2 - 0.5f)) * lr);
                float rm, rk;
                if (n < 8) {
                    rk = rtab[wv][0][n];
                    rm = mtab[wv][0][n];
                } else {
                    rk = stirling_rem(zk, rm);
                }
                bd.add(rk, rm);
            }
        }
    }
    int slot = 0;
    const int64_t base = d.qid;
    if (want_ll) wave_reduce(ll);
    if (want_bd) wave_reduce(bd);
    if (want_mi) wave_reduce(mi);
    if (lane != 0) return;
    if (reducers & FC_RED_LL) {
        float v = (ll.s + ll.c) * kInvLn2;
        scores[slot * nq + base] = v;
        if (err) err[slot * nq + base] = kEps * (24.0f * ll.mag * kInvLn2 + 2.0f * fabsf(v));
        ++slot;
    }
    if (reducers & FC_RED_MDL) {
        const float pen = 0.5f * log2f(fm) * (float)q * (float)(r - 1);
        Acc t;
        t.add(-ll.s * kInvLn2);
        t.add(-ll.c * kInvLn2);
        t.add(pen);
        float v = t.s + t.c;
        scores[slot * nq + base] = v;
        if (err) err[slot * nq + base] = kEps * (24.0f * ll.mag * kInvLn2 + 8.0f * pen + 2.0f * fabsf(v));
        ++slot;
    }
    if (reducers & FC_RED_BDEU) {
        float v = bd.s + bd.c;
        scores[slot * nq + base] = v;
        if (err) err[slot * nq + base] = kEps * (24.0f * bd.mag + 2.0f * fabsf(v));
        ++slot;
    }
    if (reducers & FC_RED_MI) {
        float v = (mi.s + mi.c) / fm;
        scores[slot * nq + base] = v;
        if (err) err[slot * nq + base] = kEps * (24.0f * mi.mag / fm + 2.0f * fabsf(v));
        ++slot;
    }
}

}  // namespace

hipError_t launch_reduce(const fc_db *db, const QDesc *descs, int64_t nd, int64_t nq,
                         const int32_t *tables, uint32_t reducers, double ess, float *scores,
                         float *err, hipStream_t s) {
    if (nd <= 0) return hipSuccess;
    int64_t blocks = (nd + 3) / 4;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)blocks), dim3(256), 0, s, descs, nd, nq, tables,
                       db->d_arity, db->d_soff, db->d_marg, db->m, reducers, (float)ess, scores,
                       err);
    return hipGetLastError();
}

}  // namespace fc
