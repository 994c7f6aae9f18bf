// Native support of the exact parent-set search of Section 4.2: the scores
// of every parent set of one size for one child, enumerated by the library
// so that no per-family arrays cross the language boundary.
//
// The subsets of candidate positions are visited in lexicographic order and
// counted in chunks through the batched counting path (the same plan and
// kernels as fc_count_reduce, hence the same scores).  With MDL, the
// penalty 1/2 log2(m) q (r - 1) is a lower bound of a family's score that
// grows with every added parent, so a set whose penalty already reaches the
// caller's bound is not counted (exact pruning).
#include <cmath>
#include <cstring>
#include <functional>
#include <thread>
#include <vector>

#include "fc_internal.h"

namespace fc {

namespace {

// scores[slot * nsets + idx[i]] = part[slot * nkept + i] for every slot.
__global__ void k_scatter_scores(const float *__restrict__ part, const int64_t *__restrict__ idx,
                                 int64_t nkept, int32_t nslots, int64_t nsets,
                                 float *__restrict__ scores) {
    const int64_t total = nkept * nslots;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t slot = t / nkept, i = t % nkept;
        scores[slot * nsets + idx[i]] = part[t];
    }
}

__global__ void k_fill_f32(float *__restrict__ p, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

unsigned grid_for(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536));
}

// C(n, k) or -1 when it exceeds 2^62.
int64_t binom(int64_t n, int64_t k) {
    if (k < 0 || k > n) return 0;
    k = std::min(k, n - k);
    double r = 1.0;
    int64_t v = 1;
    for (int64_t i = 1; i <= k; ++i) {
        r = r * (double)(n - k + i) / (double)i;
        if (r > 4.0e18) return -1;
        v = v * (n - k + i) / i;  // exact: v is C(n-k+i, i) after each step
    }
    return v;
}

constexpr int64_t kChunk = int64_t(1) << 19;  // families counted per submission

}  // namespace

}  // namespace fc

using namespace fc;

extern "C" int fc_score_parent_sets(fc_db *db, int32_t child, const int32_t *cand, int32_t ncand,
                                    int32_t size, uint32_t reducers, const fc_reduce_params *p,
                                    double prune_mdl, float *scores, int64_t nsets,
                                    void *stream) {
    clear_error();
    if (!db || (ncand > 0 && !cand) || ncand < 0 || size < 0 || size > ncand ||
        size + 1 > FC_MAX_VARS) {
        set_error("fc_score_parent_sets: need a database, 0 <= size <= ncand and size + 1 <= %d",
                  FC_MAX_VARS);
        return FC_ERR_INVALID;
    }
    if (child < 0 || child >= db->n) {
        set_error("fc_score_parent_sets: child %d out of range", child);
        return FC_ERR_INVALID;
    }
    std::vector<uint8_t> seen((size_t)db->n, 0);
    seen[(size_t)child] = 1;
    for (int32_t i = 0; i < ncand; ++i) {
        const int32_t v = cand[i];
        if (v < 0 || v >= db->n || seen[(size_t)v]++) {
            set_error("fc_score_parent_sets: candidate %d (variable %d) is out of range, "
                      "repeated or the child", i, v);
            return FC_ERR_INVALID;
        }
    }
    if (reducers == 0 || (reducers & ~(uint32_t)(FC_RED_LL | FC_RED_MDL | FC_RED_BDEU | FC_RED_MI))) {
        set_error("fc_score_parent_sets: reducer mask %#x is empty or unknown", reducers);
        return FC_ERR_INVALID;
    }
    if (prune_mdl > 0.0 && reducers != FC_RED_MDL) {
        set_error("fc_score_parent_sets: pruning needs reducers == FC_RED_MDL");
        return FC_ERR_INVALID;
    }
    const double ess = p ? p->ess : 1.0;
    if (!(ess > 0.0)) {
        set_error("fc_score_parent_sets: ess must be > 0");
        return FC_ERR_INVALID;
    }
    const int64_t want = binom(ncand, size);
    if (want < 0 || nsets != want) {
        set_error("fc_score_parent_sets: nsets=%lld but C(%d, %d) sets exist", (long long)nsets,
                  ncand, size);
        return FC_ERR_INVALID;
    }
    if (nsets > 0 && !scores) {
        set_error("fc_score_parent_sets: scores is NULL");
        return FC_ERR_INVALID;
    }
    if (nsets == 0) return FC_OK;
    hipStream_t s = (hipStream_t)stream;
    FC_HIP(hipSetDevice(db->device));
    const int nred = __builtin_popcount(reducers);
    const bool sdev = is_device_ptr(scores);
    DevBuf dall;
    float *out = scores;
    if (!sdev) {
        FC_HIP(dall.alloc(sizeof(float) * (size_t)nred * (size_t)nsets, s));
        out = (float *)dall.p;
    }
    const bool prune = prune_mdl > 0.0;
    if (prune) {  // pruned sets keep +infinity
        hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(nsets)), dim3(256), 0, s, out, nsets,
                           INFINITY);
        FC_HIP(hipGetLastError());
    }
    // penalty factor of the child: 1/2 log2(m) (r - 1), in binary64
    const double pen_unit =
        db->m > 0 ? 0.5 * std::log2((double)db->m) * (double)(db->arity[(size_t)child] - 1) : 0.0;
    // Sets are enumerated in chunks; a chunk is split over host threads, each
    // starting from the unranked subset at its first index.
    unsigned hw = std::thread::hardware_concurrency();
    const int T = (int)std::max<unsigned>(1u, std::min(16u, hw ? hw : 1u));
    struct Part {
        std::vector<int32_t> flat;
        std::vector<int64_t> idx;
    };
    std::vector<Part> parts((size_t)T);
    auto enumerate = [&](Part &pt, int64_t lo, int64_t hi) {
        pt.flat.clear();
        pt.idx.clear();
        if (lo >= hi) return;
        // unrank lo: positions of the lo-th subset in lexicographic order
        std::vector<int32_t> pos((size_t)size);
        int64_t r = lo;
        int32_t x = 0;
        for (int32_t t = 0; t < size; ++t) {
            while (binom(ncand - x - 1, size - t - 1) <= r) {
                r -= binom(ncand - x - 1, size - t - 1);
                ++x;
            }
            pos[(size_t)t] = x++;
        }
        pt.flat.reserve((size_t)(hi - lo) * (size_t)(size + 1));
        pt.idx.reserve((size_t)(hi - lo));
        for (int64_t i = lo; i < hi; ++i) {
            double q = 1.0;
            for (int32_t t = 0; t < size; ++t) q *= (double)db->arity[(size_t)cand[pos[(size_t)t]]];
            if (!prune || q * pen_unit < prune_mdl) {
                for (int32_t t = 0; t < size; ++t) pt.flat.push_back(cand[pos[(size_t)t]]);
                pt.flat.push_back(child);
                pt.idx.push_back(i);
            }
            // next subset: advance the rightmost position that can move
            int32_t t = size - 1;
            while (t >= 0 && pos[(size_t)t] == ncand - size + t) --t;
            if (t >= 0) {
                ++pos[(size_t)t];
                for (int32_t u = t + 1; u < size; ++u) pos[(size_t)u] = pos[(size_t)u - 1] + 1;
            }
        }
    };
    std::vector<int32_t> flat;
    std::vector<int64_t> off, idx;
    for (int64_t base = 0; base < nsets; base += kChunk) {
        const int64_t end = std::min(nsets, base + kChunk);
        const int tn = (end - base) >= 4096 ? T : 1;
        std::vector<std::thread> th;
        for (int t = 0; t < tn; ++t) {
            const int64_t lo = base + (end - base) * t / tn, hi = base + (end - base) * (t + 1) / tn;
            if (tn == 1)
                enumerate(parts[0], lo, hi);
            else
                th.emplace_back(enumerate, std::ref(parts[(size_t)t]), lo, hi);
        }
        for (auto &t : th) t.join();
        flat.clear();
        idx.clear();
        for (int t = 0; t < tn; ++t) {
            flat.insert(flat.end(), parts[(size_t)t].flat.begin(), parts[(size_t)t].flat.end());
            idx.insert(idx.end(), parts[(size_t)t].idx.begin(), parts[(size_t)t].idx.end());
        }
        off.resize(idx.size() + 1);
        for (size_t i = 0; i < off.size(); ++i) off[i] = (int64_t)i * (size + 1);
        const int64_t nkept = (int64_t)idx.size();
        if (nkept == 0) continue;
        // the chunk's scores and set indices in a workspace of the handle
        const size_t pbytes = (sizeof(float) * (size_t)nred * (size_t)nkept + 255) & ~(size_t)255;
        Workspace *w = workspace_acquire(db, pbytes + sizeof(int64_t) * (size_t)nkept, s);
        if (!w) {
            set_error("fc_score_parent_sets: device workspace could not be allocated");
            return FC_ERR_NOMEM;
        }
        struct Release {
            fc_db *db;
            Workspace *w;
            hipStream_t s;
            ~Release() { workspace_release(db, w, s); }
        } release{db, w, s};
        float *dpart = (float *)w->p;
        int64_t *didx = (int64_t *)((char *)w->p + pbytes);
        Staging *st = staging_acquire(sizeof(int64_t) * (size_t)nkept);
        if (!st) {
            set_error("fc_score_parent_sets: pinned staging allocation failed");
            return FC_ERR_NOMEM;
        }
        std::memcpy(st->host, idx.data(), sizeof(int64_t) * (size_t)nkept);
        const hipError_t e = hipMemcpyAsync(didx, st->host, sizeof(int64_t) * (size_t)nkept,
                                            hipMemcpyHostToDevice, s);
        staging_release(st, s);
        FC_HIP(e);
        int rc = count_reduce_device(db, flat.data(), off.data(), nkept, reducers, ess, dpart, s);
        if (rc) return rc;
        hipLaunchKernelGGL(k_scatter_scores, dim3(grid_for(nkept * nred)), dim3(256), 0, s,
                           (const float *)dpart, (const int64_t *)didx, nkept, nred, nsets, out);
        FC_HIP(hipGetLastError());
    }
    if (!sdev) {
        FC_HIP(hipMemcpyAsync(scores, out, sizeof(float) * (size_t)nred * (size_t)nsets,
                              hipMemcpyDeviceToHost, s));
        FC_HIP(hipStreamSynchronize(s));
    }
    return FC_OK;
}
