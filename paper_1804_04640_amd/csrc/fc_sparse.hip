// Sparse contingency tables for queries whose full table dwarfs the data
// (prod r_v >> m): only the configurations that occur, at most min(q r, m) of
// them (Section 3.2), as (mixed-radix key, count) pairs in increasing key
// order.  Sort-and-segment: every instance's key is formed on the device,
// radix-sorted over just the significant bits, and run-length encoded -- the
// MSD ordering of Section 3.3 taken to completion, without any dense table.
//
// Batches: consecutive queries form windows (at most kWindowKeys keys).
// Within a window the queries are ordered by key space and cut into groups;
// query t of a group contributes the composite keys base_t + key_t(p), where
// base_t is the sum of the key spaces of the group's queries before it, so
// one radix sort over the group's keys, on ceil(log2(sum of key spaces))
// bits, orders every query's keys after its query and one run-length
// encoding yields every query's runs.  Composite keys are 32-bit when the
// group's key spaces sum to at most 2^32.  A window's run counts are scanned
// in the caller's query order and every group then copies its runs to their
// packed output positions.  A single query is a window of one.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "fc_internal.h"

namespace fc {
namespace {

struct BatchSpec {
    int32_t var[FC_MAX_VARS];
    uint64_t stride[FC_MAX_VARS];
    uint64_t cells;  // key space of the query (product of its arities)
    uint64_t base;   // first composite key of the query within its group
    int64_t orig;    // index of the query in the caller's batch
    int32_t k;
    int32_t pad;
};

constexpr int kKeysPerThread = 8;

// Keys of 8 consecutive instances per thread: one 8-byte load per column
// (columns are padded to whole tiles, so the load stays inside the column),
// all loads issued before the arithmetic.  blockIdx.y is the query's place
// in its group.
template <typename K>
__global__ __launch_bounds__(256) void k_keys_batch(const uint8_t *__restrict__ cols, int64_t m,
                                                    int64_t pitch,
                                                    const BatchSpec *__restrict__ specs,
                                                    K *__restrict__ keys, int top_lo, int top_width,
                                                    uint32_t *__restrict__ top_hist) {
    __shared__ uint32_t hist[256];
    hist[threadIdx.x] = 0u;
    __syncthreads();
    const int32_t j = blockIdx.y;
    const BatchSpec q = specs[j];
    K *out = keys + (int64_t)j * m;
    const uint32_t dmask = (1u << top_width) - 1u;
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
        for (int e = 0; e < kKeysPerThread; ++e) key[e] = q.base;
#pragma unroll
        for (int t = 0; t < FC_MAX_VARS; ++t) {
            if (t < q.k) {
                const uint64_t st = q.stride[t];
#pragma unroll
                for (int e = 0; e < kKeysPerThread; ++e)
                    key[e] += ((w[t] >> (8 * e)) & 0xFF) * st;
            }
        }
        const int ne = (int)min((int64_t)kKeysPerThread, m - p0);
#pragma unroll
        for (int e = 0; e < kKeysPerThread; ++e)
            if (e < ne) atomicAdd(&hist[(uint32_t)(key[e] >> top_lo) & dmask], 1u);
        if (ne == kKeysPerThread) {
#pragma unroll
            for (int e = 0; e < kKeysPerThread; ++e) out[p0 + e] = (K)key[e];
        } else {
            for (int e = 0; e < ne; ++e) out[p0 + e] = (K)key[e];
        }
    }
    __syncthreads();
    const uint32_t c = hist[threadIdx.x];
    if (c) atomicAdd(&top_hist[threadIdx.x], c);
}

// Runs of each query of a group: [run_lo, run_hi) of the group's run list,
// stored at the query's caller index.
template <typename K>
__global__ void k_group_runs(const K *__restrict__ uniq, const uint32_t *__restrict__ nruns,
                             const BatchSpec *__restrict__ specs, int32_t G,
                             int64_t *__restrict__ run_lo, int64_t *__restrict__ run_hi) {
    const int64_t nr = *nruns;
    auto lower = [&](uint64_t first) {
        int64_t lo = 0, hi = nr;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((uint64_t)uniq[mid] < first) lo = mid + 1; else hi = mid;
        }
        return lo;
    };
    for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < G; t += gridDim.x * blockDim.x) {
        const int64_t j = specs[t].orig;
        run_lo[j] = lower(specs[t].base);
        run_hi[j] = t + 1 < G ? lower(specs[t + 1].base) : nr;
    }
}

// Output offsets of the window's queries [w0, w0 + wn) in caller order:
// off[j] = *total + (runs of the window's queries before j); off[w0 + wn]
// and *total advance past the window.  One workgroup of kScanThreads.
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void k_window_scan(
    const int64_t *__restrict__ run_lo, const int64_t *__restrict__ run_hi, int64_t w0, int64_t wn,
    int64_t *__restrict__ total, int64_t *__restrict__ off) {
    __shared__ int64_t part[kScanThreads];
    const int64_t base = *total;
    const int64_t per = (wn + kScanThreads - 1) / kScanThreads;
    const int64_t a0 = (int64_t)threadIdx.x * per;
    const int64_t a = a0 < wn ? a0 : wn, b = a + per < wn ? a + per : wn;
    int64_t s = 0;
    for (int64_t i = a; i < b; ++i) s += run_hi[w0 + i] - run_lo[w0 + i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {  // inclusive scan of the per-thread sums
        const int64_t v = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t o = base + part[threadIdx.x] - s;
    for (int64_t i = a; i < b; ++i) {
        off[w0 + i] = o;
        o += run_hi[w0 + i] - run_lo[w0 + i];
    }
    if (threadIdx.x == kScanThreads - 1) {
        off[w0 + wn] = base + part[kScanThreads - 1];
        *total = base + part[kScanThreads - 1];
    }
}

// Copies the runs of each query of a group (blockIdx.y = its place in the
// group) to off[j] in the packed output, keys less the query's base.  The
// window's runs end at *win_end.  truncate: pairs at positions < cap are
// written; otherwise a window that does not fit whole writes nothing.
// Either way *overflow is set when the runs exceed cap.
template <typename K>
__global__ void k_emit_group(const K *__restrict__ uniq, const uint32_t *__restrict__ cnt,
                             const BatchSpec *__restrict__ specs,
                             const int64_t *__restrict__ run_lo, const int64_t *__restrict__ run_hi,
                             const int64_t *__restrict__ off, const int64_t *__restrict__ win_end,
                             int64_t *__restrict__ keys, int32_t *__restrict__ counts, int64_t cap,
                             int32_t truncate, int32_t *__restrict__ overflow) {
    const BatchSpec q = specs[blockIdx.y];
    const int64_t j = q.orig, lo = run_lo[j], dst = off[j];
    int64_t n = run_hi[j] - lo;
    if (*win_end > cap) {
        if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *overflow = 1;
        if (!truncate) return;
        const int64_t room = cap > dst ? cap - dst : 0;
        if (n > room) n = room;
    }
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        keys[dst + r] = (int64_t)((uint64_t)uniq[lo + r] - q.base);
        counts[dst + r] = (int32_t)cnt[lo + r];
    }
}

int sparse_spec(const fc_db *db, const int32_t *vars, int32_t k, const char *who, BatchSpec *spec) {
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
    spec->cells = (uint64_t)cells;
    return FC_OK;
}

unsigned bits_of(unsigned __int128 S) {  // bits of a key in [0, S)
    unsigned b = 1;
    while (b < 64 && ((unsigned __int128)1 << b) < S) ++b;
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
    int64_t q0;      // first place in processing order
    int32_t G;       // queries
    unsigned end_bit;
    bool wide;       // 64-bit composite keys
    size_t tmp_bytes;
    size_t ret_off;  // its retained runs within the window's region
};

struct Window {
    int64_t w0, wn;  // caller queries [w0, w0 + wn)
    size_t g0, ng;   // its groups
};

// Estimated microseconds of one group's sort and run-length encoding on
// MI355X by the MSD partition (fc_msd.hip): a fixed cost per 8-bit level
// (its eight launches run whether or not the level has segments) plus a
// cost per key that depends on the key width, measured on the high-arity
// workload.  Used only to choose groups.
double group_cost_us(int64_t nk, unsigned end_bit, bool wide) {
    const double levels = (double)((end_bit + 7) / 8);
    const double ns = wide ? 0.048 : 0.036;
    return 30.0 + 40.0 * levels + 1e-3 * ns * (double)nk;
}

template <typename K>
size_t sort_tmp_bytes(int64_t nk, unsigned end_bit, hipStream_t s, int *rc) {
    (void)end_bit;
    (void)s;
    (void)rc;
    return msd_scratch_bytes(nk, sizeof(K));
}

// Retained runs of one group: unique keys, counts, run count.
template <typename K>
struct Runs {
    K *uniq;
    uint32_t *cnt, *nruns;
    void carve(Carve &c, int64_t nk) {
        uniq = c.take<K>((size_t)nk);
        cnt = c.take<uint32_t>((size_t)nk);
        nruns = c.take<uint32_t>(1);
    }
};

// Per-window device state shared by its groups.
struct WindowBufs {
    const BatchSpec *specs;  // processing order
    int64_t *run_lo, *run_hi, *off, *total;
    int32_t *overflow;
    char *retained, *kin, *ksort, *tmp;
    int64_t *keys;
    int32_t *counts;
    int64_t cap;
    int32_t truncate;
};

// One group through key formation, sort, run-length encoding and the
// per-query run bounds, all enqueued on s.
template <typename K>
int sparse_group(fc_db *db, const Group &g, double col_bytes, const WindowBufs &B, hipStream_t s) {
    const int64_t m = db->m, nk = (int64_t)g.G * m;
    K *kin = (K *)B.kin, *ksort = (K *)B.ksort;
    Carve c;
    c.base = B.retained + g.ret_off;
    Runs<K> R;
    R.carve(c, nk);
    const char *kname = sizeof(K) == 8 ? "k_keys_batch<u64>" : "k_keys_batch<u32>";
    // the keys' top-digit histogram (the partition's first level) is taken
    // as they are formed
    uint32_t *top_hist = msd_top_hist(B.tmp, nk, sizeof(K));
    const int top_lo = std::max((int)g.end_bit - 8, 0), top_width = (int)g.end_bit - top_lo;
    FC_HIP(fill_zero_i32((int32_t *)top_hist, 256, s));
    {
        // algorithmic bytes: the group's columns read, its keys written
        ProfScope ps(kname, s, col_bytes + (double)sizeof(K) * (double)nk, 0.0);
        const int64_t per_q = (m + kKeysPerThread - 1) / kKeysPerThread;
        const int64_t bx = std::max<int64_t>(
            1, std::min<int64_t>((per_q + 255) / 256, (8 * (int64_t)db->cu_count + g.G - 1) / g.G));
        hipLaunchKernelGGL(k_keys_batch<K>, dim3((unsigned)bx, (unsigned)g.G), dim3(256), 0, s,
                           db->d_cols, m, db->pitch, B.specs + g.q0, kin, top_lo, top_width,
                           top_hist);
        FC_HIP(hipGetLastError());
        ps.end(s);
    }
    {
        // algorithmic bytes: the keys read and written once
        ProfScope ps("msd sort+rle", s, 2.0 * (double)sizeof(K) * (double)nk, 0.0);
        const int rc = msd_sort_rle<K>(db, kin, ksort, nk, g.end_bit, R.uniq, R.cnt, R.nruns,
                                       B.tmp, true, s);
        ps.end(s);
        if (rc != FC_OK) return rc;
    }
    hipLaunchKernelGGL(k_group_runs<K>, dim3((unsigned)((g.G + 255) / 256)), dim3(256), 0, s,
                       R.uniq, R.nruns, B.specs + g.q0, g.G, B.run_lo, B.run_hi);
    FC_HIP(hipGetLastError());
    return FC_OK;
}

// A group's runs copied to their packed output positions.
template <typename K>
int sparse_emit(fc_db *db, const Group &g, const int64_t *win_end, const WindowBufs &B,
                hipStream_t s) {
    const int64_t m = db->m, nk = (int64_t)g.G * m;
    Carve c;
    c.base = B.retained + g.ret_off;
    Runs<K> R;
    R.carve(c, nk);
    const int64_t bx = std::max<int64_t>(
        1, std::min<int64_t>((m + 255) / 256, (16 * (int64_t)db->cu_count + g.G - 1) / g.G));
    hipLaunchKernelGGL(k_emit_group<K>, dim3((unsigned)bx, (unsigned)g.G), dim3(256), 0, s,
                       R.uniq, R.cnt, B.specs + g.q0, B.run_lo, B.run_hi, B.off, win_end, B.keys,
                       B.counts, B.cap, B.truncate, B.overflow);
    FC_HIP(hipGetLastError());
    return FC_OK;
}

// Windows of consecutive queries, each cut into groups.  proc receives the
// specs in processing order (window by window, by key space within a
// window) with their group bases set.
int plan_groups(const std::vector<BatchSpec> &specs, int64_t m, hipStream_t s,
                std::vector<BatchSpec> &proc, std::vector<Group> &groups,
                std::vector<Window> &windows) {
    const int64_t nq = (int64_t)specs.size();
    // at most kWindowKeys keys per window (m alone when m is larger), at most
    // kGroupKeys keys per group of several queries, at most kGroupMax queries
    // per group (the grid's y extent)
    constexpr int64_t kWindowKeys = int64_t(1) << 27, kWindowQueries = int64_t(1) << 20;
    constexpr int64_t kGroupKeys = int64_t(1) << 26;
    constexpr int32_t kGroupMax = 65535;
    const int64_t wq = std::min<int64_t>(kWindowQueries, std::max<int64_t>(1, kWindowKeys / m));
    const int64_t gmax = std::min<int64_t>(kGroupMax, std::max<int64_t>(1, kGroupKeys / m));
    proc.resize((size_t)nq);
    std::vector<int64_t> idx;
    std::vector<unsigned __int128> P;
    std::vector<double> best;
    std::vector<int64_t> from;
    for (int64_t w0 = 0; w0 < nq; w0 += wq) {
        const int64_t wn = std::min(wq, nq - w0);
        idx.resize((size_t)wn);
        std::iota(idx.begin(), idx.end(), w0);
        std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
            return specs[(size_t)a].cells < specs[(size_t)b].cells;
        });
        P.assign((size_t)wn + 1, 0);
        for (int64_t i = 0; i < wn; ++i) P[(size_t)i + 1] = P[(size_t)i] + specs[(size_t)idx[(size_t)i]].cells;
        // cheapest cut into groups; the candidate ends from place i are the
        // last place each key width / pass count still admits
        best.assign((size_t)wn + 1, 1e300);
        from.assign((size_t)wn + 1, -1);
        best[0] = 0.0;
        for (int64_t i = 0; i < wn; ++i) {
            const int64_t emax = std::min(wn, i + gmax);
            int64_t cand[10];
            int nc = 0;
            cand[nc++] = i + 1;
            for (int b = 8; b <= 64; b += 8) {
                const unsigned __int128 lim = P[(size_t)i] + ((unsigned __int128)1 << std::min(b, 63));
                const int64_t e = (int64_t)(std::upper_bound(P.begin() + i + 1, P.begin() + emax + 1, lim) -
                                            P.begin()) - 1;
                if (e > i + 1 && e != cand[nc - 1]) cand[nc++] = e;
            }
            for (int c = 0; c < nc; ++c) {
                const int64_t e = cand[c];
                const unsigned __int128 S = P[(size_t)e] - P[(size_t)i];
                const unsigned eb = bits_of(S);
                const double v = best[(size_t)i] + group_cost_us((e - i) * m, eb, S > ((unsigned __int128)1 << 32));
                if (v < best[(size_t)e]) {
                    best[(size_t)e] = v;
                    from[(size_t)e] = i;
                }
            }
        }
        std::vector<int64_t> cuts;
        for (int64_t e = wn; e > 0; e = from[(size_t)e]) cuts.push_back(e);
        std::reverse(cuts.begin(), cuts.end());
        Window win{w0, wn, groups.size(), 0};
        int64_t i = 0;
        size_t ret = 0;
        for (int64_t e : cuts) {
            uint64_t base = 0;
            for (int64_t t = i; t < e; ++t) {
                BatchSpec &b = proc[(size_t)(w0 + t)];
                b = specs[(size_t)idx[(size_t)t]];
                b.base = base;
                b.orig = idx[(size_t)t];
                base += b.cells;
            }
            const unsigned __int128 S = P[(size_t)e] - P[(size_t)i];
            Group g{w0 + i, (int32_t)(e - i), bits_of(S), S > ((unsigned __int128)1 << 32), 0, 0};
            const int64_t nk = (int64_t)g.G * m;
            int rc = FC_OK;
            g.tmp_bytes = g.wide ? sort_tmp_bytes<uint64_t>(nk, g.end_bit, s, &rc)
                                 : sort_tmp_bytes<uint32_t>(nk, g.end_bit, s, &rc);
            if (rc != FC_OK) return rc;
            Carve c;
            c.off = ret;
            if (g.wide) {
                Runs<uint64_t> R;
                R.carve(c, nk);
            } else {
                Runs<uint32_t> R;
                R.carve(c, nk);
            }
            g.ret_off = (ret + 255) & ~(size_t)255;
            ret = c.off;
            groups.push_back(g);
            i = e;
        }
        win.ng = groups.size() - win.g0;
        windows.push_back(win);
    }
    return FC_OK;
}

// The shared driver: windows and groups planned over validated specs;
// offsets (nq+1) and the total land in host memory; keys/counts (device or
// host memory) receive the pairs.  truncate: single-query semantics (the
// first cap pairs).
int sparse_run(fc_db *db, const std::vector<BatchSpec> &specs, int64_t *keys, int32_t *counts,
               int64_t cap, int32_t truncate, int64_t *out_off, int64_t *total_out,
               bool *overflow_out, const char *who, hipStream_t s) {
    const int64_t nq = (int64_t)specs.size(), m = db->m;
    std::vector<BatchSpec> proc;
    std::vector<Group> groups;
    std::vector<Window> windows;
    int rc = plan_groups(specs, m, s, proc, groups, windows);
    if (rc != FC_OK) return rc;
    const bool kd = cap > 0 && is_device_ptr(keys), cd = cap > 0 && is_device_ptr(counts);
    if (kd != cd) {
        set_error("%s: keys and counts must both be device or both host memory", who);
        return FC_ERR_INVALID;
    }
    const int64_t dev_cap = cap > 0 ? (kd ? cap : std::min<int64_t>(cap, nq * m)) : 0;
    // one workspace: specs, run bounds, offsets, total, overflow flag, device
    // copies of host outputs; then the largest window's retained runs and
    // its largest group's keys and sort scratch
    Carve head;
    head.take<BatchSpec>((size_t)nq);
    head.take<int64_t>((size_t)nq);
    head.take<int64_t>((size_t)nq);
    head.take<int64_t>((size_t)nq + 1);
    head.take<int64_t>(1);
    head.take<int32_t>(2);
    if (cap > 0 && !kd) {
        head.take<int64_t>((size_t)dev_cap);
        head.take<int32_t>((size_t)dev_cap);
    }
    const size_t head_bytes = (head.off + 255) & ~(size_t)255;
    size_t win_bytes = 0;
    for (const Window &w : windows) {
        size_t ret = 0, keyb = 0, tmpb = 0;
        for (size_t gi = w.g0; gi < w.g0 + w.ng; ++gi) {
            const Group &g = groups[gi];
            const int64_t nk = (int64_t)g.G * m;
            Carve c;
            c.off = g.ret_off;
            if (g.wide) {
                Runs<uint64_t> R;
                R.carve(c, nk);
            } else {
                Runs<uint32_t> R;
                R.carve(c, nk);
            }
            ret = std::max(ret, c.off);
            keyb = std::max(keyb, (g.wide ? 8 : 4) * (size_t)nk);
            tmpb = std::max(tmpb, g.tmp_bytes);
        }
        Carve c;
        c.off = ret;
        c.take<char>(keyb);
        c.take<char>(keyb);
        c.take<char>(tmpb);
        win_bytes = std::max(win_bytes, c.off);
    }
    Workspace *w = workspace_acquire(db, head_bytes + win_bytes, s);
    if (!w) {
        set_error("%s: a device workspace of %zu bytes could not be allocated", who,
                  head_bytes + win_bytes);
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
    WindowBufs B;
    BatchSpec *d_specs = h.take<BatchSpec>((size_t)nq);
    B.specs = d_specs;
    B.run_lo = h.take<int64_t>((size_t)nq);
    B.run_hi = h.take<int64_t>((size_t)nq);
    B.off = h.take<int64_t>((size_t)nq + 1);
    B.total = h.take<int64_t>(1);
    B.overflow = h.take<int32_t>(2);
    B.keys = keys;
    B.counts = counts;
    if (cap > 0 && !kd) {
        B.keys = h.take<int64_t>((size_t)dev_cap);
        B.counts = h.take<int32_t>((size_t)dev_cap);
    }
    B.cap = dev_cap;
    B.truncate = truncate;
    B.retained = (char *)w->p + head_bytes;

    Staging *st = staging_acquire(sizeof(BatchSpec) * (size_t)nq);
    if (!st) {
        set_error("%s: pinned staging allocation failed", who);
        return FC_ERR_NOMEM;
    }
    std::memcpy(st->host, proc.data(), sizeof(BatchSpec) * (size_t)nq);
    const hipError_t ce = hipMemcpyAsync(d_specs, st->host, sizeof(BatchSpec) * (size_t)nq,
                                         hipMemcpyHostToDevice, s);
    staging_release(st, s);
    FC_HIP(ce);
    FC_HIP(fill_zero_i32((int32_t *)B.total, 2, s));
    FC_HIP(fill_zero_i32(B.overflow, 2, s));
    for (const Window &win : windows) {
        size_t ret = 0, keyb = 0;
        for (size_t gi = win.g0; gi < win.g0 + win.ng; ++gi) {
            const Group &g = groups[gi];
            const int64_t nk = (int64_t)g.G * m;
            Carve c;
            c.off = g.ret_off;
            if (g.wide) {
                Runs<uint64_t> R;
                R.carve(c, nk);
            } else {
                Runs<uint32_t> R;
                R.carve(c, nk);
            }
            ret = std::max(ret, c.off);
            keyb = std::max(keyb, (g.wide ? 8 : 4) * (size_t)nk);
        }
        Carve c;
        c.base = B.retained;
        c.off = ret;
        B.kin = c.take<char>(keyb);
        B.ksort = c.take<char>(keyb);
        B.tmp = c.take<char>(1);
        for (size_t gi = win.g0; gi < win.g0 + win.ng; ++gi) {
            const Group &g = groups[gi];
            double col_bytes = 0.0;  // one byte per variable and instance
            for (int32_t t = 0; t < g.G; ++t) col_bytes += (double)proc[(size_t)(g.q0 + t)].k * (double)m;
            rc = g.wide ? sparse_group<uint64_t>(db, g, col_bytes, B, s)
                        : sparse_group<uint32_t>(db, g, col_bytes, B, s);
            if (rc != FC_OK) return rc;
        }
        hipLaunchKernelGGL(k_window_scan, dim3(1), dim3(kScanThreads), 0, s, B.run_lo, B.run_hi,
                           win.w0, win.wn, B.total, B.off);
        FC_HIP(hipGetLastError());
        const int64_t *win_end = B.off + win.w0 + win.wn;
        for (size_t gi = win.g0; gi < win.g0 + win.ng; ++gi) {
            const Group &g = groups[gi];
            rc = g.wide ? sparse_emit<uint64_t>(db, g, win_end, B, s)
                        : sparse_emit<uint32_t>(db, g, win_end, B, s);
            if (rc != FC_OK) return rc;
        }
    }
    int64_t total = 0;
    int32_t ovf = 0;
    FC_HIP(hipMemcpyAsync(out_off, B.off, sizeof(int64_t) * (size_t)(nq + 1),
                          hipMemcpyDeviceToHost, s));
    FC_HIP(hipMemcpyAsync(&total, B.total, sizeof total, hipMemcpyDeviceToHost, s));
    FC_HIP(hipMemcpyAsync(&ovf, B.overflow, sizeof ovf, hipMemcpyDeviceToHost, s));
    FC_HIP(hipStreamSynchronize(s));
    *total_out = total;
    *overflow_out = ovf != 0 || total > cap;
    const int64_t n_copy = truncate ? std::min(total, cap) : (*overflow_out ? 0 : total);
    if (n_copy > 0 && !kd) {
        FC_HIP(hipMemcpyAsync(keys, B.keys, sizeof(int64_t) * (size_t)n_copy,
                              hipMemcpyDeviceToHost, s));
        FC_HIP(hipMemcpyAsync(counts, B.counts, sizeof(int32_t) * (size_t)n_copy,
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
    const int rc = sparse_spec(db, vars, k, who, &specs[0]);
    if (rc != FC_OK) return rc;
    FC_HIP(hipSetDevice(db->device));
    if (db->m == 0) {
        *nnz = 0;
        return FC_OK;
    }
    int64_t off[2];
    bool ovf = false;
    return sparse_run(db, specs, keys, counts, cap, 1, off, nnz, &ovf, who, (hipStream_t)stream);
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
    for (int64_t i = 0; i < nq; ++i) {
        const int64_t k = var_off[i + 1] - var_off[i];
        if (k < 1 || k > FC_MAX_VARS) {
            set_error("%s: query %lld has %lld variables (need 1..%d)", who, (long long)i,
                      (long long)k, FC_MAX_VARS);
            return FC_ERR_INVALID;
        }
        const int rc = sparse_spec(db, vars_flat + var_off[i], (int32_t)k, who,
                                   &specs[(size_t)i]);
        if (rc != FC_OK) return rc;
    }
    if (nq == 0 || db->m == 0) {
        for (int64_t i = 0; i <= nq; ++i) out_off[i] = 0;
        *total_nnz = 0;
        return FC_OK;
    }
    FC_HIP(hipSetDevice(db->device));
    bool ovf = false;
    const int rc = sparse_run(db, specs, keys, counts, cap, 0, out_off, total_nnz, &ovf, who,
                              (hipStream_t)stream);
    if (rc != FC_OK) return rc;
    if (ovf) {
        set_error("%s: %lld configurations do not fit cap = %lld (out_off and total_nnz are set; "
                  "keys and counts are unspecified)", who, (long long)*total_nnz, (long long)cap);
        return FC_ERR_RANGE;
    }
    return FC_OK;
}
