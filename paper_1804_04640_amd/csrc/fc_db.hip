// Device-resident database: state columns, per-state bit-vectors, marginals.
//
// The database of Section 2 is held column-major (as the Radix strategy of
// Section 3.3 wants), one uint8 per state, each column padded to whole
// 4096-row tiles.  Per-state bitmaps of Section 3.2 are stored as 64-bit
// words, one row of words per (variable, state).  Per-variable marginal
// counts (the precomputed first partition level of Section 3.3) and
// entropies (the Bitmap traversal order of Section 3.2) are computed once.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "fc_internal.h"

namespace fc {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

void clear_error() { g_err.clear(); }

bool is_device_ptr(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

__global__ void k_fill_zero_i32(int32_t *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0;
}

hipError_t fill_zero_i32(int32_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_zero_i32, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

// ------------------------------------------------------------ staging pool
static std::mutex g_stage_mu;
static std::vector<Staging *> g_stage_free;

static size_t g_stage_count = 0;
constexpr size_t kStageMax = 12;

Staging *staging_acquire(size_t bytes) {
    // Prefer the smallest free buffer whose last copy has completed and that
    // is large enough, then a new buffer (up to kStageMax), then the largest
    // completed one, which must grow (pinning memory is slow: buffers are
    // resized only when the pool is full, and small requests never take the
    // large buffers), and only then wait for the oldest: the host can plan
    // ahead of the device.
    Staging *st = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        int fit = -1, largest = -1;
        for (size_t i = 0; i < g_stage_free.size(); ++i) {
            Staging *c = g_stage_free[i];
            const bool idle = !c->done || hipEventQuery(c->done) == hipSuccess;
            if (!idle) continue;
            if (c->cap >= bytes && (fit < 0 || c->cap < g_stage_free[(size_t)fit]->cap))
                fit = (int)i;
            if (largest < 0 || c->cap > g_stage_free[(size_t)largest]->cap) largest = (int)i;
        }
        int pick = fit;
        if (pick < 0 && g_stage_count >= kStageMax) pick = largest;
        if (pick < 0 && g_stage_count >= kStageMax && !g_stage_free.empty()) pick = 0;
        if (pick >= 0) {
            st = g_stage_free[(size_t)pick];
            g_stage_free.erase(g_stage_free.begin() + pick);
        } else {
            ++g_stage_count;
        }
    }
    (void)hipGetLastError();  // hipEventQuery reports "not ready" as an error code
    if (!st) st = new (std::nothrow) Staging();
    if (!st) return nullptr;
    if (st->done) (void)hipEventSynchronize(st->done);  // previous copy out of it
    if (st->cap < bytes) {
        if (st->host) (void)hipHostFree(st->host);
        st->host = nullptr;
        st->cap = 0;
        size_t cap = bytes < (1u << 20) ? (1u << 20) : bytes + bytes / 4;
        if (hipHostMalloc(&st->host, cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            st->host = nullptr;
            delete st;
            return nullptr;
        }
        st->cap = cap;
    }
    if (!st->done && hipEventCreateWithFlags(&st->done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        st->done = nullptr;
    }
    return st;
}

void staging_release(Staging *st, hipStream_t s) {
    if (!st) return;
    if (st->done) (void)hipEventRecord(st->done, s);
    std::lock_guard<std::mutex> lk(g_stage_mu);
    g_stage_free.push_back(st);
}

// ------------------------------------------------------- device workspaces
constexpr size_t kWorkspaceMax = 4;

Workspace *workspace_acquire(fc_db *db, size_t bytes, hipStream_t s) {
    // The smallest idle workspace that is large enough, else a new one (up to
    // kWorkspaceMax), else the largest idle one grown, else a new one beyond
    // the limit (calls never wait for each other on the host).
    Workspace *w = nullptr;
    {
        std::lock_guard<std::mutex> lk(db->ws_mu);
        int fit = -1, largest = -1;
        for (size_t i = 0; i < db->ws_free.size(); ++i) {
            const Workspace *c = db->ws_free[i];
            if (c->cap >= bytes && (fit < 0 || c->cap < db->ws_free[(size_t)fit]->cap))
                fit = (int)i;
            if (largest < 0 || c->cap > db->ws_free[(size_t)largest]->cap) largest = (int)i;
        }
        int pick = fit;
        if (pick < 0 && db->ws_count >= kWorkspaceMax) pick = largest;
        if (pick >= 0) {
            w = db->ws_free[(size_t)pick];
            db->ws_free.erase(db->ws_free.begin() + pick);
        } else {
            ++db->ws_count;
        }
    }
    if (!w) w = new (std::nothrow) Workspace();
    if (!w) return nullptr;
    if (w->cap < bytes) {
        if (w->p) {
            if (w->done) (void)hipEventSynchronize(w->done);
            (void)hipFree(w->p);
            {
                std::lock_guard<std::mutex> lk(db->ws_mu);
                db->device_bytes -= (int64_t)w->cap;
            }
            w->p = nullptr;
            w->cap = 0;
        }
        const size_t cap = bytes + bytes / 8;
        if (hipMalloc(&w->p, cap) != hipSuccess) {
            (void)hipGetLastError();
            w->p = nullptr;
            if (w->done) (void)hipEventDestroy(w->done);
            delete w;
            std::lock_guard<std::mutex> lk(db->ws_mu);
            --db->ws_count;
            return nullptr;
        }
        w->cap = cap;
        std::lock_guard<std::mutex> lk(db->ws_mu);
        db->device_bytes += (int64_t)cap;
    }
    if (!w->done && hipEventCreateWithFlags(&w->done, hipEventDisableTiming) != hipSuccess) {
        // without its event a workspace cannot be handed over in stream order
        (void)hipGetLastError();
        w->done = nullptr;
        (void)hipFree(w->p);
        std::lock_guard<std::mutex> lk(db->ws_mu);
        db->device_bytes -= (int64_t)w->cap;
        delete w;
        --db->ws_count;
        return nullptr;
    }
    if (hipStreamWaitEvent(s, w->done, 0) != hipSuccess) {
        // back to the idle list untouched: its event still marks the last use
        (void)hipGetLastError();
        std::lock_guard<std::mutex> lk(db->ws_mu);
        db->ws_free.push_back(w);
        return nullptr;
    }
    return w;
}

void workspace_release(fc_db *db, Workspace *w, hipStream_t s) {
    if (!w) return;
    if (w->done) (void)hipEventRecord(w->done, s);
    std::lock_guard<std::mutex> lk(db->ws_mu);
    db->ws_free.push_back(w);
}

// ------------------------------------------------------------ kernels
// Row-major [m][n] -> column-major [n][pitch] through an LDS tile (rows
// [m, pitch) of the destination receive state 0).
__global__ void k_transpose(const uint8_t *__restrict__ rm, int64_t m, int32_t n,
                            uint8_t *__restrict__ cols, int64_t pitch) {
    __shared__ uint8_t tile[64][65];
    int64_t p0 = (int64_t)blockIdx.x * 64;
    int32_t v0 = blockIdx.y * 64;
    int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
    for (int r = ty; r < 64; r += 4) {
        int64_t p = p0 + r;
        int32_t v = v0 + tx;
        tile[r][tx] = (p < m && v < n) ? rm[p * n + v] : 0;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        int32_t v = v0 + r;
        int64_t p = p0 + tx;
        if (v < n && p < pitch) cols[(int64_t)v * pitch + p] = tile[tx][r];
    }
}

// Checks every state against its arity and counts the states of each
// variable (the marginals).  One workgroup per (variable, row slab).
__global__ void k_check_marg(const uint8_t *__restrict__ cols, int64_t m, int64_t pitch,
                             const uint8_t *__restrict__ arity, const int32_t *__restrict__ soff,
                             int32_t *__restrict__ marg, int32_t *__restrict__ bad) {
    __shared__ int32_t h[256];
    int32_t v = blockIdx.y;
    int r = arity[v];
    for (int i = threadIdx.x; i < 256; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const uint8_t *col = cols + (int64_t)v * pitch;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int nbad = 0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += stride) {
        int s = col[p];
        if (s >= r) ++nbad;
        atomicAdd(&h[s], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < r; i += blockDim.x)
        if (h[i]) atomicAdd(&marg[soff[v] + i], h[i]);
    if (nbad) atomicAdd(bad, nbad);
}

// 4-bit copy of the columns for databases whose arities are all at most 16:
// byte b of a column holds instance 2b in its low and 2b + 1 in its high
// nibble.  Each thread packs 8 instances (two input words -> one word) of
// the word range [d_lo, d_hi) of every column.
__global__ void k_pack_nib(const uint8_t *__restrict__ cols, int64_t pitch, int32_t n,
                           int64_t d_lo, int64_t d_hi, uint8_t *__restrict__ nib) {
    const int64_t per = d_hi - d_lo;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per * n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = (int32_t)(i / per);
        const int64_t d = d_lo + i % per;
        const uint2 x = *reinterpret_cast<const uint2 *>(cols + (int64_t)v * pitch + 8 * d);
        const uint32_t even = __builtin_amdgcn_perm(x.y, x.x, 0x06040200u);  // instances 0,2,4,6
        const uint32_t odd = __builtin_amdgcn_perm(x.y, x.x, 0x07050301u);   // instances 1,3,5,7
        reinterpret_cast<uint32_t *>(nib + (int64_t)v * (pitch / 2))[d] = even | (odd << 4);
    }
}

static hipError_t pack_nib(fc_db *db, int64_t d_lo, int64_t d_hi, hipStream_t s) {
    if (!db->d_nib || d_hi <= d_lo) return hipSuccess;
    const int64_t total = (d_hi - d_lo) * db->n;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_pack_nib, dim3((unsigned)blocks), dim3(256), 0, s, db->d_cols, db->pitch,
                       db->n, d_lo, d_hi, db->d_nib);
    return hipGetLastError();
}

// Per-state bit-vectors: bit (p mod 64) of word p/64 of row (v, s) is set when
// instance p of variable v is in state s.  One wave per 64-row word; padding
// rows (p >= m) contribute no bits.
__global__ void k_bitvectors(const uint8_t *__restrict__ cols, int64_t m, int64_t pitch,
                             int64_t wpitch, int64_t w_lo, int64_t w_hi,
                             const uint8_t *__restrict__ arity,
                             const int32_t *__restrict__ soff, uint64_t *__restrict__ bits) {
    int32_t v = blockIdx.y;
    int lane = threadIdx.x & 63;
    int64_t w = w_lo + (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (w >= w_hi) return;
    int64_t p = w * 64 + lane;
    int s = (p < m) ? cols[(int64_t)v * pitch + p] : 255;
    int r = arity[v];
    uint64_t *row = bits + (int64_t)soff[v] * wpitch + w;
    for (int st = 0; st < r; ++st) {
        uint64_t b = __ballot(s == st);
        if (lane == (st & 63)) row[(int64_t)st * wpitch] = b;
    }
}

}  // namespace fc

using namespace fc;

extern "C" const char *fc_last_error(void) { return g_err.c_str(); }

extern "C" void fc_db_destroy(fc_db *db) {
    if (!db) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(db->device);
    (void)hipDeviceSynchronize();
    if (db->d_cols) (void)hipFree(db->d_cols);
    if (db->d_nib) (void)hipFree(db->d_nib);
    if (db->d_bits) (void)hipFree(db->d_bits);
    if (db->d_arity) (void)hipFree(db->d_arity);
    if (db->d_soff) (void)hipFree(db->d_soff);
    if (db->d_marg) (void)hipFree(db->d_marg);
    for (Workspace *w : db->ws_free) {
        if (w->p) (void)hipFree(w->p);
        if (w->done) (void)hipEventDestroy(w->done);
        delete w;
    }
    (void)hipSetDevice(cur);
    delete db;
}

namespace {
struct DbGuard {
    fc_db *db;
    ~DbGuard() {
        if (db) fc_db_destroy(db);
    }
};
}  // namespace

static int db_alloc(void **p, size_t bytes, fc_db *db) {
    hipError_t e = hipMalloc(p, bytes ? bytes : 16);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error("device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        return FC_ERR_NOMEM;
    }
    db->device_bytes += (int64_t)bytes;
    return FC_OK;
}

extern "C" int fc_db_create(const uint8_t *data, int64_t m, int32_t n, const uint8_t *arity,
                            int32_t layout, uint32_t flags, void *stream, fc_db **out) {
    clear_error();
    if (!out) {
        set_error("fc_db_create: out is NULL");
        return FC_ERR_INVALID;
    }
    *out = nullptr;
    if (n < 1 || m < 0 || !arity || (m > 0 && !data)) {
        set_error("fc_db_create: need n >= 1, m >= 0, arity and data (n=%d m=%lld)", n,
                  (long long)m);
        return FC_ERR_INVALID;
    }
    if (m >= (int64_t(1) << 31)) {
        set_error("fc_db_create: m=%lld does not fit int32 counts", (long long)m);
        return FC_ERR_RANGE;
    }
    if (layout != FC_COL_MAJOR && layout != FC_ROW_MAJOR) {
        set_error("fc_db_create: unknown layout %d", layout);
        return FC_ERR_INVALID;
    }
    for (int32_t v = 0; v < n; ++v)
        if (arity[v] == 0) {
            set_error("fc_db_create: variable %d has arity 0", v);
            return FC_ERR_INVALID;
        }
    hipStream_t s = (hipStream_t)stream;
    fc_db *db = new (std::nothrow) fc_db();
    if (!db) {
        set_error("fc_db_create: host allocation failed");
        return FC_ERR_NOMEM;
    }
    DbGuard guard{db};
    FC_HIP(hipGetDevice(&db->device));
    FC_HIP(hipDeviceGetAttribute(&db->cu_count, hipDeviceAttributeMultiprocessorCount, db->device));
    {
        // Per-call scratch (tables, plans) comes from the device's default
        // stream-ordered pool; keep freed blocks cached in it instead of
        // returning them at every synchronisation, so that steady batches
        // reuse memory instead of mapping it anew.
        hipMemPool_t pool = nullptr;
        if (hipDeviceGetDefaultMemPool(&pool, db->device) == hipSuccess && pool) {
            uint64_t keep = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        }
        (void)hipGetLastError();
    }
    db->m = m;
    db->n = n;
    db->m_pad = ((m + kTileRows - 1) / kTileRows) * kTileRows;
    if (db->m_pad == 0) db->m_pad = kTileRows;
    db->words = db->m_pad / 64;
    db->pitch = db->m_pad;
    db->arity.assign(arity, arity + n);
    db->state_off.resize((size_t)n + 1);
    db->state_off[0] = 0;
    for (int32_t v = 0; v < n; ++v) db->state_off[v + 1] = db->state_off[v] + arity[v];
    const int32_t sum_r = db->state_off[n];

    int rc;
    if ((rc = db_alloc((void **)&db->d_cols, (size_t)n * (size_t)db->pitch, db))) return rc;
    if ((rc = db_alloc((void **)&db->d_arity, (size_t)n, db))) return rc;
    if ((rc = db_alloc((void **)&db->d_soff, sizeof(int32_t) * ((size_t)n + 1), db))) return rc;
    if ((rc = db_alloc((void **)&db->d_marg, sizeof(int32_t) * (size_t)sum_r, db))) return rc;
    FC_HIP(hipMemcpyAsync(db->d_arity, arity, (size_t)n, hipMemcpyHostToDevice, s));
    FC_HIP(hipMemcpyAsync(db->d_soff, db->state_off.data(), sizeof(int32_t) * ((size_t)n + 1),
                          hipMemcpyHostToDevice, s));
    FC_HIP(fill_zero_i32(db->d_marg, sum_r, s));
    // padding rows hold state 0 (removed from every count arithmetically)
    FC_HIP(fill_zero_i32((int32_t *)db->d_cols, (int64_t)n * db->pitch / 4, s));

    const bool on_dev = (flags & FC_DB_DATA_ON_DEVICE) != 0;
    if (m > 0) {
        if (layout == FC_COL_MAJOR) {
            FC_HIP(hipMemcpy2DAsync(db->d_cols, (size_t)db->pitch, data, (size_t)m, (size_t)m,
                                    (size_t)n,
                                    on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        } else {
            const uint8_t *src = data;
            DevBuf tmp;
            if (!on_dev) {
                FC_HIP(tmp.alloc((size_t)m * (size_t)n, s));
                FC_HIP(hipMemcpyAsync(tmp.p, data, (size_t)m * (size_t)n, hipMemcpyHostToDevice,
                                      s));
                src = (const uint8_t *)tmp.p;
            }
            dim3 grid((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64));
            hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, s, src, m, n, db->d_cols,
                               db->pitch);
            FC_HIP(hipGetLastError());
            FC_HIP(hipStreamSynchronize(s));  // tmp is freed on s after this
        }
    }
    // validation + marginals
    DevBuf bad;
    FC_HIP(bad.alloc(sizeof(int32_t), s));
    FC_HIP(fill_zero_i32((int32_t *)bad.p, 1, s));
    if (m > 0) {
        int64_t slabs = (m + 65535) / 65536;
        if (slabs > 64) slabs = 64;
        hipLaunchKernelGGL(k_check_marg, dim3((unsigned)slabs, (unsigned)n), dim3(256), 0, s,
                           db->d_cols, m, db->pitch, db->d_arity, db->d_soff, db->d_marg,
                           (int32_t *)bad.p);
        FC_HIP(hipGetLastError());
    }
    int32_t nbad = 0;
    std::vector<int32_t> marg32((size_t)sum_r);
    FC_HIP(hipMemcpyAsync(&nbad, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FC_HIP(hipMemcpyAsync(marg32.data(), db->d_marg, sizeof(int32_t) * (size_t)sum_r,
                          hipMemcpyDeviceToHost, s));
    FC_HIP(hipStreamSynchronize(s));
    if (nbad) {
        set_error("fc_db_create: %d states are not below their variable's arity "
                  "(the database must be complete)", nbad);
        return FC_ERR_INVALID;
    }
    db->marg.assign(marg32.begin(), marg32.end());
    db->entropy.assign((size_t)n, 0.0f);
    for (int32_t v = 0; v < n; ++v) {
        double h = 0.0;
        for (int st = 0; st < arity[v] && m > 0; ++st) {
            double pr = (double)db->marg[db->state_off[v] + st] / (double)m;
            if (pr > 0) h -= pr * std::log2(pr);
        }
        db->entropy[v] = (float)h;
    }
    bool small_arity = true;
    for (int32_t v = 0; v < n; ++v) small_arity = small_arity && arity[v] <= 16;
    if (small_arity) {
        if ((rc = db_alloc((void **)&db->d_nib, (size_t)n * (size_t)(db->pitch / 2), db)))
            return rc;
        FC_HIP(pack_nib(db, 0, db->m_pad / 8, s));
    }
    if (flags & FC_DB_BITVECTORS) {
        size_t bytes = sizeof(uint64_t) * (size_t)sum_r * (size_t)(db->pitch / 64);
        if ((rc = db_alloc((void **)&db->d_bits, bytes, db))) return rc;
        dim3 grid((unsigned)((db->words + 3) / 4), (unsigned)n);
        hipLaunchKernelGGL(k_bitvectors, grid, dim3(256), 0, s, db->d_cols, m, db->pitch,
                           db->pitch / 64, (int64_t)0, db->words, db->d_arity, db->d_soff,
                           db->d_bits);
        FC_HIP(hipGetLastError());
        FC_HIP(hipStreamSynchronize(s));
    }
    *out = db;
    guard.db = nullptr;
    return FC_OK;
}

extern "C" int fc_db_trim(fc_db *db) {
    clear_error();
    if (!db) {
        set_error("fc_db_trim: NULL database handle");
        return FC_ERR_INVALID;
    }
    std::vector<Workspace *> idle;
    {
        std::lock_guard<std::mutex> lk(db->ws_mu);
        idle.swap(db->ws_free);
        db->ws_count -= idle.size();
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    FC_HIP(hipSetDevice(db->device));
    for (Workspace *w : idle) {
        if (w->done) (void)hipEventSynchronize(w->done);  // its last user has finished
        if (w->p) (void)hipFree(w->p);
        if (w->done) (void)hipEventDestroy(w->done);
        {
            std::lock_guard<std::mutex> lk(db->ws_mu);
            db->device_bytes -= (int64_t)w->cap;
        }
        delete w;
    }
    (void)hipSetDevice(cur);
    return FC_OK;
}

extern "C" int fc_db_info(const fc_db *db, int64_t *m, int32_t *n, int32_t *has_bits,
                          int64_t *device_bytes) {
    if (!db) {
        set_error("fc_db_info: NULL handle");
        return FC_ERR_INVALID;
    }
    if (m) *m = db->m;
    if (n) *n = db->n;
    if (has_bits) *has_bits = db->d_bits != nullptr;
    if (device_bytes) *device_bytes = db->device_bytes;
    return FC_OK;
}

extern "C" int fc_db_marginals(const fc_db *db, int64_t *counts, float *entropy_bits) {
    if (!db) {
        set_error("fc_db_marginals: NULL handle");
        return FC_ERR_INVALID;
    }
    if (counts) std::memcpy(counts, db->marg.data(), sizeof(int64_t) * db->marg.size());
    if (entropy_bits) std::memcpy(entropy_bits, db->entropy.data(), sizeof(float) * db->n);
    return FC_OK;
}

extern "C" int fc_db_append(fc_db *db, const uint8_t *data, int64_t m_new, int32_t layout,
                            uint32_t flags, void *stream) {
    clear_error();
    if (!db || m_new < 0 || (m_new > 0 && !data)) {
        set_error("fc_db_append: need a database, m_new >= 0 and data");
        return FC_ERR_INVALID;
    }
    if (layout != FC_COL_MAJOR && layout != FC_ROW_MAJOR) {
        set_error("fc_db_append: unknown layout %d", layout);
        return FC_ERR_INVALID;
    }
    if (m_new == 0) return FC_OK;
    const int64_t m_old = db->m, m = m_old + m_new;
    if (m >= (int64_t(1) << 31)) {
        set_error("fc_db_append: %lld instances do not fit int32 counts", (long long)m);
        return FC_ERR_RANGE;
    }
    hipStream_t s = (hipStream_t)stream;
    FC_HIP(hipSetDevice(db->device));
    const int32_t n = db->n, sum_r = db->state_off[n];
    const bool on_dev = (flags & FC_DB_DATA_ON_DEVICE) != 0;
    // 1. the new instances, column-major [n][m_new], validated and counted
    DevBuf tmp, raw, bad, cnt;
    FC_HIP(tmp.alloc((size_t)n * (size_t)m_new, s));
    if (layout == FC_COL_MAJOR) {
        FC_HIP(hipMemcpyAsync(tmp.p, data, (size_t)n * (size_t)m_new,
                              on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    } else {
        const uint8_t *src = data;
        if (!on_dev) {
            FC_HIP(raw.alloc((size_t)n * (size_t)m_new, s));
            FC_HIP(hipMemcpyAsync(raw.p, data, (size_t)n * (size_t)m_new, hipMemcpyHostToDevice, s));
            src = (const uint8_t *)raw.p;
        }
        dim3 grid((unsigned)((m_new + 63) / 64), (unsigned)((n + 63) / 64));
        hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, s, src, m_new, n, (uint8_t *)tmp.p,
                           m_new);
        FC_HIP(hipGetLastError());
    }
    FC_HIP(bad.alloc(sizeof(int32_t), s));
    FC_HIP(cnt.alloc(sizeof(int32_t) * (size_t)sum_r, s));
    FC_HIP(fill_zero_i32((int32_t *)bad.p, 1, s));
    FC_HIP(fill_zero_i32((int32_t *)cnt.p, sum_r, s));
    {
        int64_t slabs = std::min<int64_t>((m_new + 65535) / 65536, 64);
        hipLaunchKernelGGL(k_check_marg, dim3((unsigned)slabs, (unsigned)n), dim3(256), 0, s,
                           (const uint8_t *)tmp.p, m_new, m_new, db->d_arity, db->d_soff,
                           (int32_t *)cnt.p, (int32_t *)bad.p);
        FC_HIP(hipGetLastError());
    }
    int32_t nbad = 0;
    std::vector<int32_t> add((size_t)sum_r);
    FC_HIP(hipMemcpyAsync(&nbad, bad.p, sizeof nbad, hipMemcpyDeviceToHost, s));
    FC_HIP(hipMemcpyAsync(add.data(), cnt.p, sizeof(int32_t) * (size_t)sum_r,
                          hipMemcpyDeviceToHost, s));
    FC_HIP(hipStreamSynchronize(s));
    if (nbad) {
        set_error("fc_db_append: %d new states are not below their variable's arity "
                  "(nothing was appended)", nbad);
        return FC_ERR_INVALID;
    }
    // 2. the scanned extent grows to the new tile count; the allocation (the
    //    column pitch) only when the extent outgrows it, then geometrically
    FC_HIP(hipDeviceSynchronize());  // no launch may still read the old buffers
    const int64_t m_pad = ((m + kTileRows - 1) / kTileRows) * kTileRows;
    const bool regrown = m_pad > db->pitch;
    if (regrown) {
        const int64_t grown = ((db->pitch + db->pitch / 2 + kTileRows - 1) / kTileRows) * kTileRows;
        const int64_t pitch = std::min<int64_t>(std::max(m_pad, grown), int64_t(1) << 31);
        const int64_t wpitch = pitch / 64;
        uint8_t *cols = nullptr;
        if (hipMalloc(&cols, (size_t)n * (size_t)pitch) != hipSuccess) {
            (void)hipGetLastError();
            set_error("fc_db_append: device allocation failed");
            return FC_ERR_NOMEM;
        }
        uint64_t *bits = nullptr;
        if (db->d_bits &&
            hipMalloc(&bits, sizeof(uint64_t) * (size_t)sum_r * (size_t)wpitch) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(cols);
            set_error("fc_db_append: device allocation failed");
            return FC_ERR_NOMEM;
        }
        uint8_t *nib = nullptr;
        if (db->d_nib && hipMalloc(&nib, (size_t)n * (size_t)(pitch / 2)) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(cols);
            if (bits) (void)hipFree(bits);
            set_error("fc_db_append: device allocation failed");
            return FC_ERR_NOMEM;
        }
        // every row past m holds state 0 and no bit, in all three stores
        FC_HIP(fill_zero_i32((int32_t *)cols, (int64_t)n * pitch / 4, s));
        FC_HIP(hipMemcpy2DAsync(cols, (size_t)pitch, db->d_cols, (size_t)db->pitch,
                                (size_t)db->m_pad, (size_t)n, hipMemcpyDeviceToDevice, s));
        if (nib) {
            FC_HIP(fill_zero_i32((int32_t *)nib, (int64_t)n * pitch / 8, s));
            FC_HIP(hipMemcpy2DAsync(nib, (size_t)(pitch / 2), db->d_nib, (size_t)(db->pitch / 2),
                                    (size_t)(db->m_pad / 2), (size_t)n, hipMemcpyDeviceToDevice,
                                    s));
        }
        if (bits) {
            FC_HIP(fill_zero_i32((int32_t *)bits, 2 * (int64_t)sum_r * wpitch, s));
            FC_HIP(hipMemcpy2DAsync(bits, sizeof(uint64_t) * (size_t)wpitch, db->d_bits,
                                    sizeof(uint64_t) * (size_t)(db->pitch / 64),
                                    sizeof(uint64_t) * (size_t)db->words, (size_t)sum_r,
                                    hipMemcpyDeviceToDevice, s));
        }
        FC_HIP(hipStreamSynchronize(s));
        (void)hipFree(db->d_cols);
        db->device_bytes += (int64_t)n * (pitch - db->pitch);
        db->d_cols = cols;
        if (nib) {
            (void)hipFree(db->d_nib);
            db->device_bytes += (int64_t)n * (pitch - db->pitch) / 2;
            db->d_nib = nib;
        }
        if (bits) {
            (void)hipFree(db->d_bits);
            db->device_bytes += (int64_t)sizeof(uint64_t) * sum_r * (wpitch - db->pitch / 64);
            db->d_bits = bits;
        }
        db->pitch = pitch;
    }
    db->m_pad = m_pad;
    db->words = m_pad / 64;
    // 3. the new instances into the columns, then the packed words and the
    //    bit-vector words they touch (rows past m stay state 0 / no bit)
    FC_HIP(hipMemcpy2DAsync(db->d_cols + m_old, (size_t)db->pitch, tmp.p, (size_t)m_new,
                            (size_t)m_new, (size_t)n, hipMemcpyDeviceToDevice, s));
    FC_HIP(pack_nib(db, m_old / 8, (m + 7) / 8, s));
    if (db->d_bits) {
        const int64_t w_lo = m_old / 64, w_hi = (m + 63) / 64;
        dim3 grid((unsigned)((w_hi - w_lo + 3) / 4), (unsigned)n);
        hipLaunchKernelGGL(k_bitvectors, grid, dim3(256), 0, s, db->d_cols, m, db->pitch,
                           db->pitch / 64, w_lo, w_hi, db->d_arity, db->d_soff, db->d_bits);
        FC_HIP(hipGetLastError());
    }
    std::vector<int32_t> marg32((size_t)sum_r);
    for (int32_t i = 0; i < sum_r; ++i) {
        db->marg[(size_t)i] += add[(size_t)i];
        marg32[(size_t)i] = (int32_t)db->marg[(size_t)i];
    }
    FC_HIP(hipMemcpyAsync(db->d_marg, marg32.data(), sizeof(int32_t) * (size_t)sum_r,
                          hipMemcpyHostToDevice, s));
    FC_HIP(hipStreamSynchronize(s));
    db->m = m;
    for (int32_t v = 0; v < n; ++v) {
        double h = 0.0;
        for (int st = 0; st < db->arity[v]; ++st) {
            const double pr = (double)db->marg[db->state_off[v] + st] / (double)m;
            if (pr > 0) h -= pr * std::log2(pr);
        }
        db->entropy[v] = (float)h;
    }
    db->epoch += 1;
    return FC_OK;
}
