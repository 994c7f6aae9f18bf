// Internal declarations of the fastcount library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <mutex>
#include <string>
#include <functional>
#include <vector>

#include "fastcount.h"

namespace fc {

// Rows are stored in tiles of this many instances; every column is padded to
// a whole number of tiles with state 0 and the padding is removed from the
// counts arithmetically (it always lands in key 0).
constexpr int64_t kTileRows = 4096;
constexpr int kWaves = 4;            // waves per counting workgroup
constexpr int kBlock = 64 * kWaves;  // threads per counting workgroup
constexpr int kXcds = 8;             // MI355X: 8 XCDs, workgroups round-robin
constexpr int kLdsBytesMax = 160 * 1024;

// Work descriptor of one counting unit (one query, or one key window of a
// partitioned query).  64 bytes, read once per workgroup.
struct alignas(16) QDesc {
    int64_t table_off;  // cell offset of the query's table
    int32_t var[FC_MAX_VARS];
    int32_t cells;      // cells of the whole table
    int32_t k;          // variables in the query
    int32_t win_base;   // first key of the window (0 when not partitioned); for a
                        // Bitmap descriptor, its tree-walk order (3 bits per level)
    int32_t win_cells;  // keys in the window
    int32_t qid;        // query index in the caller's batch
    int32_t tiles;      // kTileRows tiles scanned: the padded extent m_pad / kTileRows
};
static_assert(sizeof(QDesc) == 64, "QDesc must be 64 bytes");

struct Tuning {
    int64_t chunk_rows = 131072;        // histogram rows per workgroup (at least)
    int64_t bitmap_chunk_rows = 65536;  // bitmap rows per workgroup (at least)
    int bitmap_words = 2;               // 64-row words per thread per tree walk
    int persistent_max_queries = 256;   // small batches: one persistent launch
    int packed_columns = 1;             // histograms read the 4-bit columns when present
    int bitmap_order = 1;               // 1: bitmap trees walk variables by ascending entropy
    int derive = 1;                     // 1: automatic plans sum tables out of supersets
    int one_pass = 1;                   // 1: one-pass partition for tables beyond LDS
    int row_sweep = 1;                  // 1: histogram workgroups sweep their chunks in step
    // bitmap_cells[k-1][b]: bitmap for k variables and <= 2^(b+2) cells
    uint8_t bitmap_cells[FC_MAX_VARS][6] = {};
    Tuning() {
        for (int k = 0; k < FC_MAX_VARS; ++k)
            for (int b = 0; b < 3; ++b) bitmap_cells[k][b] = 1;  // up to 16 cells
    }
    bool bitmap_for(int k, int64_t cells) const {
        for (int b = 0; b < 6; ++b)
            if (cells <= (int64_t(4) << b)) return bitmap_cells[k - 1][b] != 0;
        return false;
    }
};

// Device workspace kept by a database handle between calls (large sort
// scratch whose allocation and release cost more host time than the work):
// handed from call to call in stream order through `done`.
struct Workspace {
    void *p = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;  // last use of the memory, on its caller's stream
};

}  // namespace fc

struct fc_db {
    int device = 0;
    int cu_count = 256;
    // m_pad: m rounded up to whole tiles, the extent every scan covers;
    // words = m_pad / 64.  pitch: rows allocated per column (a multiple of
    // kTileRows, >= m_pad; appends grow it geometrically), the stride of the
    // columns; the packed columns' stride is pitch / 2 bytes and the
    // bit-vectors' pitch / 64 words.  Rows in [m, pitch) hold state 0.
    int64_t m = 0, m_pad = 0, words = 0, pitch = 0;
    int32_t n = 0;
    std::vector<uint8_t> arity;      // n
    std::vector<int32_t> state_off;  // n+1, prefix sums of arities
    std::vector<int64_t> marg;       // sum of arities
    std::vector<float> entropy;      // n, bits
    uint8_t *d_cols = nullptr;       // [n][pitch] states
    uint8_t *d_nib = nullptr;        // [n][pitch/2] states, 4 bits each (all arities <= 16)
    uint64_t *d_bits = nullptr;      // [sum r][pitch/64] per-state bit-vectors
    uint8_t *d_arity = nullptr;      // [n]
    int32_t *d_soff = nullptr;       // [n+1]
    int32_t *d_marg = nullptr;       // [sum r]
    int64_t device_bytes = 0;
    uint64_t epoch = 0;              // bumped by every append
    fc::Tuning tune;
    std::mutex ws_mu;                       // guards the workspace list
    std::vector<fc::Workspace *> ws_free;   // idle workspaces
    size_t ws_count = 0;                    // workspaces in existence
};

namespace fc {

void set_error(const char *fmt, ...);
void clear_error();

#define FC_HIP(call)                                                        \
    do {                                                                    \
        hipError_t e_ = (call);                                             \
        if (e_ != hipSuccess) {                                             \
            ::fc::set_error("%s: %s", #call, hipGetErrorString(e_));        \
            return FC_ERR_DEVICE;                                           \
        }                                                                   \
    } while (0)

// Device pointer test (torch tensors, hipMalloc); host memory otherwise.
bool is_device_ptr(const void *p);

// Zero `n` int32 values with a kernel (graph-capture safe, no memset node).
hipError_t fill_zero_i32(int32_t *p, int64_t n, hipStream_t s);

// Stream-ordered scratch owned by one call.
struct DevBuf {
    void *p = nullptr;
    hipStream_t s = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() {
        if (p) (void)hipFreeAsync(p, s);
    }
    hipError_t alloc(size_t bytes, hipStream_t st) {
        s = st;
        return hipMallocAsync(&p, bytes ? bytes : 16, st);
    }
};

// Pinned host staging buffers, reused across calls; one per concurrent call.
struct Staging {
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;  // last H2D copy out of this buffer
};
Staging *staging_acquire(size_t bytes);
void staging_release(Staging *st, hipStream_t s);

// A workspace of at least `bytes` for work enqueued on `s` (which is made to
// wait for the workspace's previous user); nullptr when device memory is
// exhausted.  Released with workspace_release after the last enqueue.
Workspace *workspace_acquire(fc_db *db, size_t bytes, hipStream_t s);
void workspace_release(fc_db *db, Workspace *w, hipStream_t s);

// Launch profiling: RAII bracket of one launch with events on its stream.
bool profiling_on();
void set_capturing(bool on);  // this thread is recording a graph: no event brackets
// Device time of this thread's bracketed launches: between begin and end,
// every launch the thread brackets adds its event-timed duration (ms) to
// *sink; end waits for them.  Independent of the per-kernel aggregates.
void device_time_begin(double *sink);
void device_time_end();
struct ProfScope {
    int slot = -1;
    ProfScope(const char *name, hipStream_t s, double alg_bytes, double alg_ops);
    void end(hipStream_t s);
};

// Counts and reduces a batch (validated inside) into device scores
// [slot * nq + i], tables in stream-ordered scratch (fc_count.hip).
int count_reduce_device(fc_db *db, const int32_t *vars_flat, const int64_t *var_off, int64_t nq,
                        uint32_t reducers, double ess, float *scores, hipStream_t s);

// Gram of bit-vector rows (fc_pairs.hip): C[i][j] = Count(row i AND row j)
// for every i <= j of the np = rowidx entries (np a multiple of 128; -1 is
// an all-zero padding row), over all instances, on the matrix cores.  C
// (np x np int32, leading dimension ldc) must be zero on entry; entries
// below the diagonal are unspecified.  name/alg_bytes/alg_ops label the
// launch for profiling.
hipError_t launch_gram(const fc_db *db, const int32_t *rowidx, int32_t np, int32_t *C,
                       int64_t ldc, const char *name, double alg_bytes, double alg_ops,
                       hipStream_t s);

// Host fork-join (fc_pool.hip): f(0) on the calling thread, f(1) ..
// f(T - 1) on persistent workers; returns when all have returned.
void parallel_for(int T, const std::function<void(int)> &f);

// Sorted distinct keys and their counts (fc_msd.hip): keys[0, nk) (clobbered,
// as is alt[0, nk)) with only bits below end_bit set give uniq[0, *nruns)
// ascending and cnt[i] = occurrences of uniq[i]; *nruns is written on the
// device.  scratch: msd_scratch_bytes(nk, sizeof(K)) bytes.  With
// top_given, the 256 words at msd_top_hist(scratch, ...) already hold the
// histogram of the keys' top digit (bits [max(end_bit - 8, 0), end_bit)),
// which the caller took while forming the keys.  Everything is enqueued on
// s; the host does not wait.
size_t msd_scratch_bytes(int64_t nk, size_t key_bytes);
uint32_t *msd_top_hist(void *scratch, int64_t nk, size_t key_bytes);
template <typename K>
int msd_sort_rle(const fc_db *db, K *keys, K *alt, int64_t nk, unsigned end_bit, K *uniq,
                 uint32_t *cnt, uint32_t *nruns, void *scratch, bool top_given, hipStream_t s);

// Reducer launch (fc_reduce.hip).  descs: exactly one QDesc per query
// (device, any order); scores[slot * nq + qid].
hipError_t launch_reduce(const fc_db *db, const QDesc *descs, int64_t nd, int64_t nq,
                         const int32_t *tables, uint32_t reducers, double ess,
                         float *scores, float *err, hipStream_t s);

}  // namespace fc
