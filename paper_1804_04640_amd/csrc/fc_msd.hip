// Sorted distinct keys and their counts, for the sparse tables: an MSD
// partition of the keys by 8-bit digits from the top (Section 3.3's MSD
// radix order: each level splits a segment of keys by its next digit into
// 256 contiguous buckets), until a bucket holds at most kBigKeys keys or
// no digit is left; each such leaf is then sorted in registers (one
// thread), across one wave's lanes or in LDS by one workgroup, by the
// rank of each key among the keys it can be confused with, and
// run-length encoded.
//
// Every position p of the key array belongs to exactly one leaf, which
// writes, at its own positions, its runs (key, count) and a flag per
// position (1 where a run is stored).  One exclusive scan of the flags
// gives every run its place in the output, which is in key order because
// the partition keeps each bucket at its place in key order.
//
// Levels run on the device from lists the previous level appends to
// (segments of the next level, and three queues of leaves by size); the
// host enqueues every level without waiting, and a level without segments
// exits at once.
#include <algorithm>

#include "fc_internal.h"

namespace fc {
namespace {

constexpr int kMsdThreads = 256;
constexpr int kTileKeys = 4096;            // keys per partition workgroup (16 per thread)
constexpr int kLeafKeys = 1024;            // keys a leaf workgroup of kLeafThreads sorts in LDS
constexpr int kBigThreads = 1024;
constexpr int kBigKeys = 8192;             // keys a leaf workgroup of kBigThreads sorts in LDS
// bits such a leaf splits its keys by
template <typename K> constexpr int big_digit() { return sizeof(K) == 8 ? 10 : 11; }
constexpr int kTinyKeys = 16;              // leaves one thread sorts in registers
constexpr int kLeafThreads = 128;          // one workgroup per leaf of up to kLeafKeys keys
constexpr int kLeafDigit = 9;              // bits such a leaf splits its keys by
constexpr int kScanBlock = 4096;           // flags per scan workgroup

struct MSeg {
    int64_t off, len;
    int64_t tile0;  // first tile of this segment in the level's tile space
    int64_t pad;
};

struct MCtl {
    int32_t nseg[2];     // segments of the level (ping-pong by level parity)
    int64_t tiles[2];    // tiles of those segments
    uint32_t total;      // runs
    uint32_t nmid[3];    // leaves of the level queued for k_msd_small, k_msd_leaves (two sizes)
};

__device__ __forceinline__ uint32_t digit_of(uint64_t key, int lo, int width) {
    return (uint32_t)(key >> lo) & ((1u << width) - 1u);
}

// Segment of tile t: the last segment whose first tile is <= t.
__device__ __forceinline__ int32_t seg_of_tile(const MSeg *segs, int32_t n, int64_t t) {
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (segs[mid].tile0 <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The root segment; its digit counts (256 threads) start at zero, or are
// the histogram the caller took (top != nullptr).
__global__ void k_msd_init(MCtl *ctl, MSeg *segs0, uint32_t *counts0, const uint32_t *top,
                           int64_t nk) {
    counts0[threadIdx.x] = top ? top[threadIdx.x] : 0u;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        segs0[0].off = 0;
        segs0[0].len = nk;
        segs0[0].tile0 = 0;
        ctl->nseg[0] = 1;
        ctl->tiles[0] = (nk + kTileKeys - 1) / kTileKeys;
        ctl->nseg[1] = 0;
        ctl->tiles[1] = 0;
        ctl->total = 0;
        ctl->nmid[0] = ctl->nmid[1] = ctl->nmid[2] = 0;
    }
}

// Digit histogram of every tile of the level's segments into counts[s][d]
// (workgroups stride over the tiles).  Also clears the next level's segment
// count, which the split appends to.
template <typename K>
__global__ __launch_bounds__(kMsdThreads) void k_msd_hist(const K *__restrict__ keys,
                                                          const MSeg *__restrict__ segs,
                                                          MCtl *__restrict__ ctl, int cur,
                                                          int lo, int width,
                                                          uint32_t *__restrict__ counts) {
    __shared__ uint32_t h[256];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->nseg[cur ^ 1] = 0;
        ctl->tiles[cur ^ 1] = 0;
        ctl->nmid[0] = 0;
        ctl->nmid[1] = 0;
        ctl->nmid[2] = 0;
    }
    const int64_t nt = ctl->tiles[cur];
    const int32_t ns = ctl->nseg[cur];
    for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        const int32_t s = seg_of_tile(segs, ns, t);
        const MSeg g = segs[s];
        const int64_t a = g.off + (t - g.tile0) * kTileKeys;
        const int64_t b = min(g.off + g.len, a + (int64_t)kTileKeys);
        h[threadIdx.x] = 0u;
        __syncthreads();
        for (int64_t p = a + threadIdx.x; p < b; p += kMsdThreads)
            atomicAdd(&h[digit_of((uint64_t)keys[p], lo, width)], 1u);
        __syncthreads();
        const uint32_t c = h[threadIdx.x];
        if (c) atomicAdd(&counts[(int64_t)s * 256 + threadIdx.x], c);
        __syncthreads();
    }
}

// Per segment: bucket starts (exclusive scan of its digit counts), the
// scatter cursors, and the buckets that need another level, whose digit
// counts (next level's array) this workgroup clears.
__global__ __launch_bounds__(kMsdThreads) void k_msd_split(
    const MSeg *__restrict__ segs, MCtl *ctl, int cur, int lo, const uint32_t *__restrict__ counts,
    uint32_t *__restrict__ next_counts, int64_t *__restrict__ start, uint32_t *__restrict__ cursor,
    MSeg *__restrict__ next_segs) {
    __shared__ uint32_t sc[256];
    __shared__ int32_t made[256];
    __shared__ int32_t nmade;
    const int32_t ns = ctl->nseg[cur];
    const int d = threadIdx.x;
    for (int32_t s = blockIdx.x; s < ns; s += gridDim.x) {
        if (d == 0) nmade = 0;
        const uint32_t c = counts[(int64_t)s * 256 + d];
        sc[d] = c;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {  // inclusive scan
            const uint32_t v = d >= o ? sc[d - o] : 0u;
            __syncthreads();
            sc[d] += v;
            __syncthreads();
        }
        const int64_t st = segs[s].off + (int64_t)(sc[d] - c);
        start[(int64_t)s * 256 + d] = st;
        cursor[(int64_t)s * 256 + d] = (uint32_t)st;
        if (c > (uint32_t)kBigKeys && lo > 0) {
            const int32_t i = atomicAdd(&ctl->nseg[cur ^ 1], 1);
            next_segs[i].off = st;
            next_segs[i].len = c;
            next_segs[i].tile0 = 0;
            made[atomicAdd(&nmade, 1)] = i;
        }
        __syncthreads();
        for (int32_t j = 0; j < nmade; ++j) next_counts[(int64_t)made[j] * 256 + d] = 0u;
        __syncthreads();
    }
}

// First tiles of the next level's segments (one workgroup).
__global__ __launch_bounds__(1024) void k_msd_tiles(MSeg *segs, MCtl *ctl, int nxt) {
    __shared__ int64_t part[1024];
    const int32_t n = ctl->nseg[nxt];
    const int32_t per = (n + 1023) / 1024;
    const int32_t a = min(n, (int32_t)threadIdx.x * per), b = min(n, a + per);
    int64_t sum = 0;
    for (int32_t i = a; i < b; ++i) sum += (segs[i].len + kTileKeys - 1) / kTileKeys;
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int64_t v = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t t = part[threadIdx.x] - sum;
    for (int32_t i = a; i < b; ++i) {
        segs[i].tile0 = t;
        t += (segs[i].len + kTileKeys - 1) / kTileKeys;
    }
    if (threadIdx.x == 1023) ctl->tiles[nxt] = part[1023];
}

// Moves every key of the level's segments to its bucket (order within a
// bucket is free: the leaves sort it).  Workgroups stride over the tiles;
// a tile's keys are ranked per bucket in LDS and take one cursor atomic per
// bucket.  STAGE: they are staged in LDS in bucket order, and each bucket's
// keys leave as one contiguous run (neighbouring threads, neighbouring
// addresses); this pays below the first level, where a tile's keys spread
// over many buckets, and not at the first, where the top digit (mostly the
// query) sends a tile's keys to a few.
template <typename K, bool STAGE>
__global__ __launch_bounds__(kMsdThreads) void k_msd_scatter(const K *__restrict__ in,
                                                             K *__restrict__ out,
                                                             const MSeg *__restrict__ segs,
                                                             const MCtl *__restrict__ ctl, int cur,
                                                             int lo, int width,
                                                             uint32_t *__restrict__ cursor) {
    __shared__ uint32_t h[256], base[256], tstart[256];
    __shared__ uint32_t wsum[kMsdThreads / 64];
    __shared__ K stage[STAGE ? kTileKeys : 1];
    constexpr int E = kTileKeys / kMsdThreads;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t nt = ctl->tiles[cur];
    const int32_t ns = ctl->nseg[cur];
    for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        const int32_t s = seg_of_tile(segs, ns, t);
        const MSeg g = segs[s];
        const int64_t a = g.off + (t - g.tile0) * kTileKeys;
        const int64_t b = min(g.off + g.len, a + (int64_t)kTileKeys);
        h[threadIdx.x] = 0u;
        __syncthreads();
        K key[E];
        uint32_t rank[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t p = a + threadIdx.x + (int64_t)e * kMsdThreads;
            if (p < b) {
                key[e] = in[p];
                rank[e] = atomicAdd(&h[digit_of((uint64_t)key[e], lo, width)], 1u);
            }
        }
        __syncthreads();
        // the tile's bucket starts (exclusive scan of h, one bucket per
        // thread) and the buckets' places in the output
        const uint32_t c = h[threadIdx.x];
        uint32_t incl = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t x = __shfl_up(incl, o);
            if (lane >= o) incl += x;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        uint32_t before = 0;
#pragma unroll
        for (int w = 0; w < kMsdThreads / 64; ++w) before += w < wave ? wsum[w] : 0u;
        tstart[threadIdx.x] = before + incl - c;
        base[threadIdx.x] = c ? atomicAdd(&cursor[(int64_t)s * 256 + threadIdx.x], c) : 0u;
        __syncthreads();
        if (STAGE) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t p = a + threadIdx.x + (int64_t)e * kMsdThreads;
                if (p < b) stage[tstart[digit_of((uint64_t)key[e], lo, width)] + rank[e]] = key[e];
            }
            __syncthreads();
            const int32_t n = (int32_t)(b - a);
            for (int32_t j = threadIdx.x; j < n; j += kMsdThreads) {
                const K k = stage[j];
                const uint32_t d = digit_of((uint64_t)k, lo, width);
                out[base[d] + ((uint32_t)j - tstart[d])] = k;
            }
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t p = a + threadIdx.x + (int64_t)e * kMsdThreads;
                if (p < b) out[base[digit_of((uint64_t)key[e], lo, width)] + rank[e]] = key[e];
            }
        }
        __syncthreads();
    }
}

// Leaves.  Child (s, d) of a level's segment is a leaf when it is not
// empty and has at most kBigKeys keys or no bits left below the digit.
// Its keys lie at [start, start + len) of the level's output and agree above
// bit `bits`.  A leaf writes its runs (key, count) to rk/rc at start.. and
// sets flag[start + r] = 1 for each run r (the flags start at 0).
//
// One thread's leaf of 2..N keys at off: sorted in registers by an
// insertion network (padding with the largest key value sorts last), runs
// written where they go.
template <typename K, int N>
__device__ __forceinline__ void tiny_leaf(const K *__restrict__ keys, int64_t off, uint32_t len,
                                          K *__restrict__ rk, uint32_t *__restrict__ rc,
                                          uint8_t *__restrict__ flag) {
    K x[N];
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = i < (int)len ? keys[off + i] : ~(K)0;
#pragma unroll
    for (int i = 1; i < N; ++i)
#pragma unroll
        for (int j = i; j > 0; --j) {
            const K a = x[j - 1], b = x[j];
            x[j - 1] = a < b ? a : b;
            x[j] = a < b ? b : a;
        }
    K prev = x[0];
    uint32_t r = 0, cnt = 1;
#pragma unroll
    for (int i = 1; i < N; ++i) {
        if (i < (int)len) {
            if (x[i] == prev) {
                ++cnt;
            } else {
                rk[off + r] = prev;
                rc[off + r] = cnt;
                flag[off + r] = 1;
                ++r;
                cnt = 1;
                prev = x[i];
            }
        }
    }
    rk[off + r] = prev;
    rc[off + r] = cnt;
    flag[off + r] = 1;
}

// A queued leaf: its first position and its key count in one word.
constexpr int kLenBits = 16;  // kBigKeys < 2^kLenBits
__device__ __forceinline__ uint64_t leaf_entry(int64_t off, uint32_t len) {
    return ((uint64_t)off << kLenBits) | len;
}

// Every child of the level's segments, one thread each: children of one
// key value (or one key) and of at most kTinyKeys keys are finished here;
// leaves of 17..64 keys are queued for k_msd_small (front of `mid`), of
// 65..kLeafKeys keys for the workgroup leaves (back of `mid`), of up to
// kBigKeys keys for the large workgroup leaves (`bigq`), one atomic per
// wave and queue; larger children are segments of the next level.
__device__ __forceinline__ uint32_t wave_slots(bool want, uint32_t *counter) {
    const int lane = threadIdx.x & 63;
    const uint64_t m = __ballot(want);
    if (!m) return 0;
    const int first = __builtin_ctzll(m);
    uint32_t b0 = 0;
    if (lane == first) b0 = atomicAdd(counter, (uint32_t)__popcll(m));
    b0 = __shfl(b0, first);
    return b0 + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

template <typename K>
__global__ __launch_bounds__(kMsdThreads) void k_msd_tiny(
    const K *__restrict__ keys, MCtl *__restrict__ ctl, int cur, int lo,
    const uint32_t *__restrict__ counts, const int64_t *__restrict__ start, K *__restrict__ rk,
    uint32_t *__restrict__ rc, uint8_t *__restrict__ flag, uint64_t *__restrict__ mid,
    int64_t mid_cap, uint64_t *__restrict__ bigq) {
    const int64_t nc = (int64_t)ctl->nseg[cur] * 256;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nc; base += stride) {
        const int64_t c = base + threadIdx.x;
        const uint32_t len = c < nc ? counts[c] : 0u;
        const int64_t off = len ? start[c] : 0;
        const bool more_bits = lo > 0;
        const bool qs = more_bits && len > (uint32_t)kTinyKeys && len <= 64u;
        const bool qm = more_bits && len > 64u && len <= (uint32_t)kLeafKeys;
        const bool qb = more_bits && len > (uint32_t)kLeafKeys && len <= (uint32_t)kBigKeys;
        const uint32_t js = wave_slots(qs, &ctl->nmid[0]);
        const uint32_t jm = wave_slots(qm, &ctl->nmid[1]);
        const uint32_t jb = wave_slots(qb, &ctl->nmid[2]);
        if (qs) mid[js] = leaf_entry(off, len);
        if (qm) mid[mid_cap - 1 - (int64_t)jm] = leaf_entry(off, len);
        if (qb) bigq[jb] = leaf_entry(off, len);
        if (len == 0) continue;
        if (!more_bits || len == 1) {  // one key value: one run
            rk[off] = keys[off];
            rc[off] = len;
            flag[off] = 1;
        } else if (len <= 4u) {
            tiny_leaf<K, 4>(keys, off, len, rk, rc, flag);
        } else if (len <= 8u) {
            tiny_leaf<K, 8>(keys, off, len, rk, rc, flag);
        } else if (len <= (uint32_t)kTinyKeys) {
            tiny_leaf<K, kTinyKeys>(keys, off, len, rk, rc, flag);
        }
    }
}

// Lane l of the wave receives v from the lane whose `dst` is l (dst must
// be a permutation of the lanes).
__device__ __forceinline__ uint32_t lane_send(uint32_t v, int dst) {
    return (uint32_t)__builtin_amdgcn_ds_permute(dst << 2, (int)v);
}
__device__ __forceinline__ uint64_t lane_send(uint64_t v, int dst) {
    return (uint64_t)lane_send((uint32_t)v, dst) | ((uint64_t)lane_send((uint32_t)(v >> 32), dst) << 32);
}

// Leaves of 17..64 keys: one wave each (four waves per workgroup, each on
// its own leaves), one key per lane.  Each key's place is the number of
// keys of the leaf before it in key order (ties by lane); lanes past the
// leaf keep their own place, so the places are a permutation of the lanes
// and one forward permute sorts the leaf.  The runs follow from ballots.
template <typename K>
__global__ __launch_bounds__(kMsdThreads) void k_msd_small(const K *__restrict__ keys,
                                                           const MCtl *__restrict__ ctl,
                                                           K *__restrict__ rk,
                                                           uint32_t *__restrict__ rc,
                                                           uint8_t *__restrict__ flag,
                                                           const uint64_t *__restrict__ mid) {
    const int lane = threadIdx.x & 63;
    const int64_t nm = ctl->nmid[0];
    const int64_t waves = (int64_t)gridDim.x * (kMsdThreads / 64);
    int64_t im = (int64_t)blockIdx.x * (kMsdThreads / 64) + (threadIdx.x >> 6);
    uint64_t e = im < nm ? mid[im] : 0;
    for (; im < nm; im += waves) {
        const int64_t off = (int64_t)(e >> kLenBits);
        const int n = (int)(e & ((1u << kLenBits) - 1u));
        const K x = lane < n ? keys[off + lane] : ~(K)0;
        e = im + waves < nm ? mid[im + waves] : 0;  // the next leaf's entry, early
        int r = 0;
        for (int j = 0; j < n; ++j) {
            const K y = (K)__shfl(x, j);
            r += (y < x || (y == x && j < lane)) ? 1 : 0;
        }
        if (lane >= n) r = lane;
        const K v = lane_send(x, r);
        const K pv = (K)__shfl_up(v, 1);
        const bool head = lane < n && (lane == 0 || v != pv);
        const uint64_t mask = __ballot(head);
        if (head) {
            const uint32_t q = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
            const uint64_t later = mask & ~((2ull << lane) - 1ull);  // heads after this lane
            const int nxt = later ? __builtin_ctzll(later) : n;
            rk[off + q] = v;
            rc[off + q] = (uint32_t)(nxt - lane);
            flag[off + q] = 1;
        }
    }
}

// Workgroup barrier that orders LDS only: global loads in flight (the next
// leaf's keys) stay in flight across it.  Used where the threads share
// nothing but LDS.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Block-wide exclusive scan of one value per thread (kThr threads): wave
// scans with shuffles, then the wave totals.  Returns the exclusive
// prefix; *total receives the sum.
template <int kThr>
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t *wsum, uint32_t *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t x = __shfl_up(incl, o);
        if (lane >= o) incl += x;
    }
    if (lane == 63) wsum[wave] = incl;
    lds_barrier();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kThr / 64; ++w) {
        const uint32_t x = wsum[w];
        before += w < wave ? x : 0u;
        all += x;
    }
    *total = all;
    lds_barrier();
    return before + incl - v;
}

// Larger leaves (more than 64 keys, at most kCap, more than one bit left):
// one workgroup each, its keys in registers.  All keys of a leaf agree above
// bit lo, so the leaf sorts their low lo bits as keys of type KL (32-bit
// whenever lo <= 32) and puts the common high bits back on output.  The
// keys are split in LDS by their next bits into about as many buckets as
// keys (at most 2^kDigitMax), keeping each bucket's smallest and largest
// key; each key's place in the sorted leaf is then its bucket's start plus
// the number of keys of its bucket before it in key order (ties by
// position in the bucket), so the work per key is the size of its bucket,
// and none when the bucket holds one key value.  The sorted keys replace
// the bucketed ones in LDS, and the runs follow from ballots over them:
// each run's first key writes the run, and its position goes to a list that
// overwrites the front of the sorted keys (never ahead of the keys still to
// be read).  Entry im of the queue is q[im * step].
template <typename K, typename KL, int kThr, int kCap, int kDigitMax>
__global__ __launch_bounds__(kThr, kThr >= 1024 ? 8 : 1) void k_msd_leaves(
    const K *__restrict__ keys, const uint32_t *__restrict__ nq, int lo, K *__restrict__ rk,
    uint32_t *__restrict__ rc, uint8_t *__restrict__ flag, const uint64_t *__restrict__ q,
    int64_t step) {
    constexpr int kPer = kCap / kThr;  // keys per thread
    constexpr int kNb = 1 << kDigitMax;
    constexpr bool kRel = sizeof(KL) < sizeof(K);
    static_assert(sizeof(KL) >= 4 && kCap < 65536, "run head positions are 16-bit");
    __shared__ KL B[kCap];
    __shared__ uint32_t h[kNb], st[kNb];
    __shared__ KL mn[kNb], mx[kNb];
    __shared__ uint32_t wsum[kThr / 64];
    // run head positions, written over the sorted keys: head q of step i0
    // lands below byte 2 * (i0 + kThr), and steps after i0 read from byte
    // sizeof(KL) * (i0 + kThr - 1) on
    uint16_t *hp = (uint16_t *)B;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t nm = *nq, G = gridDim.x;
    constexpr uint32_t kLenMask = (1u << kLenBits) - 1u;
    const K low = kRel ? (K)((((uint64_t)1) << lo) - 1u) : ~(K)0;
    int64_t im = blockIdx.x;
    uint64_t e = im < nm ? q[im * step] : 0;
    for (; im < nm; im += G) {
        const int64_t off = (int64_t)(e >> kLenBits);
        const int n = (int)(e & kLenMask);
        KL x[kPer];
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            const int i = tid + t * kThr;
            x[t] = i < n ? (KL)(keys[off + i] & low) : (KL)0;
        }
        const K high = keys[off] & ~low;  // the bits all keys of the leaf share
        e = im + G < nm ? q[(im + G) * step] : 0;  // the next leaf's entry, early
        int nbits = 8;  // buckets: about one per key, 256 at least
        while (nbits < kDigitMax && (1 << nbits) < n) ++nbits;
        nbits = min(nbits, lo);
        const int dlo = lo - nbits, nb = 1 << nbits;
        const int bpt = nb >= kThr ? nb / kThr : 1;  // buckets per thread
        const int b_lo = tid * bpt;
        for (int d = tid; d < nb; d += kThr) {
            h[d] = 0;
            mn[d] = ~(KL)0;
            mx[d] = (KL)0;
        }
        lds_barrier();
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            if (tid + t * kThr < n) {
                const uint32_t d = digit_of((uint64_t)x[t], dlo, nbits);
                atomicAdd(&h[d], 1u);
                atomicMin(&mn[d], x[t]);
                atomicMax(&mx[d], x[t]);
            }
        }
        lds_barrier();
        uint32_t tot = 0;
        for (int j = 0; j < bpt; ++j)
            if (b_lo + j < nb) tot += h[b_lo + j];
        uint32_t all;
        uint32_t run = block_scan<kThr>(tot, wsum, &all);
        for (int j = 0; j < bpt; ++j) {
            const int d = b_lo + j;
            if (d < nb) {
                const uint32_t cd = h[d];
                st[d] = run;
                h[d] = run;  // becomes the scatter cursor, then the bucket's end
                run += cd;
            }
        }
        lds_barrier();
        uint32_t pos[kPer];
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            if (tid + t * kThr < n) {
                pos[t] = atomicAdd(&h[digit_of((uint64_t)x[t], dlo, nbits)], 1u);
                B[pos[t]] = x[t];
            }
        }
        lds_barrier();
#pragma unroll
        for (int t = 0; t < kPer; ++t) {  // pos becomes the place in the sorted leaf
            if (tid + t * kThr < n) {
                const uint32_t d = digit_of((uint64_t)x[t], dlo, nbits);
                const KL v = x[t];
                if (mn[d] != mx[d]) {
                    const uint32_t p = pos[t], e1b = h[d];
                    uint32_t rr = st[d], j = rr;
                    for (; j + 2 <= e1b; j += 2) {
                        const KL y0 = B[j], y1 = B[j + 1];
                        rr += (y0 < v || (y0 == v && j < p)) ? 1u : 0u;
                        rr += (y1 < v || (y1 == v && j + 1 < p)) ? 1u : 0u;
                    }
                    for (; j < e1b; ++j) {
                        const KL y = B[j];
                        rr += (y < v || (y == v && j < p)) ? 1u : 0u;
                    }
                    pos[t] = rr;
                }
            }
        }
        lds_barrier();
#pragma unroll
        for (int t = 0; t < kPer; ++t)
            if (tid + t * kThr < n) B[pos[t]] = x[t];
        lds_barrier();
        // run heads in order, kThr positions per step
        uint32_t runs = 0;
        for (int i0 = 0; i0 < n; i0 += kThr) {
            const int i = i0 + tid;
            const KL v = i < n ? B[i] : (KL)0;
            const bool head = i < n && (i == 0 || v != B[i - 1]);
            const uint64_t mask = __ballot(head);
            if (lane == 0) wsum[wave] = (uint32_t)__popcll(mask);
            lds_barrier();
            uint32_t before = 0, stp = 0;
#pragma unroll
            for (int w = 0; w < kThr / 64; ++w) {
                before += w < wave ? wsum[w] : 0u;
                stp += wsum[w];
            }
            if (head) {
                const uint32_t qq = runs + before + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
                hp[qq] = (uint16_t)i;
                rk[off + qq] = high | (K)v;
                flag[off + qq] = 1;
            }
            runs += stp;
            lds_barrier();
        }
        for (uint32_t qq = tid; qq < runs; qq += kThr) {
            const uint32_t h1 = qq + 1 < runs ? (uint32_t)hp[qq + 1] : (uint32_t)n;
            rc[off + qq] = h1 - (uint32_t)hp[qq];
        }
        lds_barrier();
    }
}

// The whole key array as one leaf (nk <= kLeafKeys keys), one wave: a
// bitonic network in LDS.
template <typename K>
__global__ __launch_bounds__(64) void k_msd_root_leaf(const K *__restrict__ keys, int64_t nk,
                                                      int bits, K *__restrict__ rk,
                                                      uint32_t *__restrict__ rc,
                                                      uint8_t *__restrict__ flag) {
    __shared__ K B[kLeafKeys];
    __shared__ uint16_t hp[kLeafKeys];
    const int lane = threadIdx.x;
    const int n = (int)nk;
    if (bits <= 0 || n == 1) {
        if (lane == 0) {
            rk[0] = keys[0];
            rc[0] = (uint32_t)n;
            flag[0] = 1;
        }
        return;
    }
    int P = 2;
    while (P < n) P <<= 1;
    for (int i = lane; i < P; i += 64) B[i] = i < n ? keys[i] : ~(K)0;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < P; i += 64) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const K x = B[i], y = B[ixj];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        B[i] = y;
                        B[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
    uint32_t runs = 0;
    for (int i0 = 0; i0 < n; i0 += 64) {
        const int i = i0 + lane;
        const bool head = i < n && (i == 0 || B[i] != B[i - 1]);
        const uint64_t mask = __ballot(head);
        if (head) hp[runs + __popcll(mask & ((1ull << lane) - 1ull))] = (uint16_t)i;
        runs += (uint32_t)__popcll(mask);
    }
    __syncthreads();
    for (uint32_t q = lane; q < runs; q += 64) {
        const uint32_t h0 = hp[q];
        const uint32_t h1 = q + 1 < runs ? (uint32_t)hp[q + 1] : (uint32_t)n;
        rk[q] = B[h0];
        rc[q] = h1 - h0;
        flag[q] = 1;
    }
}

__global__ void k_msd_clear(uint32_t *__restrict__ f, int64_t n4) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x)
        f[i] = 0u;
}

// Runs per block of kScanBlock positions.
__global__ __launch_bounds__(kMsdThreads) void k_scan_sums(const uint8_t *__restrict__ f,
                                                           int64_t n,
                                                           uint32_t *__restrict__ bsum) {
    // 16 flags (0 or 1 each) per thread in one 16-byte load: the flag array
    // is zero up to a multiple of 16 bytes; a word's four flags sum in its
    // top byte after a multiply by 0x01010101
    static_assert(kScanBlock == kMsdThreads * 16, "one 16-byte load per thread");
    __shared__ uint32_t part[kMsdThreads / 64];
    const int64_t p = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * 16;
    uint32_t s = 0;
    if (p < n) {
        const uint4 v = *reinterpret_cast<const uint4 *>(f + p);
        s = ((v.x * 0x01010101u) >> 24) + ((v.y * 0x01010101u) >> 24) +
            ((v.z * 0x01010101u) >> 24) + ((v.w * 0x01010101u) >> 24);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
#pragma unroll
        for (int w = 0; w < kMsdThreads / 64; ++w) t += part[w];
        bsum[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void k_scan_blocks(uint32_t *bsum, int64_t nb, MCtl *ctl) {
    __shared__ uint32_t part[1024];
    const int64_t per = (nb + 1023) / 1024;
    const int64_t a = min(nb, (int64_t)threadIdx.x * per), b = min(nb, a + per);
    uint32_t s = 0;
    for (int64_t i = a; i < b; ++i) s += bsum[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t r = part[threadIdx.x] - s;
    for (int64_t i = a; i < b; ++i) {
        const uint32_t v = bsum[i];
        bsum[i] = r;
        r += v;
    }
    if (threadIdx.x == 1023) ctl->total = part[1023];
}

// Runs to their places: the block's first place (scanned block sums) plus
// the flagged positions before it, taken 256 consecutive positions at a
// time so that neighbouring lanes write neighbouring places.
template <typename K>
__global__ __launch_bounds__(kMsdThreads) void k_msd_compact(
    const K *__restrict__ rk, const uint32_t *__restrict__ rc, const uint8_t *__restrict__ f,
    int64_t n, const uint32_t *__restrict__ bsum, const MCtl *__restrict__ ctl,
    K *__restrict__ uniq, uint32_t *__restrict__ cnt, uint32_t *__restrict__ nruns) {
    __shared__ uint32_t wsum[kMsdThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t base = bsum[blockIdx.x];
    for (int e = 0; e < kScanBlock / kMsdThreads; ++e) {
        const int64_t p = (int64_t)blockIdx.x * kScanBlock + (int64_t)e * kMsdThreads + threadIdx.x;
        const bool on = p < n && f[p] != 0;
        const uint64_t mask = __ballot(on);
        if (lane == 0) wsum[wave] = (uint32_t)__popcll(mask);
        __syncthreads();
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int w = 0; w < kMsdThreads / 64; ++w) {
            before += w < wave ? wsum[w] : 0u;
            all += wsum[w];
        }
        if (on) {
            const uint32_t r = base + before + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
            uniq[r] = rk[p];
            cnt[r] = rc[p];
        }
        base += all;
        __syncthreads();
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *nruns = ctl->total;
}

// Scratch layout (256-byte aligned slices).
struct MsdScratch {
    MCtl *ctl;
    MSeg *segs[2];
    uint32_t *counts[2], *cursor, *rc, *bsum;
    uint8_t *flag;
    uint32_t *top;
    int64_t *start;
    uint64_t *mid, *bigq;
    void *rk;
    int64_t seg_cap, nb, mid_cap, big_cap;
};

size_t carve_msd(char *base, int64_t nk, size_t kb, MsdScratch *S) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        char *p = base ? base + off : nullptr;
        off += bytes ? bytes : 1;
        return p;
    };
    MsdScratch s;
    s.seg_cap = nk / kBigKeys + 2;  // each next-level segment has more than kBigKeys keys
    s.nb = (nk + kScanBlock - 1) / kScanBlock;
    s.ctl = (MCtl *)take(sizeof(MCtl));
    s.top = (uint32_t *)take(sizeof(uint32_t) * 256);
    s.segs[0] = (MSeg *)take(sizeof(MSeg) * (size_t)s.seg_cap);
    s.segs[1] = (MSeg *)take(sizeof(MSeg) * (size_t)s.seg_cap);
    s.counts[0] = (uint32_t *)take(sizeof(uint32_t) * 256 * (size_t)s.seg_cap);
    s.counts[1] = (uint32_t *)take(sizeof(uint32_t) * 256 * (size_t)s.seg_cap);
    s.cursor = (uint32_t *)take(sizeof(uint32_t) * 256 * (size_t)s.seg_cap);
    s.start = (int64_t *)take(sizeof(int64_t) * 256 * (size_t)s.seg_cap);
    s.mid_cap = nk / (kTinyKeys + 1) + 1;  // each queued leaf has more than kTinyKeys keys
    s.mid = (uint64_t *)take(sizeof(uint64_t) * (size_t)s.mid_cap);
    s.big_cap = nk / (kLeafKeys + 1) + 1;
    s.bigq = (uint64_t *)take(sizeof(uint64_t) * (size_t)s.big_cap);
    s.flag = (uint8_t *)take((size_t)((nk + 15) / 16 * 16));  // whole 16-byte loads
    s.rc = (uint32_t *)take(sizeof(uint32_t) * (size_t)nk);
    s.rk = take(kb * (size_t)nk);
    s.bsum = (uint32_t *)take(sizeof(uint32_t) * (size_t)s.nb);
    if (S) *S = s;
    return off;
}

// The two leaf sizes of one level; KL is the type the leaves sort the keys'
// low lo bits as.
template <typename K, typename KL>
void launch_leaves(const MsdScratch &S, const K *out, int lo, K *rk, int64_t nc, int cus,
                   hipStream_t s) {
    hipLaunchKernelGGL((k_msd_leaves<K, KL, kLeafThreads, kLeafKeys, kLeafDigit>),
                       dim3((unsigned)std::min<int64_t>(nc, 16 * (int64_t)cus)), dim3(kLeafThreads),
                       0, s, out, &S.ctl->nmid[1], lo, rk, S.rc, S.flag, S.mid + (S.mid_cap - 1),
                       (int64_t)-1);
    hipLaunchKernelGGL((k_msd_leaves<K, KL, kBigThreads, kBigKeys, big_digit<KL>()>),
                       dim3((unsigned)std::min<int64_t>(nc, 2 * (int64_t)cus)), dim3(kBigThreads),
                       0, s, out, &S.ctl->nmid[2], lo, rk, S.rc, S.flag, S.bigq, (int64_t)1);
}

}  // namespace

size_t msd_scratch_bytes(int64_t nk, size_t key_bytes) {
    return carve_msd(nullptr, nk, key_bytes, nullptr);
}

uint32_t *msd_top_hist(void *scratch, int64_t nk, size_t key_bytes) {
    MsdScratch S;
    carve_msd((char *)scratch, nk, key_bytes, &S);
    return S.top;
}

template <typename K>
int msd_sort_rle(const fc_db *db, K *keys, K *alt, int64_t nk, unsigned end_bit, K *uniq,
                 uint32_t *cnt, uint32_t *nruns, void *scratch, bool top_given, hipStream_t s) {
    if (nk <= 0) return FC_OK;
    if (nk >= (int64_t(1) << 32)) {
        set_error("msd_sort_rle: %lld keys exceed the 32-bit positions", (long long)nk);
        return FC_ERR_RANGE;
    }
    MsdScratch S;
    carve_msd((char *)scratch, nk, sizeof(K), &S);
    const int cus = db->cu_count > 0 ? db->cu_count : 256;
    K *buf[2] = {keys, alt};
    K *rk = (K *)S.rk;
    hipLaunchKernelGGL(k_msd_init, dim3(1), dim3(256), 0, s, S.ctl, S.segs[0], S.counts[0],
                       top_given ? (const uint32_t *)S.top : nullptr, nk);
    const int64_t n4 = (nk + 15) / 16 * 4;  // flag words, to a multiple of 16 bytes
    hipLaunchKernelGGL(k_msd_clear, dim3((unsigned)std::min<int64_t>((n4 + 255) / 256, 8 * cus)),
                       dim3(256), 0, s, (uint32_t *)S.flag, n4);
    FC_HIP(hipGetLastError());
    if (nk <= kLeafKeys || end_bit == 0) {
        hipLaunchKernelGGL(k_msd_root_leaf<K>, dim3(1), dim3(64), 0, s, keys, nk, (int)end_bit,
                           rk, S.rc, S.flag);
        FC_HIP(hipGetLastError());
    } else {
        // every level is enqueued; a level without segments exits at once.
        // Level l has at most 256^l segments, and never more than seg_cap.
        const int levels = (int)((end_bit + 7) / 8);
        const int64_t tiles_max = (nk + kTileKeys - 1) / kTileKeys;
        int64_t nseg_max = 1;
        for (int l = 0; l < levels; ++l) {
            const int cur = l & 1, hi = (int)end_bit - 8 * l;
            const int lo = std::max(hi - 8, 0), width = hi - lo;
            const K *in = buf[cur];
            K *out = buf[cur ^ 1];
            const int64_t gt = std::min<int64_t>(tiles_max + nseg_max, 16 * (int64_t)cus);
            const int64_t nc = nseg_max * 256;
            if (l > 0 || !top_given)  // the root's counts may be given
                hipLaunchKernelGGL(k_msd_hist<K>, dim3((unsigned)gt), dim3(kMsdThreads), 0, s, in,
                                   S.segs[cur], S.ctl, cur, lo, width, S.counts[cur]);
            hipLaunchKernelGGL(k_msd_split, dim3((unsigned)std::min<int64_t>(nseg_max, 8 * cus)),
                               dim3(kMsdThreads), 0, s, S.segs[cur], S.ctl, cur, lo, S.counts[cur],
                               S.counts[cur ^ 1], S.start, S.cursor, S.segs[cur ^ 1]);
            hipLaunchKernelGGL(k_msd_tiles, dim3(1), dim3(1024), 0, s, S.segs[cur ^ 1], S.ctl,
                               cur ^ 1);
            if (l == 0)
                hipLaunchKernelGGL((k_msd_scatter<K, false>), dim3((unsigned)gt), dim3(kMsdThreads),
                                   0, s, in, out, S.segs[cur], S.ctl, cur, lo, width, S.cursor);
            else
                hipLaunchKernelGGL((k_msd_scatter<K, true>), dim3((unsigned)gt), dim3(kMsdThreads),
                                   0, s, in, out, S.segs[cur], S.ctl, cur, lo, width, S.cursor);
            hipLaunchKernelGGL(k_msd_tiny<K>,
                               dim3((unsigned)std::min<int64_t>((nc + kMsdThreads - 1) / kMsdThreads,
                                                                8 * (int64_t)cus)),
                               dim3(kMsdThreads), 0, s, out, S.ctl, cur, lo, S.counts[cur],
                               S.start, rk, S.rc, S.flag, S.mid, S.mid_cap, S.bigq);
            hipLaunchKernelGGL(k_msd_small<K>, dim3((unsigned)std::min<int64_t>((nc + 3) / 4, 16 * (int64_t)cus)),
                               dim3(kMsdThreads), 0, s, out, S.ctl, rk, S.rc, S.flag, S.mid);
            if (sizeof(K) > 4 && lo <= 32)
                launch_leaves<K, uint32_t>(S, out, lo, rk, nc, cus, s);
            else
                launch_leaves<K, K>(S, out, lo, rk, nc, cus, s);
            FC_HIP(hipGetLastError());
            nseg_max = std::min<int64_t>(nseg_max * 256, S.seg_cap);
        }
    }
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)S.nb), dim3(kMsdThreads), 0, s, S.flag, nk,
                       S.bsum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, S.bsum, S.nb, S.ctl);
    hipLaunchKernelGGL(k_msd_compact<K>, dim3((unsigned)S.nb), dim3(kMsdThreads), 0, s, rk, S.rc,
                       S.flag, nk, S.bsum, S.ctl, uniq, cnt, nruns);
    FC_HIP(hipGetLastError());
    return FC_OK;
}

template int msd_sort_rle<uint32_t>(const fc_db *, uint32_t *, uint32_t *, int64_t, unsigned,
                                    uint32_t *, uint32_t *, uint32_t *, void *, bool, hipStream_t);
template int msd_sort_rle<uint64_t>(const fc_db *, uint64_t *, uint64_t *, int64_t, unsigned,
                                    uint64_t *, uint32_t *, uint32_t *, void *, bool, hipStream_t);

}  // namespace fc
