// Data-parallel primitives for the GPMA+ update, written for gfx950 wave64:
// exclusive scan, keys-only LSD radix sort, unique and stream compaction.
// The paper builds its update from such primitives (Section 5.2: sort,
// run-length encoding, exclusive scan); these are our own.
#include "common.h"

using namespace gpma_dev;

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;   // 2048

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / kWave;
// 64-key chunks per wave: 16 (4096-key tiles) for large inputs, 4 (1024-key
// tiles) for batches, so a 2^16-key batch still spreads over 64 workgroups
constexpr int kChunksLarge = 16;
constexpr int kChunksSmall = 4;
constexpr int kChunksMin = 2;
constexpr uint64_t kSmallSortMax = 1ull << 20;
constexpr uint64_t kFuseTiles = 128;
constexpr uint64_t kScanSingleMax = 2048;   // one workgroup, two items per thread

inline uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

__global__ void __launch_bounds__(kScanThreads)
k_scan_reduce(const uint32_t *__restrict__ in, uint64_t n, uint32_t *__restrict__ tile_sums) {
    __shared__ uint32_t lds[kScanThreads / kWave + 1];
    uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        uint64_t idx = base + (uint64_t)i * kScanThreads + threadIdx.x;
        if (idx < n) s += in[idx];
    }
    uint32_t tot;
    block_exclusive_scan(s, &tot, lds);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

// one workgroup: exclusive scan of the tile sums in place, total to *total
__global__ void __launch_bounds__(1024)
k_scan_top(uint32_t *__restrict__ sums, uint64_t ntiles, uint32_t *__restrict__ total) {
    __shared__ uint32_t lds[1024 / kWave + 1];
    uint32_t carry = 0;
    for (uint64_t base = 0; base < ntiles; base += blockDim.x) {
        uint64_t idx = base + threadIdx.x;
        uint32_t v = idx < ntiles ? sums[idx] : 0;
        uint32_t tot;
        uint32_t e = block_exclusive_scan(v, &tot, lds);
        if (idx < ntiles) sums[idx] = carry + e;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

// small inputs: one workgroup, each thread owns a contiguous run of items
__global__ void __launch_bounds__(1024)
k_scan_single(const uint32_t *__restrict__ in, uint32_t *__restrict__ out, uint64_t n,
              uint32_t *__restrict__ total) {
    __shared__ uint32_t lds[1024 / kWave + 1];
    const uint64_t per = (n + blockDim.x - 1) / blockDim.x;
    const uint64_t b = (uint64_t)threadIdx.x * per;
    const uint64_t e = b + per < n ? b + per : n;
    uint32_t s = 0;
    for (uint64_t i = b; i < e; i++) s += in[i];
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, &tot, lds);
    for (uint64_t i = b; i < e; i++) {
        const uint32_t v = in[i];
        out[i] = run;
        run += v;
    }
    if (threadIdx.x == 0 && total) *total = tot;
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_apply(const uint32_t *__restrict__ in, uint32_t *__restrict__ out, uint64_t n,
             const uint32_t *__restrict__ tile_offs) {
    __shared__ uint32_t lds[kScanThreads / kWave + 1];
    // each thread takes kScanItems consecutive items so the scan order is the
    // array order
    uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        uint64_t idx = base + i;
        v[i] = idx < n ? in[idx] : 0;
        s += v[i];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, &tot, lds) + tile_offs[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        uint64_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
}

// ---------------------------------------------------------------------------
// radix sort

struct DigitMap {
    uint32_t shift, mask, dbits, V;
    __device__ __forceinline__ uint32_t operator()(uint64_t k) const {
        uint64_t src = k >> 32;
        uint32_t dst = (uint32_t)k;
        uint64_t d = (dst == kGuardDst) ? (uint64_t)V : (uint64_t)dst;
        uint64_t ck = (src << dbits) | d;
        return (uint32_t)(ck >> shift) & mask;
    }
};

template <int CH>
__global__ void __launch_bounds__(kSortThreads)
k_radix_upsweep(const uint64_t *__restrict__ keys, uint64_t n, const uint32_t *__restrict__ n_dev,
                DigitMap dm, uint32_t ntiles, int tile_major, uint32_t *__restrict__ counts,
                Ctl *__restrict__ check) {
    constexpr int kSortTile = kSortThreads * CH;
    if (n_dev && *n_dev < n) n = *n_dev;
    __shared__ uint32_t hist[256];
    for (int i = threadIdx.x; i < 256; i += kSortThreads) hist[i] = 0;
    __syncthreads();
    uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    bool bad = false;
#pragma unroll 4
    for (int i = 0; i < CH; i++) {
        uint64_t idx = base + (uint64_t)i * kSortThreads + threadIdx.x;
        if (idx < n) {
            const uint64_t k = keys[idx];
            atomicAdd(&hist[dm(k)], 1u);
            bad |= key_src(k) >= dm.V || key_dst(k) >= dm.V;
        }
    }
    // batch validation rides on the first pass: src < V and dst < V
    if (check && __ballot(bad) && __lane_id() == 0) atomicOr(&check->err, 1u);
    __syncthreads();
    // digit-major for the global scan; tile-major when each downsweep block
    // derives its own offsets (coalesced reads there)
    for (uint32_t d = threadIdx.x; d <= dm.mask; d += kSortThreads)
        counts[tile_major ? (uint64_t)blockIdx.x * (dm.mask + 1) + d : (uint64_t)d * ntiles + blockIdx.x] = hist[d];
}

// Stable scatter of one tile.  Wave w owns keys [w*1024, (w+1)*1024) of the
// tile and walks them in 64-key chunks; lanes holding the same digit find
// each other with one ballot per digit bit, so the rank of a key among equal
// digits is (keys of that digit in earlier chunks) + (lower lanes in this
// chunk).  Per-wave digit counts are then prefixed across waves.
template <int CH>
__global__ void __launch_bounds__(kSortThreads)
k_radix_downsweep(const uint64_t *__restrict__ keys, uint64_t n, const uint32_t *__restrict__ n_dev,
                  DigitMap dm, uint32_t bits, uint32_t ntiles, const uint32_t *__restrict__ offs,
                  int fuse_offsets, uint64_t *__restrict__ out) {
    if (n_dev && *n_dev < n) n = *n_dev;
    constexpr int kSortChunks = CH;
    constexpr int kSortTile = kSortThreads * CH;
    constexpr int kSortWaveSpan = kWave * CH;
    __shared__ uint32_t wcnt[kSortWaves][256];
    __shared__ uint32_t goff[256];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    for (int i = threadIdx.x; i < kSortWaves * 256; i += kSortThreads) (&wcnt[0][0])[i] = 0;
    __syncthreads();

    const uint64_t base = (uint64_t)blockIdx.x * kSortTile + (uint64_t)w * kSortWaveSpan;
    const uint64_t ltmask = lanemask_lt();
    uint64_t k[kSortChunks];
    uint32_t rk[kSortChunks];
#pragma unroll
    for (int c = 0; c < kSortChunks; c++) {
        uint64_t idx = base + (uint64_t)c * kWave + lane;
        bool valid = idx < n;
        k[c] = valid ? keys[idx] : 0;
        uint32_t d = dm(k[c]);
        uint64_t m = __ballot(valid);
        for (uint32_t b = 0; b < bits; b++) {
            uint32_t bit = (d >> b) & 1u;
            uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        uint32_t before = wcnt[w][d];
        rk[c] = before + (uint32_t)__popcll(m & ltmask);
        wave_lds_sync();
        if (valid && (uint32_t)(__ffsll((unsigned long long)m) - 1) == (uint32_t)lane)
            wcnt[w][d] = before + (uint32_t)__popcll(m);
        wave_lds_sync();
    }
    __syncthreads();
    if (fuse_offsets) {
        // few tiles: derive this tile's digit offsets from the raw counts
        // (digits below d over all tiles, plus digit d in earlier tiles)
        __shared__ uint32_t dtot[257];
        for (uint32_t d = threadIdx.x; d <= dm.mask; d += kSortThreads) {
            uint32_t tot = 0, before = 0;
            const uint32_t nb = dm.mask + 1;
#pragma unroll 8
            for (uint32_t t = 0; t < ntiles; t++) {
                const uint32_t c = offs[(uint64_t)t * nb + d];   // tile-major: coalesced over d
                tot += c;
                before += t < blockIdx.x ? c : 0u;
            }
            dtot[d] = tot;
            goff[d] = before;
        }
        __syncthreads();
        // one digit per thread (at most 256 digits, 256 threads)
        __shared__ uint32_t sl[kSortThreads / kWave + 1];
        const uint32_t d = threadIdx.x;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(d <= dm.mask ? dtot[d] : 0u, &tot, sl);
        if (d <= dm.mask) goff[d] += ex;
    }
    for (uint32_t d = threadIdx.x; d <= dm.mask; d += kSortThreads) {
        uint32_t run = 0;
#pragma unroll
        for (int ww = 0; ww < kSortWaves; ww++) {
            uint32_t t = wcnt[ww][d];
            wcnt[ww][d] = run;
            run += t;
        }
        if (!fuse_offsets) goff[d] = offs[(uint64_t)d * ntiles + blockIdx.x];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kSortChunks; c++) {
        uint64_t idx = base + (uint64_t)c * kWave + lane;
        if (idx < n) {
            uint32_t d = dm(k[c]);
            out[goff[d] + wcnt[w][d] + rk[c]] = k[c];
        }
    }
}

// ---------------------------------------------------------------------------
// flags for compaction

__global__ void k_flag_unique(const uint64_t *__restrict__ a, uint64_t n,
                              const uint32_t *__restrict__ n_dev, uint32_t *__restrict__ flags) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t lim = n_dev ? *n_dev : n;
    flags[i] = (i < lim && (i == 0 || a[i] != a[i - 1])) ? 1u : 0u;
}

__global__ void k_scatter_unique(const uint64_t *__restrict__ a, uint64_t n,
                                 const uint32_t *__restrict__ n_dev,
                                 const uint32_t *__restrict__ pos, uint64_t *__restrict__ out) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t lim = n_dev ? *n_dev : n;
    if (i < lim && (i == 0 || a[i] != a[i - 1])) out[pos[i]] = a[i];
}

__global__ void __launch_bounds__(256)
k_flag_pending(const uint8_t *__restrict__ status, const uint32_t *__restrict__ n_dev,
               uint64_t n_max, uint32_t *__restrict__ flags, int del, uint64_t cap_h,
               Ctl *__restrict__ ctl) {
    __shared__ uint32_t red[3][256 / kWave];
    const uint64_t n = *n_dev;
    uint32_t done = 0, noop = 0, head = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_max; i += stride) {
        uint32_t f = 0;
        if (i < n) {
            const uint8_t st = status[i];
            const uint8_t state = st & kStateMask;
            f = state == kPending;
            done += state == kDone;
            noop += state == kNoop;
            head += (st & kHead) ? 1u : 0u;
        }
        flags[i] = f;
    }
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        done += __shfl_xor(done, d, kWave);
        noop += __shfl_xor(noop, d, kWave);
        head += __shfl_xor(head, d, kWave);
    }
    const int w = threadIdx.x / kWave;
    if (__lane_id() == 0) { red[0][w] = done; red[1][w] = noop; red[2][w] = head; }
    __syncthreads();
    if (threadIdx.x == 0 && ctl) {
        uint32_t a = 0, b = 0, c = 0;
        for (int k = 0; k < 256 / kWave; k++) { a += red[0][k]; b += red[1][k]; c += red[2][k]; }
        if (a) {
            atomicAdd((unsigned long long *)&ctl->applied, (unsigned long long)a);
            atomicAdd((unsigned long long *)&ctl->dn, (unsigned long long)(del ? -(int64_t)a : (int64_t)a));
        }
        if (b) atomicAdd((unsigned long long *)&ctl->noops, (unsigned long long)b);
        if (c) {
            atomicAdd(&ctl->segs, c);
            atomicAdd((unsigned long long *)&ctl->rewritten, (unsigned long long)(c * cap_h));
        }
    }
}

__global__ void k_scatter_pending(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ leaf,
                                  const uint8_t *__restrict__ status,
                                  const uint32_t *__restrict__ n_dev, uint64_t n_max,
                                  const uint32_t *__restrict__ pos, uint64_t *__restrict__ keys_out,
                                  uint32_t *__restrict__ leaf_out, uint8_t *__restrict__ status_out) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_max || i >= *n_dev || (status[i] & kStateMask) != kPending) return;
    uint32_t p = pos[i];
    keys_out[p] = keys[i];
    leaf_out[p] = leaf[i];
    status_out[p] = kPending;
}

// Two-launch compaction for up to kCmpMaxTiles tiles of kCmpTile items: a
// count pass writes per-tile totals (and statistics), a scatter pass derives
// its tile's offset from the totals before it, scans its items in order and
// writes the kept ones.  Block 0 of the scatter pass publishes the total.
constexpr int kCmpItems = 8;
constexpr int kCmpTile = 256 * kCmpItems;
constexpr uint64_t kCmpMaxTiles = 1024;

template <int N>
__device__ __forceinline__ void block_sum_n(uint32_t (&v)[N], uint32_t (*lds)[256 / kWave]) {
#pragma unroll
    for (int k = 0; k < N; k++)
#pragma unroll
        for (int d = kWave / 2; d >= 1; d >>= 1) v[k] += __shfl_xor(v[k], d, kWave);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if (__lane_id() == 0)
#pragma unroll
        for (int k = 0; k < N; k++) lds[k][w] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; k++) {
        uint32_t t = 0;
        for (int j = 0; j < 256 / kWave; j++) t += lds[k][j];
        v[k] = t;
    }
}

// sum of tile counts before tile t, and of all tiles
__device__ __forceinline__ void tile_prefix(const uint32_t *__restrict__ cnt, uint32_t ntiles, uint32_t t,
                                            uint32_t *before, uint32_t *total) {
    __shared__ uint32_t lds[2][256 / kWave];
    uint32_t v[2] = {0, 0};
    for (uint32_t i = threadIdx.x; i < ntiles; i += blockDim.x) {
        const uint32_t c = cnt[i];
        v[1] += c;
        v[0] += i < t ? c : 0u;
    }
    block_sum_n<2>(v, lds);
    *before = v[0];
    *total = v[1];
}

__device__ __forceinline__ uint64_t dyn_limit(const uint32_t *n_dev, uint64_t n_max) {
    if (!n_dev) return n_max;
    const uint64_t n = *n_dev;
    return n < n_max ? n : n_max;
}

__device__ __forceinline__ bool unique_head(const uint64_t *a, uint64_t i, uint64_t lim) {
    return i < lim && (i == 0 || a[i] != a[i - 1]);
}

__global__ void __launch_bounds__(256)
k_unique_count(const uint64_t *__restrict__ a, uint64_t n_max, const uint32_t *__restrict__ n_dev,
               uint32_t *__restrict__ tile_cnt) {
    __shared__ uint32_t lds[1][256 / kWave];
    const uint64_t lim = dyn_limit(n_dev, n_max);
    const uint64_t base = (uint64_t)blockIdx.x * kCmpTile;
    uint32_t v[1] = {0};
#pragma unroll
    for (int q = 0; q < kCmpItems; q++) v[0] += unique_head(a, base + q * 256 + threadIdx.x, lim) ? 1u : 0u;
    block_sum_n<1>(v, lds);
    if (threadIdx.x == 0) tile_cnt[blockIdx.x] = v[0];
}

__global__ void __launch_bounds__(256)
k_unique_scatter(const uint64_t *__restrict__ a, uint64_t n_max, const uint32_t *__restrict__ n_dev,
                 const uint32_t *__restrict__ tile_cnt, uint32_t ntiles, uint64_t *__restrict__ out,
                 uint32_t *__restrict__ count_dev) {
    __shared__ uint32_t lds[256 / kWave + 1];
    uint32_t before, total;
    tile_prefix(tile_cnt, ntiles, blockIdx.x, &before, &total);
    if (blockIdx.x == 0 && threadIdx.x == 0) *count_dev = total;
    const uint64_t lim = dyn_limit(n_dev, n_max);
    const uint64_t base = (uint64_t)blockIdx.x * kCmpTile + (uint64_t)threadIdx.x * kCmpItems;
    uint32_t f = 0;
#pragma unroll
    for (int q = 0; q < kCmpItems; q++) f |= (unique_head(a, base + q, lim) ? 1u : 0u) << q;
    uint32_t tot;
    uint32_t pos = before + block_exclusive_scan(__popc(f), &tot, lds);
#pragma unroll
    for (int q = 0; q < kCmpItems; q++)
        if (f & (1u << q)) out[pos++] = a[base + q];
}

// pending updates per tile, plus the level's statistics per tile:
// st[0..ntiles) pending, then done, noop, merged-segment heads
__global__ void __launch_bounds__(256)
k_pending_count(const uint8_t *__restrict__ status, const uint32_t *__restrict__ n_dev, uint64_t n_max,
                uint32_t ntiles, uint32_t *__restrict__ st) {
    __shared__ uint32_t lds[4][256 / kWave];
    const uint64_t n = dyn_limit(n_dev, n_max);
    const uint64_t base = (uint64_t)blockIdx.x * kCmpTile;
    uint32_t v[4] = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < kCmpItems; q++) {
        const uint64_t i = base + q * 256 + threadIdx.x;
        if (i < n) {
            const uint8_t x = status[i];
            const uint8_t state = x & kStateMask;
            v[0] += state == kPending;
            v[1] += state == kDone;
            v[2] += state == kNoop;
            v[3] += (x & kHead) ? 1u : 0u;
        }
    }
    block_sum_n<4>(v, lds);
    if (threadIdx.x < 4) st[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = v[threadIdx.x];
}

__global__ void __launch_bounds__(256)
k_pending_scatter(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ leaf,
                  const uint8_t *__restrict__ status, const uint32_t *__restrict__ n_dev, uint64_t n_max,
                  const uint32_t *__restrict__ st, uint32_t ntiles, uint64_t *__restrict__ keys_out,
                  uint32_t *__restrict__ leaf_out, uint8_t *__restrict__ status_out,
                  uint32_t *__restrict__ count_dev, int del, uint64_t cap_h, Ctl *__restrict__ ctl) {
    __shared__ uint32_t lds[256 / kWave + 1];
    __shared__ uint32_t red[3][256 / kWave];
    uint32_t before, total;
    tile_prefix(st, ntiles, blockIdx.x, &before, &total);
    if (blockIdx.x == 0 && !ctl && threadIdx.x == 0) *count_dev = total;
    if (blockIdx.x == 0 && ctl) {
        // the level's statistics, once
        uint32_t v[3] = {0, 0, 0};
        for (uint32_t i = threadIdx.x; i < ntiles; i += blockDim.x) {
            v[0] += st[ntiles + i];
            v[1] += st[2 * (uint64_t)ntiles + i];
            v[2] += st[3 * (uint64_t)ntiles + i];
        }
        block_sum_n<3>(v, red);
        if (threadIdx.x == 0) {
            *count_dev = total;
            if (v[0]) {
                atomicAdd((unsigned long long *)&ctl->applied, (unsigned long long)v[0]);
                atomicAdd((unsigned long long *)&ctl->dn,
                          (unsigned long long)(del ? -(int64_t)v[0] : (int64_t)v[0]));
            }
            if (v[1]) atomicAdd((unsigned long long *)&ctl->noops, (unsigned long long)v[1]);
            if (v[2]) {
                atomicAdd(&ctl->segs, v[2]);
                atomicAdd((unsigned long long *)&ctl->rewritten, (unsigned long long)(v[2] * cap_h));
            }
        }
    }
    const uint64_t n = dyn_limit(n_dev, n_max);
    const uint64_t base = (uint64_t)blockIdx.x * kCmpTile + (uint64_t)threadIdx.x * kCmpItems;
    uint32_t f = 0;
#pragma unroll
    for (int q = 0; q < kCmpItems; q++) {
        const uint64_t i = base + q;
        f |= (i < n && (status[i] & kStateMask) == kPending ? 1u : 0u) << q;
    }
    uint32_t tot;
    uint32_t pos = before + block_exclusive_scan(__popc(f), &tot, lds);
#pragma unroll
    for (int q = 0; q < kCmpItems; q++)
        if (f & (1u << q)) {
            keys_out[pos] = keys[base + q];
            leaf_out[pos] = leaf[base + q];
            status_out[pos] = kPending;
            pos++;
        }
}

__global__ void k_flag_edges(const uint64_t *__restrict__ slots, uint64_t cap,
                             uint32_t *__restrict__ flags) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    uint64_t k = slots[i];
    flags[i] = is_edge_entry(k) ? 1u : 0u;   // live, not a guard
}

__global__ void k_scatter_edges(const uint64_t *__restrict__ slots, uint64_t cap,
                                const uint32_t *__restrict__ pos, uint64_t *__restrict__ out) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    uint64_t k = slots[i];
    if (is_edge_entry(k)) out[pos[i]] = k;
}

}  // namespace

namespace gpma_host {

size_t scan_tmp_words(uint64_t n) { return div_up(n ? n : 1, kScanTile) + 1; }

void scan_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *total_dev, uint32_t *tmp,
              hipStream_t s) {
    if (n == 0) {
        if (total_dev) hipMemsetAsync(total_dev, 0, sizeof(uint32_t), s);
        return;
    }
    if (n <= kScanSingleMax) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, s, in, out, n, total_dev);
        return;
    }
    uint64_t ntiles = div_up(n, kScanTile);
    hipLaunchKernelGGL(k_scan_reduce, dim3((uint32_t)ntiles), dim3(kScanThreads), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, tmp, ntiles, total_dev);
    hipLaunchKernelGGL(k_scan_apply, dim3((uint32_t)ntiles), dim3(kScanThreads), 0, s, in, out, n,
                       tmp);
}

void scan_u32_one_block(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *total_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, s, in, out, n, total_dev);
}

// keys per tile: 256 threads x 64-key chunks per wave x CH
static uint64_t sort_tile(uint64_t n, int small_chunks) {
    return (uint64_t)kSortThreads * (n <= kSmallSortMax ? (uint64_t)small_chunks : (uint64_t)kChunksLarge);
}

size_t radix_tmp_words(uint64_t n) {
    // sized for the smallest tiles a caller may pick
    uint64_t ntiles = div_up(n ? n : 1, sort_tile(n, kChunksMin));
    uint64_t m = 256 * ntiles;
    return m + scan_tmp_words(m);
}

template <int CH>
static void radix_pass(const uint64_t *src, uint64_t n, const uint32_t *n_dev, DigitMap dm, uint32_t bits,
                       uint64_t ntiles, uint32_t *counts, uint32_t *stmp, Ctl *check, uint64_t *dst, hipStream_t s) {
    const uint64_t mm = (uint64_t)(dm.mask + 1) * ntiles;
    // up to kFuseTiles tiles the downsweep derives its offsets itself
    const int fuse = ntiles <= kFuseTiles;
    hipLaunchKernelGGL(k_radix_upsweep<CH>, dim3((uint32_t)ntiles), dim3(kSortThreads), 0, s, src, n, n_dev, dm,
                       (uint32_t)ntiles, fuse, counts, check);
    if (!fuse) scan_u32(counts, counts, mm, nullptr, stmp, s);
    hipLaunchKernelGGL(k_radix_downsweep<CH>, dim3((uint32_t)ntiles), dim3(kSortThreads), 0, s, src, n, n_dev, dm,
                       bits, (uint32_t)ntiles, counts, fuse, dst);
}

const uint64_t *radix_sort_keys(const uint64_t *in, uint64_t n, uint32_t sbits, uint32_t dbits,
                                uint32_t V, uint64_t *buf_a, uint64_t *buf_b, uint32_t *tmp,
                                hipStream_t s, const uint32_t *n_dev, Ctl *check, int small_chunks) {
    if (small_chunks != 2 && small_chunks != 8) small_chunks = kChunksSmall;
    uint32_t total = sbits + dbits;
    if (total == 0) total = 1;
    uint32_t passes = (total + 7) / 8;
    uint32_t bits = (total + passes - 1) / passes;
    const bool small = n <= kSmallSortMax;
    const int ch = small ? small_chunks : kChunksLarge;
    uint64_t ntiles = div_up(n ? n : 1, sort_tile(n, small_chunks));
    uint64_t m = 256 * ntiles;
    uint32_t *counts = tmp;
    uint32_t *stmp = tmp + m;
    const uint64_t *src = in;
    uint64_t *dst = buf_a;
    for (uint32_t p = 0; p < passes; p++) {
        DigitMap dm{p * bits, (1u << bits) - 1u, dbits, V};
        Ctl *chk = p == 0 ? check : nullptr;
        switch (ch) {
            case 2: radix_pass<2>(src, n, n_dev, dm, bits, ntiles, counts, stmp, chk, dst, s); break;
            case 8: radix_pass<8>(src, n, n_dev, dm, bits, ntiles, counts, stmp, chk, dst, s); break;
            case kChunksLarge: radix_pass<kChunksLarge>(src, n, n_dev, dm, bits, ntiles, counts, stmp, chk, dst, s); break;
            default: radix_pass<kChunksSmall>(src, n, n_dev, dm, bits, ntiles, counts, stmp, chk, dst, s); break;
        }
        src = dst;
        dst = (dst == buf_a) ? buf_b : buf_a;
    }
    return src;
}

void unique_sorted_dyn(const uint64_t *in, const uint32_t *n_dev, uint64_t n_max, uint64_t *out,
                       uint32_t *count_dev, uint32_t *flags, uint32_t *tmp, hipStream_t s) {
    if (n_max == 0) {
        hipMemsetAsync(count_dev, 0, sizeof(uint32_t), s);
        return;
    }
    const uint64_t ntiles = div_up(n_max, kCmpTile);
    if (ntiles <= kCmpMaxTiles) {
        hipLaunchKernelGGL(k_unique_count, dim3((uint32_t)ntiles), dim3(256), 0, s, in, n_max, n_dev, tmp);
        hipLaunchKernelGGL(k_unique_scatter, dim3((uint32_t)ntiles), dim3(256), 0, s, in, n_max, n_dev, tmp,
                           (uint32_t)ntiles, out, count_dev);
        return;
    }
    uint32_t g = (uint32_t)div_up(n_max, 256);
    hipLaunchKernelGGL(k_flag_unique, dim3(g), dim3(256), 0, s, in, n_max, n_dev, flags);
    scan_u32(flags, flags, n_max, count_dev, tmp, s);
    hipLaunchKernelGGL(k_scatter_unique, dim3(g), dim3(256), 0, s, in, n_max, n_dev, flags, out);
}

void unique_sorted(const uint64_t *in, uint64_t n, uint64_t *out, uint32_t *count_dev,
                   uint32_t *flags, uint32_t *tmp, hipStream_t s) {
    unique_sorted_dyn(in, nullptr, n, out, count_dev, flags, tmp, s);
}

void compact_pending(const uint64_t *keys, const uint32_t *leaf, const uint8_t *status,
                     const uint32_t *n_dev, uint64_t n_max, uint64_t *keys_out, uint32_t *leaf_out,
                     uint8_t *status_out, uint32_t *count_dev, uint32_t *flags, uint32_t *tmp,
                     bool del, uint64_t cap_h, Ctl *ctl, hipStream_t s) {
    if (n_max == 0) {
        hipMemsetAsync(count_dev, 0, sizeof(uint32_t), s);
        return;
    }
    const uint64_t ntiles = div_up(n_max, kCmpTile);
    if (ntiles <= kCmpMaxTiles) {
        hipLaunchKernelGGL(k_pending_count, dim3((uint32_t)ntiles), dim3(256), 0, s, status, n_dev, n_max,
                           (uint32_t)ntiles, tmp);
        hipLaunchKernelGGL(k_pending_scatter, dim3((uint32_t)ntiles), dim3(256), 0, s, keys, leaf, status, n_dev,
                           n_max, tmp, (uint32_t)ntiles, keys_out, leaf_out, status_out, count_dev, del ? 1 : 0,
                           cap_h, ctl);
        return;
    }
    uint32_t g = (uint32_t)div_up(n_max, 256);
    const uint32_t gf = g < 64 ? g : 64;   // few blocks: one stats atomic each
    hipLaunchKernelGGL(k_flag_pending, dim3(gf), dim3(256), 0, s, status, n_dev, n_max, flags,
                       del ? 1 : 0, cap_h, ctl);
    scan_u32(flags, flags, n_max, count_dev, tmp, s);
    hipLaunchKernelGGL(k_scatter_pending, dim3(g), dim3(256), 0, s, keys, leaf, status, n_dev, n_max,
                       flags, keys_out, leaf_out, status_out);
}

void compact_edges(const uint64_t *slots, uint64_t cap, uint64_t *out, uint32_t *count_dev,
                   uint32_t *flags, uint32_t *tmp, hipStream_t s) {
    uint32_t g = (uint32_t)div_up(cap, 256);
    hipLaunchKernelGGL(k_flag_edges, dim3(g), dim3(256), 0, s, slots, cap, flags);
    scan_u32(flags, flags, cap, count_dev, tmp, s);
    hipLaunchKernelGGL(k_scatter_edges, dim3(g), dim3(256), 0, s, slots, cap, flags, out);
}

}  // namespace gpma_host
