// Splitter (sample) sort of the update keys of a batch window, for inputs up
// to kSsMaxKeys keys: ascending 64-bit order -- the order of the LSD radix
// sort of the compressed key (src << dbits) | dst for every key a window
// holds (dst < V) -- in four or six launches instead of two per 8-bit digit.
// The paper sorts each batch with a radix sort (Section 5.2); sorting a window
// of batches this way is our design.
//
//   1. one workgroup sorts a regular sample of the keys (bitonic, in
//      registers and LDS) and picks B - 1 splitters (B buckets of about
//      kSsTarget keys); the paired form takes them from its caller, whose
//      copying launch samples them on the side;
//   2. each 2048-key tile counts its keys per bucket (binary search over the
//      splitters in LDS);
//   3. each tile scatters its keys to their buckets; it derives its offsets
//      from the counts itself when they are few (else one scan of the counts
//      runs first);
//   4. one 1024-thread workgroup per bucket sorts it (bitonic) and writes it
//      back in place; a bucket larger than kSsLdsKeys (many equal keys) is
//      sorted by the same workgroup in global memory, a stable LSD radix pass
//      of 1024 keys a round.
//
// Keys equal to one another always fall in one bucket, so the buckets in
// order, each sorted, are the sorted input.  Every launch reads the key count
// from the device, so the sequence can be captured in a graph once per size
// class.
#include "common.h"
#include "pair.h"
#include "bitonic.h"

using namespace gpma_dev;

namespace {

constexpr int kSsThreads = 1024;                         // sample and bucket workgroups
constexpr int kSsWaves = kSsThreads / kWave;             // 16
constexpr uint32_t kSsLdsKeys = 4096;                    // keys a bucket workgroup sorts in registers / LDS
constexpr int kSsTileThreads = 1024;
constexpr int kSsTileItems = 2;
constexpr uint32_t kSsTile = kSsTileThreads * kSsTileItems;   // 2048 keys a count / scatter tile
constexpr uint32_t kSsMaxBuckets = 1024;
constexpr uint32_t kSsOversample = 4;                    // sample keys per bucket
constexpr uint64_t kSsMaxKeys = 1ull << 20;
constexpr uint64_t kSsTarget = 512;                      // keys a bucket holds on average (at most)
constexpr uint64_t kSsFuseCounts = 1ull << 14;           // counts a scatter tile prefixes itself

__host__ __device__ inline uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

__device__ __forceinline__ uint64_t dyn_n(const uint32_t *n_dev, uint64_t n_max) {
    if (!n_dev) return n_max;
    const uint64_t n = *n_dev;
    return n < n_max ? n : n_max;
}

// the m <= 1024*R keys src[0..m) sorted into dst[0..m) (src may equal dst)
template <int R>
__device__ void sort_small(const uint64_t *src, uint64_t *dst, uint32_t m, uint64_t *lds) {
    uint32_t P = kWave;
    while (P < m) P <<= 1;
    uint64_t k[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint32_t idx = (uint32_t)r * 1024u + threadIdx.x;
        k[r] = idx < m ? src[idx] : ~0ull;   // padding sorts last
    }
    block_bitonic<R>(k, lds, P);
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint32_t idx = (uint32_t)r * 1024u + threadIdx.x;
        if (idx < m) dst[idx] = k[r];
    }
}

// number of splitters below c (the first j with spl[j] >= c)
__device__ __forceinline__ uint32_t bucket_of(const uint64_t *spl, uint32_t nspl, uint64_t c) {
    uint32_t lo = 0, hi = nspl;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (spl[mid] < c) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// 1. sample -> splitters, one workgroup
struct SsSplitArgs {
    const uint64_t *keys;
    uint64_t n_max;
    const uint32_t *n_dev;
    uint32_t B;
    uint64_t *spl;
};

template <int R>
struct SsSplittersOp {
    using Args = SsSplitArgs;
    static __device__ __forceinline__ void run(const Args &a) {
        const uint64_t *__restrict__ keys = a.keys;
        const uint64_t n_max = a.n_max;
        const uint32_t *__restrict__ n_dev = a.n_dev;
        const uint32_t B = a.B;
        uint64_t *__restrict__ spl = a.spl;
        __shared__ uint64_t lds[1024 * R];
        const uint64_t n = dyn_n(n_dev, n_max);
        if (B < 2) return;
        if (n == 0) {
            for (uint32_t j = threadIdx.x; j + 1 < B; j += kSsThreads) spl[j] = ~0ull;
            return;
        }
        constexpr uint32_t S = 1024u * R;   // sample size (B * kSsOversample, at least 1024)
        uint64_t k[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            const uint32_t idx = (uint32_t)r * 1024u + threadIdx.x;
            k[r] = keys[((uint64_t)idx * n) / S];
        }
        block_bitonic<R>(k, lds, S);
#pragma unroll
        for (int r = 0; r < R; r++) lds[(uint32_t)r * 1024u + threadIdx.x] = k[r];
        __syncthreads();
        for (uint32_t j = threadIdx.x; j + 1 < B; j += kSsThreads) spl[j] = lds[((uint64_t)(j + 1) * S) / B];
    }
};

template <int R>
__global__ void __launch_bounds__(kSsThreads)
k_ss_splitters(const uint64_t *__restrict__ keys, uint64_t n_max, const uint32_t *__restrict__ n_dev, uint32_t B,
               uint64_t *__restrict__ spl) {
    SsSplittersOp<R>::run(SsSplitArgs{keys, n_max, n_dev, B, spl});
}

// 2. per-tile bucket counts, bucket-major: cnt[b * ntiles + tile]
struct SsCountOp {
    struct Args {
        const uint64_t *keys;
        uint64_t n_max;
        const uint32_t *n_dev;
        const uint64_t *spl;
        uint32_t B;
        uint32_t ntiles;
        uint32_t *cnt;
        uint32_t *bump;    // optional: a counter advanced by one once the keys are in place
        uint32_t *clear;   // optional (with bump): a word set to zero at the same time
    };
    static __device__ __forceinline__ void run(const Args &a) {
        if (a.bump && blockIdx.x == 0 && threadIdx.x == 0) {
            *a.bump += 1;
            *a.clear = 0;
        }
        const uint64_t *__restrict__ keys = a.keys;
        uint64_t n_max = a.n_max;
        const uint32_t *__restrict__ n_dev = a.n_dev;
        const uint64_t *__restrict__ spl = a.spl;
        uint32_t B = a.B;
        uint32_t ntiles = a.ntiles;
        uint32_t *__restrict__ cnt = a.cnt;
        __shared__ uint64_t s_spl[kSsMaxBuckets];
        __shared__ uint32_t hist[kSsMaxBuckets];
        const uint64_t n = dyn_n(n_dev, n_max);
        for (uint32_t j = threadIdx.x; j < B; j += kSsTileThreads) {
            hist[j] = 0;
            if (j + 1 < B) s_spl[j] = spl[j];
        }
        __syncthreads();
        const uint64_t base = (uint64_t)blockIdx.x * kSsTile;
#pragma unroll
        for (int q = 0; q < kSsTileItems; q++) {
            const uint64_t i = base + (uint64_t)q * kSsTileThreads + threadIdx.x;
            if (i < n) atomicAdd(&hist[bucket_of(s_spl, B - 1, keys[i])], 1u);
        }
        __syncthreads();
        for (uint32_t j = threadIdx.x; j < B; j += kSsTileThreads) cnt[(uint64_t)j * ntiles + blockIdx.x] = hist[j];
    }
};

__global__ void __launch_bounds__(kSsTileThreads)
k_ss_count(const uint64_t *__restrict__ keys, uint64_t n_max, const uint32_t *__restrict__ n_dev,
           const uint64_t *__restrict__ spl, uint32_t B, uint32_t ntiles, uint32_t *__restrict__ cnt,
           uint32_t *bump, uint32_t *clear) {
    SsCountOp::run(SsCountOp::Args{keys, n_max, n_dev, spl, B, ntiles, cnt, bump, clear});
}

// 3. scatter each tile's keys to their buckets (order within a bucket is
// free: the bucket is sorted next).  fused: cnt holds the raw counts; the
// tile derives its offsets (buckets before b over all tiles, bucket b over
// earlier tiles) and block 0 writes the bucket starts bst[0..B].  Else cnt
// holds the exclusive scan of the counts.
struct SsScatterOp {
    struct Args {
        const uint64_t *keys;
        uint64_t n_max;
        const uint32_t *n_dev;
        const uint64_t *spl;
        uint32_t B;
        uint32_t ntiles;
        const uint32_t *cnt;
        int fused;
        uint32_t *bst;
        uint64_t *out;
    };
    static __device__ __forceinline__ void run(const Args &a) {
        const uint64_t *__restrict__ keys = a.keys;
        uint64_t n_max = a.n_max;
        const uint32_t *__restrict__ n_dev = a.n_dev;
        const uint64_t *__restrict__ spl = a.spl;
        uint32_t B = a.B;
        uint32_t ntiles = a.ntiles;
        const uint32_t *__restrict__ cnt = a.cnt;
        int fused = a.fused;
        uint32_t *__restrict__ bst = a.bst;
        uint64_t *__restrict__ out = a.out;
        __shared__ uint64_t s_spl[kSsMaxBuckets];
        __shared__ uint32_t cur[kSsMaxBuckets];
        __shared__ uint32_t s_tot[kSsMaxBuckets];
        __shared__ uint32_t scan_lds[kSsTileThreads / kWave + 1];
        const uint64_t n = dyn_n(n_dev, n_max);
        const uint64_t base = (uint64_t)blockIdx.x * kSsTile;
        if (base >= n && !(fused && blockIdx.x == 0)) return;   // block-uniform
        for (uint32_t j = threadIdx.x; j + 1 < B; j += kSsTileThreads) s_spl[j] = spl[j];
        if (fused) {
            // bucket b's total and its count in earlier tiles (a 16-byte aligned
            // row of ntiles words per bucket)
            for (uint32_t b = threadIdx.x; b < B; b += kSsTileThreads) {
                const uint32_t *row = cnt + (uint64_t)b * ntiles;
                uint32_t tot = 0, before = 0;
                if ((ntiles & 3u) == 0) {
                    const uint4 *r4 = reinterpret_cast<const uint4 *>(row);
#pragma unroll 4
                    for (uint32_t x4 = 0; x4 < ntiles / 4; x4++) {
                        const uint4 c = r4[x4];
                        const uint32_t x = 4 * x4;
                        tot += c.x + c.y + c.z + c.w;
                        before += (x < blockIdx.x ? c.x : 0u) + (x + 1 < blockIdx.x ? c.y : 0u) +
                                  (x + 2 < blockIdx.x ? c.z : 0u) + (x + 3 < blockIdx.x ? c.w : 0u);
                    }
                } else {
                    for (uint32_t x = 0; x < ntiles; x++) {
                        const uint32_t c = row[x];
                        tot += c;
                        before += x < blockIdx.x ? c : 0u;
                    }
                }
                s_tot[b] = tot;
                cur[b] = before;
            }
            __syncthreads();
            // bucket starts: thread t prefixes kPer buckets from kPer*t (B <= 1024)
            constexpr uint32_t kPer = kSsMaxBuckets / kSsTileThreads;
            uint32_t mine = 0;
#pragma unroll
            for (uint32_t q = 0; q < kPer; q++) {
                const uint32_t b = threadIdx.x * kPer + q;
                mine += b < B ? s_tot[b] : 0u;
            }
            uint32_t all;
            uint32_t run = block_exclusive_scan(mine, &all, scan_lds);
#pragma unroll
            for (uint32_t q = 0; q < kPer; q++) {
                const uint32_t b = threadIdx.x * kPer + q;
                if (b < B) {
                    cur[b] += run;
                    if (blockIdx.x == 0) bst[b] = run;
                    run += s_tot[b];
                }
            }
            if (blockIdx.x == 0 && threadIdx.x == 0) bst[B] = all;
        } else {
            for (uint32_t j = threadIdx.x; j < B; j += kSsTileThreads) cur[j] = cnt[(uint64_t)j * ntiles + blockIdx.x];
        }
        __syncthreads();
        if (base >= n) return;
#pragma unroll
        for (int q = 0; q < kSsTileItems; q++) {
            const uint64_t i = base + (uint64_t)q * kSsTileThreads + threadIdx.x;
            if (i < n) {
                const uint64_t k = keys[i];
                out[atomicAdd(&cur[bucket_of(s_spl, B - 1, k)], 1u)] = k;
            }
        }
    }
};

__global__ void __launch_bounds__(kSsTileThreads)
k_ss_scatter(const uint64_t *__restrict__ keys, uint64_t n_max, const uint32_t *__restrict__ n_dev,
             const uint64_t *__restrict__ spl, uint32_t B, uint32_t ntiles, const uint32_t *__restrict__ cnt,
             int fused, uint32_t *__restrict__ bst, uint64_t *__restrict__ out) {
    SsScatterOp::run(SsScatterOp::Args{keys, n_max, n_dev, spl, B, ntiles, cnt, fused, bst, out});
}

// 4. sort bucket b = blockIdx.x, [starts[b*stride], starts[(b+1)*stride])
// of `in` (the last bucket ends at n), into the same range of `out`
struct SsBucketOp {
    struct Args {
        uint64_t *in;
        uint64_t *out;
        uint64_t n_max;
        const uint32_t *n_dev;
        const uint32_t *starts;
        uint32_t stride;
        uint32_t B;
        uint32_t dbits;
        uint32_t bits;
        uint32_t passes;
    };
    static __device__ __forceinline__ void run(const Args &a) {
        uint64_t *__restrict__ in = a.in;
        uint64_t *__restrict__ out = a.out;
        uint64_t n_max = a.n_max;
        const uint32_t *__restrict__ n_dev = a.n_dev;
        const uint32_t *__restrict__ starts = a.starts;
        uint32_t stride = a.stride;
        uint32_t B = a.B;
        uint32_t dbits = a.dbits;
        uint32_t bits = a.bits;
        uint32_t passes = a.passes;
        __shared__ uint64_t lds[kSsLdsKeys];
        __shared__ uint32_t wcnt[kSsWaves][256];
        __shared__ uint32_t goff[256];
        __shared__ uint32_t scan_lds[kSsThreads / kWave + 1];
        const uint64_t n = dyn_n(n_dev, n_max);
        const uint32_t b = blockIdx.x;
        const uint64_t lo = starts[(uint64_t)b * stride];
        const uint64_t hi = b + 1 < B ? (uint64_t)starts[(uint64_t)(b + 1) * stride] : n;
        if (hi <= lo) return;   // block-uniform
        const uint64_t m = hi - lo;
        if (m <= 1024) { sort_small<1>(in + lo, out + lo, (uint32_t)m, lds); return; }
        if (m <= 2048) { sort_small<2>(in + lo, out + lo, (uint32_t)m, lds); return; }
        if (m <= kSsLdsKeys) { sort_small<4>(in + lo, out + lo, (uint32_t)m, lds); return; }
        // A bucket larger than that: stable LSD passes over the compressed key
        // (src << dbits) | dst between this bucket's range of `in` and of `out`,
        // 1024 keys a round (position r + threadIdx.x).
        const uint32_t lane = __lane_id();
        const uint32_t w = threadIdx.x / kWave;
        const uint64_t ltmask = lanemask_lt();
        const uint32_t mask = (1u << bits) - 1u;
        auto digit = [&](uint64_t k, uint32_t shift) {
            return (uint32_t)((((k >> 32) << dbits) | (uint64_t)(uint32_t)k) >> shift) & mask;
        };
        uint64_t *src = in + lo;
        uint64_t *dst = out + lo;
        for (uint32_t p = 0; p < passes; p++) {
            const uint32_t shift = p * bits;
            if (threadIdx.x < 256) goff[threadIdx.x] = 0;
            __syncthreads();
            for (uint64_t i = threadIdx.x; i < m; i += kSsThreads) atomicAdd(&goff[digit(src[i], shift)], 1u);
            __syncthreads();
            {
                const uint32_t h = threadIdx.x < 256 ? goff[threadIdx.x] : 0u;
                uint32_t all;
                const uint32_t ex = block_exclusive_scan(h, &all, scan_lds);
                if (threadIdx.x < 256) goff[threadIdx.x] = ex;
            }
            for (uint64_t r = 0; r < m; r += kSsThreads) {
                for (uint32_t i = threadIdx.x; i < kSsWaves * 256; i += kSsThreads) (&wcnt[0][0])[i] = 0;
                __syncthreads();
                const uint64_t i = r + threadIdx.x;
                const bool valid = i < m;
                const uint64_t key = valid ? src[i] : 0;
                const uint32_t d = digit(key, shift);
                uint64_t mm = __ballot(valid);
                for (uint32_t bb = 0; bb < bits; bb++) {
                    const uint32_t bit = (d >> bb) & 1u;
                    const uint64_t x = __ballot(bit);
                    mm &= bit ? x : ~x;
                }
                const uint32_t rank = (uint32_t)__popcll(mm & ltmask);
                if (valid && (uint32_t)(__ffsll((unsigned long long)mm) - 1) == lane) wcnt[w][d] = (uint32_t)__popcll(mm);
                __syncthreads();
                if (valid) {
                    uint32_t before = 0;
                    for (uint32_t ww = 0; ww < w; ww++) before += wcnt[ww][d];
                    dst[goff[d] + before + rank] = key;
                }
                __syncthreads();
                if (threadIdx.x < 256) {
                    uint32_t t = 0;
                    for (uint32_t ww = 0; ww < (uint32_t)kSsWaves; ww++) t += wcnt[ww][threadIdx.x];
                    goff[threadIdx.x] += t;
                }
                __syncthreads();
            }
            uint64_t *t = src;
            src = dst;
            dst = t;
        }
        if (src != out + lo)   // an even number of passes: the keys are in `in`
            for (uint64_t i = threadIdx.x; i < m; i += kSsThreads) out[lo + i] = src[i];
    }
};

__global__ void __launch_bounds__(1024)
k_ss_bucket(uint64_t *__restrict__ in, uint64_t *__restrict__ out, uint64_t n_max, const uint32_t *__restrict__ n_dev,
            const uint32_t *__restrict__ starts, uint32_t stride, uint32_t B, uint32_t dbits,
            uint32_t bits, uint32_t passes) {
    SsBucketOp::run(SsBucketOp::Args{in, out, n_max, n_dev, starts, stride, B, dbits, bits, passes});
}

uint32_t ss_buckets(uint64_t n_max) {
    uint64_t b = 1;
    while (b * kSsTarget < n_max && b < kSsMaxBuckets) b <<= 1;
    return (uint32_t)b;
}

}  // namespace

namespace gpma_host {

uint32_t splitter_buckets(uint64_t n_max) { return ss_buckets(n_max); }

uint64_t *splitter_spl(uint32_t *tmp) { return reinterpret_cast<uint64_t *>(tmp); }

uint32_t splitter_sample_size(uint64_t n_max) {
    const uint32_t S = ss_buckets(n_max) * kSsOversample;
    return S <= 1024 ? 1024 : (S <= 2048 ? 2048 : 4096);
}

bool splitter_sort_fits(uint64_t n_max) { return n_max >= 1 && n_max <= kSsMaxKeys; }

size_t splitter_tmp_words(uint64_t n_max) {
    if (!splitter_sort_fits(n_max)) return 0;
    const uint64_t cw = (uint64_t)ss_buckets(n_max) * div_up(n_max, kSsTile);
    return 2 * kSsMaxBuckets + (kSsMaxBuckets + 4) + cw + scan_tmp_words(cw);
}

const uint64_t *splitter_sort_keys(const uint64_t *in, uint64_t n_max, const uint32_t *n_dev, uint32_t sbits,
                                   uint32_t dbits, uint32_t V, uint64_t *buf_a, uint64_t *buf_b, uint32_t *tmp,
                                   hipStream_t s, uint32_t *bump, uint32_t *clear) {
    uint32_t total = sbits + dbits;
    if (total == 0) total = 1;
    const uint32_t passes = (total + 7) / 8;
    const uint32_t bits = (total + passes - 1) / passes;
    // the result lands where the radix sort's would (an odd pass count: buf_a)
    uint64_t *fin = (passes & 1) ? buf_a : buf_b;
    uint64_t *mid = fin == buf_a ? buf_b : buf_a;
    const uint32_t B = ss_buckets(n_max);
    const uint64_t ntiles = div_up(n_max, kSsTile);
    const uint64_t cw = (uint64_t)B * ntiles;
    uint64_t *spl = reinterpret_cast<uint64_t *>(tmp);   // 2 * kSsMaxBuckets words
    uint32_t *bst = tmp + 2 * kSsMaxBuckets;             // kSsMaxBuckets + 1 words
    uint32_t *cnt = bst + kSsMaxBuckets + 4;             // 16-byte aligned rows
    uint32_t *stmp = cnt + cw;
    const uint32_t S = B * kSsOversample;
    if (S <= 1024)
        hipLaunchKernelGGL(k_ss_splitters<1>, dim3(1), dim3(kSsThreads), 0, s, in, n_max, n_dev, B, spl);
    else if (S <= 2048)
        hipLaunchKernelGGL(k_ss_splitters<2>, dim3(1), dim3(kSsThreads), 0, s, in, n_max, n_dev, B, spl);
    else
        hipLaunchKernelGGL(k_ss_splitters<4>, dim3(1), dim3(kSsThreads), 0, s, in, n_max, n_dev, B, spl);
    hipLaunchKernelGGL(k_ss_count, dim3((uint32_t)ntiles), dim3(kSsTileThreads), 0, s, in, n_max, n_dev, spl, B,
                       (uint32_t)ntiles, cnt, bump, clear);
    const bool fused = cw <= kSsFuseCounts;
    if (!fused) scan_u32(cnt, cnt, cw, nullptr, stmp, s);
    hipLaunchKernelGGL(k_ss_scatter, dim3((uint32_t)ntiles), dim3(kSsTileThreads), 0, s, in, n_max, n_dev, spl, B,
                       (uint32_t)ntiles, cnt, fused ? 1 : 0, bst, mid);
    hipLaunchKernelGGL(k_ss_bucket, dim3(B), dim3(kSsThreads), 0, s, mid, fin, n_max, n_dev, fused ? bst : cnt,
                       fused ? 1u : (uint32_t)ntiles, B, dbits, bits, passes);
    return fin;
}

bool splitter_sort_pairable(uint64_t n_max) {
    return splitter_sort_fits(n_max) && (uint64_t)ss_buckets(n_max) * div_up(n_max, kSsTile) <= kSsFuseCounts;
}

// Two sorts of the same size in one set of launches (index 0 and 1 of each
// array argument); the results land as splitter_sort_keys's would, returned
// as 0 (buf_a) or 1 (buf_b).
int splitter_sort_keys2(const uint64_t *const in[2], uint64_t n_max, const uint32_t *const n_dev[2], uint32_t sbits,
                        uint32_t dbits, uint64_t *const buf_a[2], uint64_t *const buf_b[2], uint32_t *const tmp[2],
                        hipStream_t s, uint32_t *const bump[2], uint32_t *const clear[2]) {
    uint32_t total = sbits + dbits;
    if (total == 0) total = 1;
    const uint32_t passes = (total + 7) / 8;
    const uint32_t bits = (total + passes - 1) / passes;
    const int which = (passes & 1) ? 0 : 1;
    const uint32_t B = ss_buckets(n_max);
    const uint64_t ntiles = div_up(n_max, kSsTile);
    SsCountOp::Args ca[2];
    SsScatterOp::Args sa[2];
    SsBucketOp::Args ba[2];
    for (int k = 0; k < 2; k++) {
        uint64_t *fin = which ? buf_b[k] : buf_a[k];
        uint64_t *mid = which ? buf_a[k] : buf_b[k];
        uint64_t *spl = reinterpret_cast<uint64_t *>(tmp[k]);
        uint32_t *bst = tmp[k] + 2 * kSsMaxBuckets;
        uint32_t *cnt = bst + kSsMaxBuckets + 4;
        ca[k] = {in[k], n_max, n_dev[k], spl, B, (uint32_t)ntiles, cnt, bump ? bump[k] : nullptr,
                 bump ? clear[k] : nullptr};
        sa[k] = {in[k], n_max, n_dev[k], spl, B, (uint32_t)ntiles, cnt, 1, bst, mid};
        ba[k] = {mid, fin, n_max, n_dev[k], bst, 1u, B, dbits, bits, passes};
    }
    launch_pair<SsCountOp, kSsTileThreads>((uint32_t)ntiles, ca[0], ca[1], s);
    launch_pair<SsScatterOp, kSsTileThreads>((uint32_t)ntiles, sa[0], sa[1], s);
    launch_pair<SsBucketOp, kSsThreads>(B, ba[0], ba[1], s);
    return which;
}

}  // namespace gpma_host

