// PageRank SpMV by destination bins (propagation blocking) over the
// src-major slot array (Section 6.1, PageRank as repeated SpMV; Section 4.2,
// algorithms read the array in place, skipping gaps and guards).
//
// A stored edge u->v adds contrib[u] to y[v].  Read along the src-major
// array, contrib[u] is a near-sequential read but y[v] is a random update;
// read along a dst-major array it is the other way round.  Either way one
// side is a random access per edge into a vector far larger than L2.  Here
// the edge stream is instead split by destination into fine bins of 16384
// vertices, whose slice of y (128 KiB of fp64) fits one workgroup's LDS:
//   count (once per call): per slot range, how many edges fall in each fine
//          bin; an exclusive scan of the bin-major count matrix gives every
//          (bin, range) pair its place in the record array.  The same pass
//          packs each range's edges (gaps, guards and marked entries dropped)
//          into a scratch copy, so the iterations read 8 bytes per edge
//          instead of 8 bytes per slot;
//   bin   (per iteration):  stream the packed edges, write one 8-byte record
//          per edge: the contribution with its low mantissa bits replaced by
//          the destination's offset in its bin (records of the bins this
//          range feeds only a few are staged in LDS and leave as one run per
//          bin, see k_pb_bin_quiet);
//   split (optional, more than 64 fine bins only): the bin pass writes
//          coarse bins of 64 fine bins (2^20 vertices), so each workgroup has
//          at most 64 runs open, and this pass splits each coarse run into
//          its fine bins; the positions come from the same count matrix (a
//          coarse run of range w holds exactly range w's records of those
//          fine bins), so no pass needs an atomic in HBM.  On MI355X the
//          direct form measured faster at scale 24 (L2 merges the scattered
//          partial lines well enough), so it is the default;
//   accum (per iteration):  a workgroup per piece of a fine bin sums its
//          records into the LDS slice with fp64 LDS atomics and writes the
//          slice out (store for a bin in one piece, fp64 atomics for a split
//          bin).
// The HBM traffic is streams and per-bin runs; the random updates stay in LDS.
// Contributions are carried with 38 mantissa bits (32 with coarse bins;
// relative truncation below 2^-32), sums in fp64.
#include <cstdlib>

#include "common.h"

using namespace gpma_dev;

namespace {

constexpr uint32_t kBinBits = 14;   // 16384 destinations: a 128 KiB fp64 slice (gfx950: 160 KiB LDS per workgroup)
constexpr uint32_t kBinWidth = 1u << kBinBits;
constexpr uint64_t kBinMask = kBinWidth - 1;
constexpr uint32_t kSplitBits = 6;                       // fine bins per coarse bin: 64
constexpr uint32_t kCoarseBits = kBinBits + kSplitBits;  // 2^20 vertices per coarse bin
constexpr uint64_t kCoarseMask = (1ull << kCoarseBits) - 1;
constexpr uint32_t kCountThreads = 256;
constexpr uint64_t kRanges = 4096;              // slot ranges (workgroups) per pass, unless a range would pass kMaxRangeSlots
constexpr uint32_t kAccThreads = 1024;
constexpr uint32_t kMaxBins = 4096;            // V <= 2^26
constexpr uint64_t kPieceRecords = 1ull << 18;  // records per accumulation workgroup
constexpr uint64_t kMaxRangeSlots = 1ull << 18;

__host__ __device__ inline uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

__device__ __forceinline__ uint64_t ld_nt(const uint64_t *p) { return __builtin_nontemporal_load(p); }

// Workgroup w owns the slot range [w*spw, (w+1)*spw).  Once per call the
// count pass streams that range and also packs its edges (in no particular
// order) at keys[w*spw ..], ne[w] of them; every iteration's bin pass then
// streams the packed edges instead of the gapped slots.  Each thread takes
// kUnroll pairs per step, one 16-byte load each, all issued before any is
// used (the per-edge work is a chain of dependent accesses), then fn(k) runs
// over them; entries past the end read as the empty key.  The slot pass
// reads gaps too: a gap holds the empty key, and a load that waited for its
// leaf's count would serialise the stream (the occupied prefix rarely spares
// a line).  The loop is uniform over the workgroup.
constexpr int kUnroll = 8;

template <typename F>
__device__ __forceinline__ void for_each_pair_chunk(const uint64_t *__restrict__ base, uint64_t n, F fn) {
    using u64x2 = uint64_t __attribute__((ext_vector_type(2)));
    const uint64_t step = 2 * (uint64_t)blockDim.x;
    for (uint64_t c0 = 0; c0 < n; c0 += step * kUnroll) {
        uint64_t k[2 * kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; u++) {
            const uint64_t p = c0 + 2 * threadIdx.x + u * step;
            u64x2 q = {kEmpty, kEmpty};
            if (p + 1 < n) q = __builtin_nontemporal_load((const u64x2 *)(base + p));
            else if (p < n) q.x = ld_nt(base + p);
            k[2 * u] = q.x;
            k[2 * u + 1] = q.y;
        }
        fn(k);
    }
}

__device__ __forceinline__ bool is_edge(uint64_t k) { return is_edge_entry(k); }   // live, not a guard

// The contributions of a step's packed edges.  The two edges of a pair are
// neighbours in the src-major array, so they mostly share their source (a
// skewed graph's edges sit mostly in long rows): the second reuses the
// first's value then, which spares the address unit a gather lane.
__device__ __forceinline__ void pair_contribs(const uint64_t (&k)[2 * kUnroll], const double *__restrict__ contrib,
                                              uint64_t (&v)[2 * kUnroll]) {
#pragma unroll
    for (int j = 0; j < 2 * kUnroll; j++) {
        const bool same = (j & 1) && key_src(k[j]) == key_src(k[j - 1]);
        if (is_edge(k[j]) && !same) v[j] = (uint64_t)__double_as_longlong(contrib[key_src(k[j])]);
        else v[j] = (j & 1) ? v[j - 1] : 0;
    }
}

// Place of a lane's record in its bin (bins < 64): the lanes holding the same
// bin find each other with six ballots; the lowest of them reserves the
// group's places with one LDS atomic and each lane takes base + its rank in
// the group.  Every lane of the wave must call this (valid or not).
__device__ __forceinline__ uint32_t reserve_in_bin(uint32_t *cur, uint32_t bin, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int t = 0; t < 6; t++) {
        const uint64_t bt = __ballot(valid && ((bin >> t) & 1u));
        m &= ((bin >> t) & 1u) ? bt : ~bt;
    }
    const uint32_t lane = __lane_id();
    const uint32_t leader = valid ? (uint32_t)(__ffsll((unsigned long long)m) - 1) : lane;
    uint32_t base = 0;
    if (valid && lane == leader) base = atomicAdd(&cur[bin], (uint32_t)__popcll(m));
    base = __shfl(base, (int)leader, kWave);
    return base + (uint32_t)__popcll(m & lanemask_lt());
}

__global__ void __launch_bounds__(kCountThreads)
k_pb_count(const uint64_t *__restrict__ slots, uint64_t spw, uint32_t nb, uint32_t W, uint32_t *__restrict__ counts,
           uint64_t *__restrict__ keys, uint32_t *__restrict__ ne) {
    __shared__ uint32_t hist[kMaxBins];
    __shared__ uint32_t packed;
    __shared__ uint64_t wbuf[kCountThreads / kWave][2 * kUnroll * kWave];   // a wave's edges, packed
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) hist[b] = 0;
    if (threadIdx.x == 0) packed = 0;
    __syncthreads();
    const uint32_t lane = __lane_id();
    uint64_t *out = keys + (uint64_t)blockIdx.x * spw;
    for_each_pair_chunk(slots + (uint64_t)blockIdx.x * spw, spw, [&](const uint64_t (&k)[2 * kUnroll]) {
        uint32_t c = 0;
#pragma unroll
        for (int j = 0; j < 2 * kUnroll; j++)
            if (is_edge(k[j])) {
                atomicAdd(&hist[key_dst(k[j]) >> kBinBits], 1u);
                c++;
            }
        // the wave packs its edges in LDS, reserves one stretch of the packed
        // range and writes it with consecutive lanes on consecutive edges
        uint32_t x = c;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, kWave);
            if (lane >= (uint32_t)d) x += y;
        }
        uint64_t *wb = wbuf[threadIdx.x / kWave];
        uint32_t q = x - c;
#pragma unroll
        for (int j = 0; j < 2 * kUnroll; j++)
            if (is_edge(k[j])) wb[q++] = k[j];
        const uint32_t total = __shfl(x, kWave - 1, kWave);
        uint32_t at = 0;
        if (lane == kWave - 1) at = atomicAdd(&packed, total);
        at = __shfl(at, kWave - 1, kWave);
        wave_lds_sync();
        for (uint32_t t = lane; t < total; t += kWave) out[at + t] = wb[t];
        wave_lds_sync();   // the buffer is refilled next step
    });
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) counts[(uint64_t)b * W + blockIdx.x] = hist[b];
    if (threadIdx.x == 0) ne[blockIdx.x] = packed;
}

// bin b's records occupy [offs[b*W], offs[(b+1)*W]) (the last ends at the
// total); each bin is cut into pieces of at most kPieceRecords records
__global__ void __launch_bounds__(1024)
k_pb_pieces(const uint32_t *__restrict__ offs, const uint32_t *__restrict__ total, uint32_t nb, uint32_t W,
            uint4 *__restrict__ pieces, uint32_t *__restrict__ npieces) {
    __shared__ uint32_t lds[1024 / kWave + 1];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += blockDim.x) {
        const uint32_t b = base + threadIdx.x;
        uint32_t beg = 0, end = 0, np = 0;
        if (b < nb) {
            beg = offs[(uint64_t)b * W];
            end = b + 1 < nb ? offs[(uint64_t)(b + 1) * W] : *total;
            np = (uint32_t)div_up(end - beg, kPieceRecords);
        }
        uint32_t tot;
        const uint32_t ex = carry + block_exclusive_scan(np, &tot, lds);
        for (uint32_t i = 0; i < np; i++) {
            const uint32_t pb = beg + i * (uint32_t)kPieceRecords;
            const uint32_t pe = end - pb > kPieceRecords ? pb + (uint32_t)kPieceRecords : end;
            pieces[ex + i] = make_uint4(pb, pe, b, np > 1 ? 1u : 0u);
        }
        carry += tot;
    }
    if (threadIdx.x == 0) *npieces = carry;
}

// A record: the destination's offset in its bin in the low `bits` bits and,
// above them, either the contribution's fp64 bits (SRC = false: written
// every iteration) or the source vertex (SRC = true: written once per call,
// the iterations fetch contrib[source]).
template <bool SRC>
__device__ __forceinline__ uint64_t make_record(uint64_t key, uint64_t contrib_bits, uint64_t mask) {
    const uint32_t d = key_dst(key);
    if (SRC) return ((uint64_t)key_src(key) << kBinBits) | (d & mask);
    return (contrib_bits & ~mask) | (d & mask);
}

// Bin pass for at most 64 bins (or coarse bins) of 2^bits destinations;
// cur starts at offs[b*W + w]; places are reserved per wave (ballots).
template <bool SRC>
__global__ void __launch_bounds__(kCountThreads)
k_pb_bin(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ ne, uint64_t spw,
         uint32_t nb, uint32_t W, uint32_t bits, const uint32_t *__restrict__ offs,
         const double *__restrict__ contrib, uint64_t *__restrict__ rec) {
    __shared__ uint32_t cur[1u << kSplitBits];
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) cur[b] = offs[(uint64_t)b * W + blockIdx.x];
    __syncthreads();
    const uint64_t mask = (1ull << bits) - 1;
    for_each_pair_chunk(keys + (uint64_t)blockIdx.x * spw, ne[blockIdx.x], [&](const uint64_t (&k)[2 * kUnroll]) {
        uint64_t v[2 * kUnroll] = {};
        if (!SRC) pair_contribs(k, contrib, v);
#pragma unroll
        for (int j = 0; j < 2 * kUnroll; j++) {
            const bool ok = is_edge(k[j]);
            const uint32_t d = key_dst(k[j]);
            const uint32_t pos = reserve_in_bin(cur, ok ? d >> bits : 0u, ok);
            if (ok) rec[pos] = make_record<SRC>(k[j], v[j], mask);   // plain store: L2 merges a run's partial lines
        }
    });
}

// Bin pass for more than 64 bins.  A bin that receives many records from
// the workgroup's slot range has its lines filled quickly, so L2 merges its
// scattered 8-byte stores into whole lines; a quiet bin (fewer than
// kQuietRecords records from this range) keeps partial lines open for the
// whole pass, and those are what the scattered stores cost.  Staged bins are
// taken in bin order until the stage is full.  So the quiet
// bins' records are staged in LDS, in exact-size slices laid out by a scan of
// their counts (the count matrix gives every bin's count for this range), and
// each quiet bin is written out at the end as one contiguous run; busy bins
// (and quiet bins beyond the LDS budget) are stored directly.  Dynamic LDS:
// stage records, then cur[nb] (the bin's next place in rec), soff[nb] (its
// slice in the stage, kDirect for a direct bin), fill[nb].
constexpr uint32_t kQuietRecords = 128;   // measured best of 32..512 at scale 24
constexpr uint32_t kDirect = 0xFFFFFFFFu;
constexpr uint32_t kStageThreads = 1024;

__host__ __device__ inline uint32_t stage_records(uint32_t lds_bytes, uint32_t nb) {
    const uint32_t meta = 3 * nb * (uint32_t)sizeof(uint32_t) + 1024;
    return lds_bytes > meta ? (lds_bytes - meta) / (uint32_t)sizeof(uint64_t) : 0u;
}

template <bool SRC>
__global__ void __launch_bounds__(kStageThreads)
k_pb_bin_quiet(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ ne, uint64_t spw,
               uint32_t nb, uint32_t W, const uint32_t *__restrict__ offs, const uint32_t *__restrict__ total,
               const double *__restrict__ contrib, uint64_t *__restrict__ rec, uint32_t n_stage) {
    extern __shared__ uint64_t stage[];
    uint32_t *cur = (uint32_t *)(stage + n_stage);
    uint32_t *soff = cur + nb;
    uint32_t *fill = soff + nb;
    __shared__ uint32_t s_scan[kStageThreads / kWave + 1];
    const uint64_t last = (uint64_t)nb * W;
    uint32_t used = 0;   // stage records handed out so far (uniform)
    for (uint32_t base = 0; base < nb; base += kStageThreads) {
        const uint32_t b = base + threadIdx.x;
        uint32_t beg = 0, c = 0;
        if (b < nb) {
            const uint64_t e = (uint64_t)b * W + blockIdx.x;
            beg = offs[e];
            c = (e + 1 < last ? offs[e + 1] : *total) - beg;
        }
        const bool quiet = c > 0 && c < kQuietRecords;
        uint32_t tot;
        const uint32_t off = used + block_exclusive_scan(quiet ? c : 0u, &tot, s_scan);
        if (b < nb) {
            cur[b] = beg;
            soff[b] = quiet && off + c <= n_stage ? off : kDirect;
            fill[b] = 0;
        }
        used += tot;
    }
    __syncthreads();
    for_each_pair_chunk(keys + (uint64_t)blockIdx.x * spw, ne[blockIdx.x], [&](const uint64_t (&k)[2 * kUnroll]) {
        uint64_t v[2 * kUnroll] = {};
        if (!SRC) pair_contribs(k, contrib, v);
#pragma unroll
        for (int j = 0; j < 2 * kUnroll; j++) {
            if (!is_edge(k[j])) continue;
            const uint32_t d = key_dst(k[j]);
            const uint32_t b = d >> kBinBits;
            const uint64_t r = make_record<SRC>(k[j], v[j], kBinMask);
            const uint32_t so = soff[b];
            if (so == kDirect) rec[atomicAdd(&cur[b], 1u)] = r;   // plain store: L2 merges a busy run's lines
            else stage[so + atomicAdd(&fill[b], 1u)] = r;
        }
    });
    __syncthreads();
    // each staged bin leaves as one run (at most two wave stores)
    const uint32_t lane = __lane_id();
    for (uint32_t b = threadIdx.x / kWave; b < nb; b += kStageThreads / kWave) {
        const uint32_t so = soff[b];
        if (so == kDirect) continue;   // wave-uniform
        const uint32_t n = fill[b];
        for (uint32_t t = lane; t < n; t += kWave) rec[cur[b] + t] = stage[so + t];
    }
}

// coarse count matrix from the scanned fine one: range w's records in coarse
// bin c = sum over its fine bins of (next scanned entry - this entry)
__global__ void __launch_bounds__(256)
k_pb_coarse_counts(const uint32_t *__restrict__ offs, const uint32_t *__restrict__ total, uint32_t nb,
                   uint32_t nc, uint32_t W, uint32_t *__restrict__ ccnt) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint64_t)nc * W) return;
    const uint32_t c = (uint32_t)(i / W), w = (uint32_t)(i % W);
    const uint64_t last = (uint64_t)nb * W;
    uint32_t sum = 0;
    for (uint32_t f = 0; f < (1u << kSplitBits); f++) {
        const uint32_t b = (c << kSplitBits) + f;
        if (b >= nb) break;
        const uint64_t e = (uint64_t)b * W + w;
        const uint32_t nxt = e + 1 < last ? offs[e + 1] : *total;
        sum += nxt - offs[e];
    }
    ccnt[i] = sum;
}

// one workgroup per (coarse bin c, slot range w): the range's run of coarse
// records goes to its fine bins, at the places the fine count matrix gives
__global__ void __launch_bounds__(kCountThreads)
k_pb_split(const uint64_t *__restrict__ rec1, const uint32_t *__restrict__ coffs, const uint32_t *__restrict__ total,
           const uint32_t *__restrict__ offs, uint32_t nb, uint32_t nc, uint32_t W, uint64_t *__restrict__ rec2) {
    __shared__ uint32_t cur[1u << kSplitBits];
    const uint32_t c = blockIdx.x / W, w = blockIdx.x % W;
    const uint64_t e = (uint64_t)c * W + w;
    const uint64_t beg = coffs[e];
    const uint64_t end = e + 1 < (uint64_t)nc * W ? coffs[e + 1] : *total;
    if (beg == end) return;   // block-uniform
    for (uint32_t f = threadIdx.x; f < (1u << kSplitBits); f += blockDim.x) {
        const uint32_t b = (c << kSplitBits) + f;
        cur[f] = b < nb ? offs[(uint64_t)b * W + w] : 0u;
    }
    __syncthreads();
    for (uint64_t i0 = beg + threadIdx.x; i0 < end; i0 += (uint64_t)blockDim.x * kUnroll) {
        uint64_t r[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; u++) {
            const uint64_t i = i0 + (uint64_t)u * blockDim.x;
            r[u] = i < end ? ld_nt(rec1 + i) : 0;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; u++) {
            const bool ok = i0 + (uint64_t)u * blockDim.x < end;
            const uint64_t off = r[u] & kCoarseMask;
            const uint32_t pos = reserve_in_bin(cur, (uint32_t)(off >> kBinBits), ok);
            if (ok) rec2[pos] = (r[u] & ~kCoarseMask) | (off & kBinMask);
        }
    }
}

// The value a record adds: its own high bits (SRC = false) or the
// contribution of the source it names (SRC = true).
template <bool SRC>
__device__ __forceinline__ double record_value(uint64_t r, const double *__restrict__ contrib) {
    if (SRC) return contrib[r >> kBinBits];
    return __longlong_as_double((long long)(r & ~kBinMask));
}

template <bool SRC>
__global__ void __launch_bounds__(kAccThreads)
k_pb_accum(const uint64_t *__restrict__ rec, const uint4 *__restrict__ pieces, const uint32_t *__restrict__ npieces,
           uint32_t V, const double *__restrict__ contrib, double *__restrict__ y) {
    extern __shared__ double acc[];   // kBinWidth doubles
    if (blockIdx.x >= *npieces) return;
    const uint4 pc = pieces[blockIdx.x];
    for (uint32_t j = threadIdx.x; j < kBinWidth; j += kAccThreads) acc[j] = 0.0;
    __syncthreads();
    // records per thread in flight: two for source records (measured at scale 24:
    // 1302-1327 us per step with 2, 1385 with 1, 1414 with 3, 1470-1500 with 4,
    // 1527-1542 with 8; fewer outstanding fetches per workgroup contend less
    // for the fabric), four for value records (2 was 1.4 % slower)
    constexpr uint32_t kU = SRC ? 2 : 4;
    uint64_t i = (uint64_t)pc.x + threadIdx.x;
    for (; i + (kU - 1) * kAccThreads < pc.y; i += kU * kAccThreads) {
        uint64_t r[kU];
#pragma unroll
        for (uint32_t u = 0; u < kU; u++) r[u] = ld_nt(rec + i + u * kAccThreads);
        double c[kU];
#pragma unroll
        for (uint32_t u = 0; u < kU; u++) c[u] = record_value<SRC>(r[u], contrib);
#pragma unroll
        for (uint32_t u = 0; u < kU; u++) atomicAdd(&acc[r[u] & kBinMask], c[u]);
    }
    for (; i < pc.y; i += kAccThreads) {
        const uint64_t r = ld_nt(rec + i);
        atomicAdd(&acc[r & kBinMask], record_value<SRC>(r, contrib));
    }
    __syncthreads();
    const uint64_t v0 = (uint64_t)pc.z << kBinBits;
    for (uint32_t j = threadIdx.x; j < kBinWidth; j += kAccThreads) {
        const uint64_t v = v0 + j;
        if (v >= V) break;
        const double a = acc[j];
        if (!pc.w) y[v] = a;
        else if (a != 0.0) unsafeAtomicAdd(&y[v], a);
    }
}

}  // namespace

namespace gpma_host {

// The accumulation slice exceeds the default 64 KiB of LDS; the binned form
// is offered only where the device grants it.
static int g_stage_lds = 0;   // dynamic LDS the quiet-bin stage may use (set with the attribute)

bool pb_supported(uint32_t V) {
    static int ok = -1;
    if (ok < 0) {
        const size_t bytes = kBinWidth * sizeof(double);
        int dev = 0, max_lds = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        ok = (size_t)max_lds >= bytes &&
             hipFuncSetAttribute((const void *)k_pb_accum<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)bytes) == hipSuccess &&
             hipFuncSetAttribute((const void *)k_pb_accum<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)bytes) == hipSuccess;
        // the bin pass stages in what is left of the workgroup's LDS after its scan words
        const int stage = max_lds - (int)((kStageThreads / kWave + 1) * sizeof(uint32_t)) - 256;
        ok = ok && stage > 0 &&
             hipFuncSetAttribute((const void *)k_pb_bin_quiet<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 stage) == hipSuccess &&
             hipFuncSetAttribute((const void *)k_pb_bin_quiet<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 stage) == hipSuccess;
        if (ok) g_stage_lds = stage;
        if (!ok) (void)hipGetLastError();
    }
    return ok && div_up(V, kBinWidth) <= kMaxBins;
}

PbLayout pb_layout(uint32_t V, uint64_t cap, uint32_t lf_log2, uint64_t n_edges, bool coarse) {
    PbLayout L;
    L.nb = (uint32_t)div_up(V, kBinWidth);
    // bins are written directly; `coarse` routes them through coarse bins of
    // 64 first (same result; faster where scattered stores are dear)
    L.nc = (coarse && L.nb > (1u << kSplitBits)) ? (uint32_t)div_up(V, 1ull << kCoarseBits) : 0;
    uint64_t spw = cap / kRanges;
    const uint64_t lf = 1ull << lf_log2;
    if (spw < lf) spw = lf;
    if (spw > kMaxRangeSlots) spw = kMaxRangeSlots;
    if (spw > cap) spw = cap;
    L.spw = spw;
    L.W = (uint32_t)(cap / spw);
    L.max_pieces = L.nb + div_up(n_edges, kPieceRecords) + 1;
    L.count_words = (uint64_t)L.nb * L.W;
    L.coarse_words = (uint64_t)L.nc * L.W;
    return L;
}

void launch_pb_structure(const uint64_t *slots, const PbLayout &L, uint64_t *keys, uint32_t *ne,
                         uint32_t *offs, uint32_t *total, uint32_t *scan_tmp, uint4 *pieces, uint32_t *npieces,
                         uint32_t *coffs, hipStream_t s) {
    hipLaunchKernelGGL(k_pb_count, dim3(L.W), dim3(kCountThreads), 0, s, slots, L.spw, L.nb, L.W, offs, keys, ne);
    scan_u32(offs, offs, L.count_words, total, scan_tmp, s);
    hipLaunchKernelGGL(k_pb_pieces, dim3(1), dim3(1024), 0, s, offs, total, L.nb, L.W, pieces, npieces);
    if (L.nc) {
        hipLaunchKernelGGL(k_pb_coarse_counts, dim3((uint32_t)div_up(L.coarse_words, 256)), dim3(256), 0, s, offs,
                           total, L.nb, L.nc, L.W, coffs);
        scan_u32(coffs, coffs, L.coarse_words, nullptr, scan_tmp, s);
    }
}

void launch_pb_spmv(const uint64_t *keys, const uint32_t *ne, const PbLayout &L,
                    const uint32_t *offs, const uint32_t *total, const uint4 *pieces, const uint32_t *npieces,
                    const uint32_t *coffs, const double *contrib, uint64_t *rec, uint64_t *rec2, uint32_t V,
                    double *y, hipStream_t s) {
    if (L.nc) {
        hipLaunchKernelGGL(k_pb_bin<false>, dim3(L.W), dim3(kCountThreads), 0, s, keys, ne, L.spw, L.nc, L.W,
                           kCoarseBits, coffs, contrib, rec);
        hipLaunchKernelGGL(k_pb_split, dim3((uint32_t)L.coarse_words), dim3(kCountThreads), 0, s, rec, coffs, total,
                           offs, L.nb, L.nc, L.W, rec2);
        rec = rec2;
    } else {
        launch_pb_bin(keys, ne, L, offs, total, contrib, rec, false, s);
    }
    hipLaunchKernelGGL(k_pb_accum<false>, dim3((uint32_t)L.max_pieces), dim3(kAccThreads), kBinWidth * sizeof(double),
                       s, rec, pieces, npieces, V, contrib, y);
}

void launch_pb_bin(const uint64_t *keys, const uint32_t *ne, const PbLayout &L, const uint32_t *offs,
                   const uint32_t *total, const double *contrib, uint64_t *rec, bool src_records, hipStream_t s) {
    if (L.nb <= (1u << kSplitBits)) {
        if (src_records)
            hipLaunchKernelGGL(k_pb_bin<true>, dim3(L.W), dim3(kCountThreads), 0, s, keys, ne, L.spw, L.nb, L.W,
                               kBinBits, offs, contrib, rec);
        else
            hipLaunchKernelGGL(k_pb_bin<false>, dim3(L.W), dim3(kCountThreads), 0, s, keys, ne, L.spw, L.nb, L.W,
                               kBinBits, offs, contrib, rec);
        return;
    }
    const uint32_t ns = stage_records((uint32_t)g_stage_lds, L.nb);
    const size_t lds = (size_t)ns * sizeof(uint64_t) + 3 * (size_t)L.nb * sizeof(uint32_t);
    if (src_records)
        hipLaunchKernelGGL(k_pb_bin_quiet<true>, dim3(L.W), dim3(kStageThreads), lds, s, keys, ne, L.spw, L.nb, L.W,
                           offs, total, contrib, rec, ns);
    else
        hipLaunchKernelGGL(k_pb_bin_quiet<false>, dim3(L.W), dim3(kStageThreads), lds, s, keys, ne, L.spw, L.nb, L.W,
                           offs, total, contrib, rec, ns);
}

void launch_pb_gather(const PbLayout &L, const uint4 *pieces, const uint32_t *npieces, const double *contrib,
                      const uint64_t *rec, uint32_t V, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_pb_accum<true>, dim3((uint32_t)L.max_pieces), dim3(kAccThreads), kBinWidth * sizeof(double),
                       s, rec, pieces, npieces, V, contrib, y);
}

}  // namespace gpma_host
