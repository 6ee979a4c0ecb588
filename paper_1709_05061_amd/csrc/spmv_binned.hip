// PageRank SpMV by destination bins (propagation blocking) over the
// src-major slot array (Section 6.1, PageRank as repeated SpMV; Section 4.2,
// algorithms read the array in place, skipping gaps and guards).
//
// A stored edge u->v adds contrib[u] to y[v].  Read along the src-major
// array, contrib[u] is a near-sequential read but y[v] is a random update;
// read along a dst-major array it is the other way round.  Either way one
// side is a random access per edge into a vector far larger than L2.  Here
// the edge stream is instead split by destination into bins of 8192
// vertices, whose slice of y fits one workgroup's LDS:
//   count (once per call): per slot range, how many edges fall in each bin;
//          an exclusive scan of the bin-major count matrix gives every
//          (bin, range) pair its place in the record array;
//   bin   (per iteration):  stream the slots, write one 8-byte record per
//          edge into its bin: the contribution with its low 13 mantissa bits
//          replaced by the destination's offset in the bin;
//   accum (per iteration):  a workgroup per piece of a bin sums its records
//          into the LDS slice with fp64 LDS atomics and writes the slice out
//          (store for a bin in one piece, fp64 atomics for a split bin).
// Every HBM access is a stream; the random traffic stays in LDS.
// Contributions are carried with 39 mantissa bits (relative truncation below
// 2^-39), sums in fp64.
#include "common.h"

using namespace gpma_dev;

namespace {

constexpr uint32_t kBinBits = 13;
constexpr uint32_t kBinWidth = 1u << kBinBits;
constexpr uint64_t kBinMask = kBinWidth - 1;
constexpr uint32_t kCountThreads = 256;
constexpr uint32_t kAccThreads = 1024;
constexpr uint32_t kMaxBins = 4096;            // V <= 2^25
constexpr uint64_t kPieceRecords = 1ull << 18;  // records per accumulation workgroup
constexpr uint64_t kMaxRangeSlots = 1ull << 18;

__host__ __device__ inline uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

__device__ __forceinline__ uint64_t ld_nt(const uint64_t *p) { return __builtin_nontemporal_load(p); }

// The slot range of workgroup w is [w*spw, (w+1)*spw); spw is a power of two
// no smaller than a leaf, so slot pairs (p, p+1) with p even share a leaf.
// fn(k) is called for every stored edge (guards and gaps skipped).
template <typename F>
__device__ __forceinline__ void for_each_edge(const uint64_t *__restrict__ slots, const uint16_t *__restrict__ cnt,
                                              uint32_t lf_log2, uint64_t spw, F fn) {
    const uint64_t lo = (uint64_t)blockIdx.x * spw;
    const uint64_t hi = lo + spw;
    const uint64_t lfm = (1ull << lf_log2) - 1;
    for (uint64_t p = lo + 2 * threadIdx.x; p < hi; p += 2 * (uint64_t)blockDim.x) {
        const uint32_t c = cnt[p >> lf_log2];
        const uint32_t o = (uint32_t)(p & lfm);
        if (o >= c) continue;
        const uint64_t k0 = ld_nt(slots + p);
        const uint64_t k1 = o + 1 < c ? ld_nt(slots + p + 1) : kEmpty;
        if (!is_guard(k0)) fn(k0);
        if (k1 != kEmpty && !is_guard(k1)) fn(k1);
    }
}

__global__ void __launch_bounds__(kCountThreads)
k_pb_count(const uint64_t *__restrict__ slots, const uint16_t *__restrict__ cnt, uint32_t lf_log2, uint64_t spw,
           uint32_t nb, uint32_t W, uint32_t *__restrict__ counts) {
    __shared__ uint32_t hist[kMaxBins];
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    for_each_edge(slots, cnt, lf_log2, spw, [&](uint64_t k) { atomicAdd(&hist[key_dst(k) >> kBinBits], 1u); });
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) counts[(uint64_t)b * W + blockIdx.x] = hist[b];
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

__global__ void __launch_bounds__(kCountThreads)
k_pb_bin(const uint64_t *__restrict__ slots, const uint16_t *__restrict__ cnt, uint32_t lf_log2, uint64_t spw,
         uint32_t nb, uint32_t W, const uint32_t *__restrict__ offs, const double *__restrict__ contrib,
         uint64_t *__restrict__ rec) {
    __shared__ uint32_t cur[kMaxBins];
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) cur[b] = offs[(uint64_t)b * W + blockIdx.x];
    __syncthreads();
    for_each_edge(slots, cnt, lf_log2, spw, [&](uint64_t k) {
        const uint32_t d = key_dst(k);
        const uint64_t bits = (uint64_t)__double_as_longlong(contrib[key_src(k)]);
        const uint32_t pos = atomicAdd(&cur[d >> kBinBits], 1u);
        __builtin_nontemporal_store((bits & ~kBinMask) | (d & kBinMask), rec + pos);
    });
}

__global__ void __launch_bounds__(kAccThreads)
k_pb_accum(const uint64_t *__restrict__ rec, const uint4 *__restrict__ pieces, const uint32_t *__restrict__ npieces,
           uint32_t V, double *__restrict__ y) {
    __shared__ double acc[kBinWidth];
    if (blockIdx.x >= *npieces) return;
    const uint4 pc = pieces[blockIdx.x];
    for (uint32_t j = threadIdx.x; j < kBinWidth; j += kAccThreads) acc[j] = 0.0;
    __syncthreads();
    constexpr uint32_t kU = 4;
    uint64_t i = (uint64_t)pc.x + threadIdx.x;
    for (; i + (kU - 1) * kAccThreads < pc.y; i += kU * kAccThreads) {
        uint64_t r[kU];
#pragma unroll
        for (uint32_t u = 0; u < kU; u++) r[u] = ld_nt(rec + i + u * kAccThreads);
#pragma unroll
        for (uint32_t u = 0; u < kU; u++)
            atomicAdd(&acc[r[u] & kBinMask], __longlong_as_double((long long)(r[u] & ~kBinMask)));
    }
    for (; i < pc.y; i += kAccThreads) {
        const uint64_t r = ld_nt(rec + i);
        atomicAdd(&acc[r & kBinMask], __longlong_as_double((long long)(r & ~kBinMask)));
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

bool pb_supported(uint32_t V) { return div_up(V, kBinWidth) <= kMaxBins; }

PbLayout pb_layout(uint32_t V, uint64_t cap, uint32_t lf_log2, uint64_t n_edges) {
    PbLayout L;
    L.nb = (uint32_t)div_up(V, kBinWidth);
    uint64_t spw = cap / 1024;
    const uint64_t lf = 1ull << lf_log2;
    if (spw < lf) spw = lf;
    if (spw > kMaxRangeSlots) spw = kMaxRangeSlots;
    if (spw > cap) spw = cap;
    L.spw = spw;
    L.W = (uint32_t)(cap / spw);
    L.max_pieces = L.nb + div_up(n_edges, kPieceRecords) + 1;
    L.count_words = (uint64_t)L.nb * L.W;
    return L;
}

void launch_pb_structure(const uint64_t *slots, const uint16_t *cnt, uint32_t lf_log2, const PbLayout &L,
                         uint32_t *offs, uint32_t *total, uint32_t *scan_tmp, uint4 *pieces, uint32_t *npieces,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_pb_count, dim3(L.W), dim3(kCountThreads), 0, s, slots, cnt, lf_log2, L.spw, L.nb, L.W, offs);
    scan_u32(offs, offs, L.count_words, total, scan_tmp, s);
    hipLaunchKernelGGL(k_pb_pieces, dim3(1), dim3(1024), 0, s, offs, total, L.nb, L.W, pieces, npieces);
}

void launch_pb_spmv(const uint64_t *slots, const uint16_t *cnt, uint32_t lf_log2, const PbLayout &L,
                    const uint32_t *offs, const uint4 *pieces, const uint32_t *npieces, const double *contrib,
                    uint64_t *rec, uint32_t V, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_pb_bin, dim3(L.W), dim3(kCountThreads), 0, s, slots, cnt, lf_log2, L.spw, L.nb, L.W, offs,
                       contrib, rec);
    hipLaunchKernelGGL(k_pb_accum, dim3((uint32_t)L.max_pieces), dim3(kAccThreads), 0, s, rec, pieces, npieces, V,
                       y);
}

}  // namespace gpma_host
