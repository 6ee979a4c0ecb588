// Analytics that read the PMA in place (Section 4.2: existing algorithms run
// on CSR-on-GPMA once they skip gaps and guards; Section 6.1 "Applications").
//   PageRank: matrix-based; push over the sorted slot stream, fp64 sums.
//   BFS:      vertex-centric; rows via the CSR offsets, wave per frontier row.
//   CC:       edge-centric; hooking over the slot stream + pointer jumping.
#include <algorithm>

#include "common.h"

using namespace gpma_dev;

namespace {

inline uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// slot streams are read once per pass: non-temporal loads keep them from
// evicting the vectors the pass gathers from (contributions, labels, dist)
__device__ __forceinline__ uint64_t ld_stream(const uint64_t *p) {
    return __builtin_nontemporal_load(p);
}
__device__ __forceinline__ void ld_stream2(const uint64_t *p, uint64_t &a, uint64_t &b) {
    a = __builtin_nontemporal_load(p);
    b = __builtin_nontemporal_load(p + 1);
}

// ---------------------------------------------------------------------------
// PageRank: x'[v] = (1-d)/V + d * (sum_{u->v} x[u]/outdeg(u) + D/V)

__global__ void __launch_bounds__(256)
k_pr_prep(const float *__restrict__ x, const uint32_t *__restrict__ deg, uint32_t V, int uniform,
          double *__restrict__ contrib, double *__restrict__ y, double *__restrict__ dangling) {
    __shared__ double part[256 / kWave];
    double dm = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += stride) {
        const double xv = uniform ? 1.0 / (double)V : (double)x[v];
        const uint32_t dv = deg[v];
        contrib[v] = dv ? xv / (double)dv : 0.0;
        if (!dv) dm += xv;
        y[v] = 0.0;
    }
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) dm += __shfl_xor(dm, d, kWave);
    if (__lane_id() == 0) part[threadIdx.x / kWave] = dm;
    __syncthreads();
    if (threadIdx.x == 0) {   // one atomic per block; the grid is bounded
        double t = 0.0;
        for (int w = 0; w < 256 / kWave; w++) t += part[w];
        if (t != 0.0) unsafeAtomicAdd(dangling, t);
    }
}

// Push y[dst] += contrib[src] for every stored edge of a src-major array.
// Lane pairs of slots walk the array; a leaf's gap tail is never loaded (its
// leaf count says where the packed prefix ends).  src is non-decreasing along
// the stream, so contrib[src] reads hit cache; y takes one fp64 atomic per edge.
__global__ void __launch_bounds__(256)
k_pr_push(const uint64_t *__restrict__ slots, const uint16_t *__restrict__ cnt, uint64_t cap,
          uint32_t lf_log2, const double *__restrict__ contrib, double *__restrict__ y) {
    const uint64_t lfm = (1ull << lf_log2) - 1;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x * 2;
    for (uint64_t p = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2; p < cap; p += stride) {
        const uint32_t c = cnt[p >> lf_log2];
        const uint32_t o = (uint32_t)(p & lfm);
        if (o >= c) continue;
        uint64_t k0, k1 = kEmpty;
        if (o + 1 < c) ld_stream2(slots + p, k0, k1);
        else k0 = ld_stream(slots + p);
        if (is_edge_entry(k0)) unsafeAtomicAdd(&y[key_dst(k0)], contrib[key_src(k0)]);
        if (is_edge_entry(k1)) unsafeAtomicAdd(&y[key_dst(k1)], contrib[key_src(k1)]);
    }
}

// Pull over the dst-major mirror: entry v<<32|u adds contrib[u] to y[v].  A
// wave takes 128 consecutive slots (2 per lane).  Along the array the row v is
// non-decreasing; a gap takes the row of its leaf's last entry, so the wave
// sees runs of equal rows.  A segmented inclusive scan over the lanes sums each
// run; a run wholly inside the wave is a complete row and is stored, a run
// touching either end of the wave may continue in a neighbour and is added
// atomically (y is zeroed beforehand).  At most two atomics per wave.
struct PullLane {
    uint32_t r0, r1;   // rows of the lane's two slots (kNone past the end)
    double a, b;       // their contributions (0 for gaps and guards)
};

__device__ __forceinline__ PullLane pull_load(const uint64_t *__restrict__ slots,
                                              const uint16_t *__restrict__ cnt, uint64_t cap,
                                              uint32_t lf_log2, const double *__restrict__ contrib,
                                              uint64_t p) {
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    PullLane L{kNone, kNone, 0.0, 0.0};
    if (p >= cap) return L;
    const uint64_t lfm = (1ull << lf_log2) - 1;
    const uint64_t leaf = p >> lf_log2;
    const uint32_t c = cnt[leaf];
    const uint32_t o = (uint32_t)(p & lfm);
    uint64_t k0 = kEmpty, k1 = kEmpty;
    if (o + 1 < c) ld_stream2(slots + p, k0, k1);
    else if (o < c) k0 = ld_stream(slots + p);
    uint64_t last = 0;
    if (o + 1 >= c) last = slots[(leaf << lf_log2) + c - 1];
    L.r0 = (uint32_t)(order_key(o < c ? k0 : last) >> 32);
    L.r1 = (uint32_t)(order_key(o + 1 < c ? k1 : last) >> 32);
    if (o < c && is_edge_entry(k0)) L.a = contrib[key_dst(k0)];
    if (o + 1 < c && is_edge_entry(k1)) L.b = contrib[key_dst(k1)];
    return L;
}

__device__ __forceinline__ void pull_reduce(const PullLane &L, uint32_t lane, double *__restrict__ y) {
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    double sc = (L.r0 == L.r1) ? L.a + L.b : L.b;   // running sum of the lane's tail run
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const double ys = __shfl_up(sc, d, kWave);
        const uint32_t yr = __shfl_up(L.r1, d, kWave);
        if (lane >= (uint32_t)d && yr == L.r1) sc += ys;
    }
    const double prev_s = __shfl_up(sc, 1, kWave);
    const uint32_t prev_r = __shfl_up(L.r1, 1, kWave);
    const uint32_t next_r0 = __shfl_down(L.r0, 1, kWave);
    const uint32_t first_row = __shfl(L.r0, 0, kWave);
    if (L.r0 != L.r1 && L.r0 != kNone) {
        const double va = L.a + ((lane > 0 && prev_r == L.r0) ? prev_s : 0.0);
        if (L.r0 == first_row) unsafeAtomicAdd(&y[L.r0], va); else y[L.r0] = va;
    }
    if (L.r1 != kNone && (lane == kWave - 1 || next_r0 != L.r1)) {
        if (L.r1 == first_row || lane == kWave - 1) unsafeAtomicAdd(&y[L.r1], sc); else y[L.r1] = sc;
    }
}

// Pull over the dst-major mirror: entry v<<32|u adds contrib[u] to y[v].  A
// wave takes chunks of 128 consecutive slots (2 per lane), two chunks at a
// time so each lane has four contribution gathers in flight.  Along the
// array the row v is non-decreasing; a gap takes the row of its leaf's last
// entry, so a chunk holds runs of equal rows.  A segmented inclusive scan
// over the lanes sums each run; a run wholly inside the chunk is a complete
// row and is stored, a run touching either end of the chunk may continue in
// a neighbour and is added atomically (y is zeroed beforehand).  At most two
// atomics per chunk.
__global__ void __launch_bounds__(256)
k_pr_pull(const uint64_t *__restrict__ slots, const uint16_t *__restrict__ cnt, uint64_t cap,
          uint32_t lf_log2, const double *__restrict__ contrib, double *__restrict__ y) {
    const uint32_t lane = __lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = (uint64_t)gridDim.x * blockDim.x / kWave;
    constexpr uint64_t kChunk = 2 * kWave;
    for (uint64_t base = wave * 2 * kChunk; base < cap; base += nwaves * 2 * kChunk) {
        const PullLane A = pull_load(slots, cnt, cap, lf_log2, contrib, base + 2 * lane);
        const PullLane B = pull_load(slots, cnt, cap, lf_log2, contrib, base + kChunk + 2 * lane);
        pull_reduce(A, lane, y);
        pull_reduce(B, lane, y);
    }
}

__global__ void __launch_bounds__(256)
k_pr_combine(const double *__restrict__ y, const double *__restrict__ dangling, uint32_t V,
             double damping, float *__restrict__ out) {
    uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    double inv = 1.0 / (double)V;
    out[v] = (float)((1.0 - damping) * inv + damping * (y[v] + (*dangling) * inv));
}

// ---------------------------------------------------------------------------
// BFS

__global__ void k_bfs_init(int32_t *__restrict__ dist, uint32_t V, uint32_t source,
                           uint32_t *__restrict__ queue, uint32_t *__restrict__ qcount) {
    uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < V) dist[v] = (v == source) ? 0 : -1;
    if (v == 0) {
        queue[0] = source;
        *qcount = 1;
    }
}

// Frontier expansion, load-balanced over slots rather than vertices: the
// frontier's rows [row_ptr[u], row_ptr[u+1]) are laid end to end (offs is
// the exclusive scan of their lengths, *total their sum) and every thread
// takes kBfsItems consecutive slots of that concatenation, so a hub's long
// row is spread over many threads.  Gaps and guards are skipped (the
// IsEntryExist test of Algorithm "GPU-based BFS Neighbour Gathering").  New
// vertices are claimed with a CAS on dist and appended with one atomic per
// wave.
constexpr int kBfsItems = 8;

__global__ void k_bfs_row_len(const uint32_t *__restrict__ row_ptr, const uint32_t *__restrict__ front,
                              uint32_t nfront, uint32_t *__restrict__ len) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nfront) {
        uint32_t u = front[i];
        len[i] = row_ptr[u + 1] - row_ptr[u];
    }
}

__global__ void __launch_bounds__(256)
k_bfs_expand(const uint64_t *__restrict__ slots, uint64_t cap, const uint32_t *__restrict__ row_ptr,
             const uint32_t *__restrict__ front, const uint32_t *__restrict__ offs, uint32_t nfront,
             const uint32_t *__restrict__ total, int32_t level, int32_t *__restrict__ dist,
             uint32_t *__restrict__ next, uint32_t *__restrict__ next_count) {
    const uint32_t T = *total;
    const uint32_t lane = __lane_id();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * kBfsItems;
    for (uint64_t t0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * kBfsItems; t0 < T + 0ull;
         t0 += stride) {
        // frontier entry holding slot t0: the last i with offs[i] <= t0
        uint32_t lo = 0, hi = nfront;
        while (hi - lo > 1) {
            uint32_t mid = (lo + hi) >> 1;
            if (offs[mid] <= t0) lo = mid; else hi = mid;
        }
        uint32_t i = lo;
        // slot of concatenation index t in row i: row_ptr[front[i]] + (t - offs[i]),
        // kept in 64 bits (row starts can precede their concatenation offset)
        uint32_t rend = (i + 1 < nfront) ? offs[i + 1] : T;
        uint64_t rstart = row_ptr[front[i]];
        uint64_t roff = offs[i];
        for (int q = 0; q < kBfsItems; q++) {
            const uint64_t t = t0 + q;
            bool claim = false;
            uint32_t v = 0;
            if (t < T) {
                while (t >= rend) {   // next non-empty row (rows have at least a guard)
                    i++;
                    rend = (i + 1 < nfront) ? offs[i + 1] : T;
                    rstart = row_ptr[front[i]];
                    roff = offs[i];
                }
                const uint64_t p = rstart + (t - roff);
                const uint64_t k = p < cap ? slots[p] : kEmpty;
                if (is_edge_entry(k)) {
                    v = key_dst(k);
                    if (__hip_atomic_load(&dist[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < 0)
                        claim = atomicCAS(&dist[v], -1, level + 1) == -1;
                }
            }
            const uint64_t m = __ballot(claim);
            if (m) {
                const uint32_t leader = __ffsll((unsigned long long)m) - 1;
                uint32_t base = 0;
                if (lane == leader) base = atomicAdd(next_count, (uint32_t)__popcll(m));
                base = __shfl(base, leader, kWave);
                if (claim) next[base + __popcll(m & lanemask_lt())] = v;
            }
        }
    }
}

// Bottom-up step over the dst-major mirror, whose row v lists the in-edges
// of v: a thread per vertex; an unvisited v scans its in-edges and stops at
// the first u on the current level, then joins the next level.  Only the
// thread of v writes dist[v], so no CAS is needed; a u claimed during this
// step has dist[u] = level+1 and is correctly not taken as a parent.  Used
// for large frontiers (most unvisited vertices then find a parent within a
// few in-edges).
constexpr int kBuStep = 4;

__global__ void __launch_bounds__(256)
k_bfs_bottom_up(const uint64_t *__restrict__ mslots, const uint32_t *__restrict__ mrow, uint32_t V,
                int32_t level, int32_t *__restrict__ dist, uint32_t *__restrict__ next,
                uint32_t *__restrict__ next_count) {
    const uint32_t lane = __lane_id();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v0 < V + 0ull; v0 += stride) {
        const uint32_t v = (uint32_t)v0;
        bool claim = false;
        if (dist[v] < 0) {
            // kBuStep entries at a time: their loads, then their parents'
            // distances, are in flight together (a row ends with its guard,
            // which, like gaps and marked entries, is not an edge).  A
            // distance equal to `level` cannot change during the step (only
            // unvisited vertices are written), so plain loads may hit cache.
            const uint32_t end = mrow[v + 1];
            for (uint32_t p = mrow[v]; p < end && !claim; p += kBuStep) {
                uint64_t k[kBuStep];
#pragma unroll
                for (int j = 0; j < kBuStep; j++) k[j] = p + j < end ? mslots[p + j] : kEmpty;
                int32_t d[kBuStep];
#pragma unroll
                for (int j = 0; j < kBuStep; j++) d[j] = is_edge_entry(k[j]) ? dist[(uint32_t)k[j]] : -2;
#pragma unroll
                for (int j = 0; j < kBuStep; j++) claim |= d[j] == level;
            }
            if (claim) dist[v] = level + 1;
        }
        const uint64_t m = __ballot(claim);
        if (m) {
            const uint32_t leader = __ffsll((unsigned long long)m) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(next_count, (uint32_t)__popcll(m));
            base = __shfl(base, leader, kWave);
            if (claim) next[base + __popcll(m & lanemask_lt())] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// CC: parent pointers only ever decrease (atomicMin of a root onto a smaller
// root), so every tree's root is its smallest vertex and find() terminates.

__device__ __forceinline__ uint32_t cc_find(const uint32_t *label, uint32_t x) {
    uint32_t p = __hip_atomic_load(&label[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (p != x) {
        x = p;
        p = __hip_atomic_load(&label[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return x;
}

// Union of the trees rooted at a and b: hook the larger root under the
// smaller with a compare-and-swap that succeeds only while the larger is
// still a root; when another thread hooked it first, look up both roots
// again and retry.  Every union is therefore applied (one sweep over the
// edges suffices), links always point to smaller ids (no cycles), and each
// retry follows a hook that some other thread completed.
__device__ __forceinline__ void cc_union(uint32_t *label, uint32_t a, uint32_t b) {
    while (a != b) {
        const uint32_t hi = a > b ? a : b, lo = a > b ? b : a;
        const uint32_t old = atomicCAS(&label[hi], hi, lo);
        if (old == hi) return;
        a = cc_find(label, old);
        b = cc_find(label, lo);
    }
}

__global__ void k_cc_init(uint32_t *__restrict__ label, uint32_t V) {
    uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < V) label[v] = (uint32_t)v;
}

// A grid-stride pass over slot pairs: each thread issues kCcPairs 16-byte
// loads before it uses any (the per-edge work is a chain of dependent label
// reads), then fn(k) runs over the 2*kCcPairs slots; slots past the end read
// as the empty key.  The two slots of a pair are neighbours, so an edge at an
// odd place usually shares its source with the one before it.
constexpr int kCcPairs = 4;

template <typename F>
__device__ __forceinline__ void for_slot_pairs(const uint64_t *__restrict__ slots, uint64_t cap, F fn) {
    using u64x2 = uint64_t __attribute__((ext_vector_type(2)));
    const uint64_t np = (cap + 1) >> 1;
    const uint64_t nt = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q0 < np; q0 += nt * kCcPairs) {
        uint64_t k[2 * kCcPairs];
#pragma unroll
        for (int u = 0; u < kCcPairs; u++) {
            const uint64_t p = 2 * (q0 + (uint64_t)u * nt);
            u64x2 v = {kEmpty, kEmpty};
            if (p + 1 < cap) v = __builtin_nontemporal_load((const u64x2 *)(slots + p));
            else if (p < cap) v.x = ld_stream(slots + p);
            k[2 * u] = v.x;
            k[2 * u + 1] = v.y;
        }
        fn(k);
    }
}

// Without a mirror every edge takes a union, and one slot per thread and
// step measured faster than the pair loop of the skipping sweep below.
__global__ void __launch_bounds__(256)
k_cc_hook(const uint64_t *__restrict__ slots, uint64_t cap, uint32_t *label) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < cap; p += stride) {
        uint64_t k = ld_stream(slots + p);
        if (!is_edge_entry(k)) continue;
        cc_union(label, cc_find(label, key_src(k)), cc_find(label, key_dst(k)));
    }
}

// Sampling round (the approach of Afforest, Sutton et al.): every vertex is
// hooked to the first entry of its row (out-row on the array, in-row on the
// dst-major mirror).  Row v starts after guard v-1; a leaf's gap tail may sit
// between them, so the scan skips empty slots and marked entries (at most
// one leaf's worth; a row not sampled is left to the sweeps).
__global__ void __launch_bounds__(256)
k_cc_sample(const uint64_t *__restrict__ slots, const uint32_t *__restrict__ row_ptr, uint32_t V, uint32_t lf,
            uint32_t *label) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    uint64_t p = v ? row_ptr[v] : 0;
    const uint64_t end = row_ptr[v + 1];   // one past guard v
    uint64_t k = kEmpty;
    for (uint32_t t = 0; t <= lf && p < end; t++, p++) {
        k = slots[p];
        if (is_live(k)) break;
    }
    if (!is_edge_entry(k)) return;
    cc_union(label, cc_find(label, key_src(k)), cc_find(label, key_dst(k)));
}

// Hooking sweep that skips every entry whose row vertex is in component c
// (the largest after sampling): with the array and its mirror both swept,
// an edge is skipped on both sides only when both ends are already in c.
__global__ void __launch_bounds__(256)
k_cc_hook_skip(const uint64_t *__restrict__ slots, uint64_t cap, uint32_t *label, uint32_t c) {
    for_slot_pairs(slots, cap, [&](const uint64_t (&k)[2 * kCcPairs]) {
        uint32_t ru = 0;   // a root the source had (once in c's tree, always in c's component)
#pragma unroll
        for (int j = 0; j < 2 * kCcPairs; j++) {
            if (!is_edge_entry(k[j])) continue;
            const uint32_t u = key_src(k[j]);
            if (!(j & 1) || !is_edge_entry(k[j - 1]) || key_src(k[j - 1]) != u) ru = cc_find(label, u);
            if (ru == c) continue;
            cc_union(label, cc_find(label, u), cc_find(label, key_dst(k[j])));
        }
    });
}

// labels of n vertices at a fixed stride, for picking the largest component
__global__ void k_cc_pick(const uint32_t *__restrict__ label, uint64_t stride, uint32_t n, uint32_t *__restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = label[(uint64_t)i * stride];
}

__global__ void k_cc_compress(uint32_t *label, uint32_t V) {
    uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    uint32_t r = cc_find(label, (uint32_t)v);
    __hip_atomic_store(&label[v], r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

uint32_t grid_for_stream(uint64_t n_items, uint32_t per_thread) {
    uint64_t g = div_up(div_up(n_items, per_thread), 256);
    if (g > 256 * 64) g = 256 * 64;   // persistent-ish: 64 blocks per CU
    return (uint32_t)(g ? g : 1);
}

}  // namespace

namespace gpma_host {

void launch_pr_prep(const float *x, const uint32_t *deg, uint32_t V, bool uniform, double *contrib,
                    double *y, double *dangling, hipStream_t s) {
    hipMemsetAsync(dangling, 0, sizeof(double), s);
    const uint32_t blocks = (uint32_t)std::min<uint64_t>(div_up(V, 256), 1024);
    hipLaunchKernelGGL(k_pr_prep, dim3(blocks), dim3(256), 0, s, x, deg, V, uniform ? 1 : 0, contrib,
                       y, dangling);
}

void launch_pr_push(const uint64_t *slots, const uint16_t *cnt, uint64_t cap, uint32_t lf_log2,
                    const double *contrib, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_pr_push, dim3(grid_for_stream(cap, 2)), dim3(256), 0, s, slots, cnt, cap,
                       lf_log2, contrib, y);
}

void launch_pr_pull(const uint64_t *slots, const uint16_t *cnt, uint64_t cap, uint32_t lf_log2,
                    const double *contrib, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_pr_pull, dim3(grid_for_stream(cap, 4)), dim3(256), 0, s, slots, cnt, cap,
                       lf_log2, contrib, y);
}

__global__ void k_transpose_keys(const uint64_t *__restrict__ in, uint64_t n, uint64_t *__restrict__ out) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        uint64_t k = in[i];
        out[i] = (k << 32) | (k >> 32);
    }
}

void launch_transpose_keys(const uint64_t *in, uint64_t n, uint64_t *out, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_transpose_keys, dim3((uint32_t)div_up(n, 256)), dim3(256), 0, s, in, n, out);
}

void launch_pr_combine(const double *y, const double *dangling, uint32_t V, double damping, float *out,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_pr_combine, dim3((uint32_t)div_up(V, 256)), dim3(256), 0, s, y, dangling, V,
                       damping, out);
}

void launch_bfs_init(int32_t *dist, uint32_t V, uint32_t source, uint32_t *queue, uint32_t *qcount,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_bfs_init, dim3((uint32_t)div_up(V, 256)), dim3(256), 0, s, dist, V, source,
                       queue, qcount);
}

void launch_bfs_row_len(const uint32_t *row_ptr, const uint32_t *front, uint32_t nfront, uint32_t *len,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_bfs_row_len, dim3((uint32_t)div_up(nfront, 256)), dim3(256), 0, s, row_ptr,
                       front, nfront, len);
}

void launch_bfs_expand(const uint64_t *slots, const uint32_t *row_ptr, const uint32_t *front,
                       const uint32_t *offs, uint32_t nfront, const uint32_t *total, uint64_t max_total,
                       int32_t level, int32_t *dist, uint32_t *next, uint32_t *next_count, hipStream_t s) {
    hipLaunchKernelGGL(k_bfs_expand, dim3(grid_for_stream(max_total, kBfsItems)), dim3(256), 0, s, slots,
                       max_total, row_ptr, front, offs, nfront, total, level, dist, next, next_count);
}

void launch_bfs_bottom_up(const uint64_t *mslots, const uint32_t *mrow, uint32_t V, int32_t level,
                          int32_t *dist, uint32_t *next, uint32_t *next_count, hipStream_t s) {
    hipLaunchKernelGGL(k_bfs_bottom_up, dim3(grid_for_stream(V, 1)), dim3(256), 0, s, mslots, mrow, V,
                       level, dist, next, next_count);
}

void launch_cc_init(uint32_t *label, uint32_t V, hipStream_t s) {
    hipLaunchKernelGGL(k_cc_init, dim3((uint32_t)div_up(V, 256)), dim3(256), 0, s, label, V);
}

void launch_cc_hook(const uint64_t *slots, uint64_t cap, uint32_t *label, hipStream_t s) {
    hipLaunchKernelGGL(k_cc_hook, dim3(grid_for_stream(cap, 4)), dim3(256), 0, s, slots, cap, label);
}

void launch_cc_sample(const uint64_t *slots, const uint32_t *row_ptr, uint32_t V, uint32_t lf, uint32_t *label,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_cc_sample, dim3((uint32_t)div_up(V, 256)), dim3(256), 0, s, slots, row_ptr, V, lf, label);
}

void launch_cc_hook_skip(const uint64_t *slots, uint64_t cap, uint32_t *label, uint32_t c, hipStream_t s) {
    hipLaunchKernelGGL(k_cc_hook_skip, dim3(grid_for_stream(div_up(cap, 2), kCcPairs)), dim3(256), 0, s, slots, cap,
                       label, c);
}

void launch_cc_pick(const uint32_t *label, uint64_t stride, uint32_t n, uint32_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_cc_pick, dim3((n + 255) / 256), dim3(256), 0, s, label, stride, n, out);
}

void launch_cc_compress(uint32_t *label, uint32_t V, hipStream_t s) {
    hipLaunchKernelGGL(k_cc_compress, dim3((uint32_t)div_up(V, 256)), dim3(256), 0, s, label, V);
}

}  // namespace gpma_host
