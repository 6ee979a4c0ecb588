// Analytics that read the PMA in place (Section 4.2: existing algorithms run
// on CSR-on-GPMA once they skip gaps and guards; Section 6.1 "Applications").
//   PageRank: matrix-based; push over the sorted slot stream, fp64 sums.
//   BFS:      vertex-centric; rows via the CSR offsets, wave per frontier row.
//   CC:       edge-centric; hooking over the slot stream + pointer jumping.
#include "common.h"

using namespace gpma_dev;

namespace {

inline uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// PageRank: x'[v] = (1-d)/V + d * (sum_{u->v} x[u]/outdeg(u) + D/V)

__global__ void __launch_bounds__(256)
k_pr_prep(const float *__restrict__ x, const uint32_t *__restrict__ deg, uint32_t V, int uniform,
          double *__restrict__ contrib, double *__restrict__ y, double *__restrict__ dangling) {
    __shared__ double part[256 / kWave];
    uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double dm = 0.0;
    if (v < V) {
        double xv = uniform ? 1.0 / (double)V : (double)x[v];
        uint32_t dv = deg[v];
        contrib[v] = dv ? xv / (double)dv : 0.0;
        if (!dv) dm = xv;
        y[v] = 0.0;
    }
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) dm += __shfl_xor(dm, d, kWave);
    if (__lane_id() == 0) part[threadIdx.x / kWave] = dm;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 256 / kWave; w++) t += part[w];
        if (t != 0.0) unsafeAtomicAdd(dangling, t);
    }
}

// Push y[dst] += contrib[src] for every stored edge.  The slot stream is read
// once, coalesced; src is non-decreasing along it, so contrib[src] reads hit
// cache; the scatter into y goes through fp64 atomics.
__global__ void __launch_bounds__(256)
k_pr_spmv(const uint64_t *__restrict__ slots, uint64_t cap, const double *__restrict__ contrib,
          double *__restrict__ y) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x * 2;
    for (uint64_t p = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2; p < cap; p += stride) {
        const ulonglong2 kk = *reinterpret_cast<const ulonglong2 *>(slots + p);
        if (kk.x != kEmpty && !is_guard(kk.x)) unsafeAtomicAdd(&y[key_dst(kk.x)], contrib[key_src(kk.x)]);
        if (kk.y != kEmpty && !is_guard(kk.y)) unsafeAtomicAdd(&y[key_dst(kk.y)], contrib[key_src(kk.y)]);
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

// One wave per frontier vertex walks its row [row_ptr[u], row_ptr[u+1]),
// skipping gaps and the guard (the IsEntryExist test of Algorithm "GPU-based
// BFS Neighbour Gathering").  New vertices are claimed with a CAS on dist and
// appended with one atomic per wave.
__global__ void __launch_bounds__(256)
k_bfs_expand(const uint64_t *__restrict__ slots, const uint32_t *__restrict__ row_ptr,
             const uint32_t *__restrict__ front, uint32_t nfront, int32_t level,
             int32_t *__restrict__ dist, uint32_t *__restrict__ next, uint32_t *__restrict__ next_count) {
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint32_t lane = __lane_id();
    if (wave >= nfront) return;
    const uint32_t u = front[wave];
    const uint32_t beg = row_ptr[u], end = row_ptr[u + 1];
    for (uint32_t p0 = beg; p0 < end; p0 += kWave) {
        uint32_t p = p0 + lane;
        bool claim = false;
        uint32_t v = 0;
        if (p < end) {
            uint64_t k = slots[p];
            if (k != kEmpty && !is_guard(k)) {
                v = key_dst(k);
                if (__hip_atomic_load(&dist[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < 0)
                    claim = atomicCAS(&dist[v], -1, level + 1) == -1;
            }
        }
        uint64_t m = __ballot(claim);
        if (m) {
            uint32_t leader = __ffsll((unsigned long long)m) - 1;
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

__global__ void k_cc_init(uint32_t *__restrict__ label, uint32_t V) {
    uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < V) label[v] = (uint32_t)v;
}

__global__ void __launch_bounds__(256)
k_cc_hook(const uint64_t *__restrict__ slots, uint64_t cap, uint32_t *label, uint32_t *changed) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    bool any = false;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < cap; p += stride) {
        uint64_t k = slots[p];
        if (k == kEmpty || is_guard(k)) continue;
        uint32_t a = cc_find(label, key_src(k));
        uint32_t b = cc_find(label, key_dst(k));
        if (a != b) {
            uint32_t hi = a > b ? a : b, lo = a > b ? b : a;
            atomicMin(&label[hi], lo);
            any = true;
        }
    }
    if (__ballot(any) && __lane_id() == 0) atomicOr(changed, 1u);
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
    hipLaunchKernelGGL(k_pr_prep, dim3((uint32_t)div_up(V, 256)), dim3(256), 0, s, x, deg, V,
                       uniform ? 1 : 0, contrib, y, dangling);
}

void launch_pr_spmv(const uint64_t *slots, uint64_t cap, const double *contrib, double *y,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_pr_spmv, dim3(grid_for_stream(cap, 2)), dim3(256), 0, s, slots, cap, contrib, y);
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

void launch_bfs_expand(const uint64_t *slots, const uint32_t *row_ptr, const uint32_t *front,
                       uint32_t nfront, int32_t level, int32_t *dist, uint32_t *next,
                       uint32_t *next_count, hipStream_t s) {
    uint64_t threads = (uint64_t)nfront * kWave;
    hipLaunchKernelGGL(k_bfs_expand, dim3((uint32_t)div_up(threads, 256)), dim3(256), 0, s, slots,
                       row_ptr, front, nfront, level, dist, next, next_count);
}

void launch_cc_init(uint32_t *label, uint32_t V, hipStream_t s) {
    hipLaunchKernelGGL(k_cc_init, dim3((uint32_t)div_up(V, 256)), dim3(256), 0, s, label, V);
}

void launch_cc_hook(const uint64_t *slots, uint64_t cap, uint32_t *label, uint32_t *changed,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_cc_hook, dim3(grid_for_stream(cap, 4)), dim3(256), 0, s, slots, cap, label,
                       changed);
}

void launch_cc_compress(uint32_t *label, uint32_t V, hipStream_t s) {
    hipLaunchKernelGGL(k_cc_compress, dim3((uint32_t)div_up(V, 256)), dim3(256), 0, s, label, V);
}

}  // namespace gpma_host
