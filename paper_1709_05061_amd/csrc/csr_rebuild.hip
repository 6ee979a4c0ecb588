// Comparator: a plain CSR (sorted edge array without gaps, plus row offsets)
// rebuilt on every batch, the role the GPU CSR of cuSparse plays among the
// paper's baselines (Section 6, "GPU-based CSR": updates are applied by
// rebuilding the format).  A batch is sorted, its no-ops are dropped, the
// remainder is merged into (or removed from) the whole edge array, and the
// row offsets are recomputed: O(|E|) work per batch however small the batch,
// which is what GPMA+ avoids.
#include <algorithm>

#include "common.h"

using namespace gpma_dev;

namespace {

inline uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// flag[i] = 1 when U[i] changes the set: absent for an insert, present for a
// delete (U sorted unique, A sorted)
__global__ void k_csr_effective(const uint64_t *__restrict__ A, uint64_t na, const uint64_t *__restrict__ U,
                                const uint32_t *__restrict__ nu, uint64_t b, int del, uint32_t *__restrict__ flag) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= b) return;
    if (t >= *nu) {   // past the distinct keys: nothing (the scan covers all b)
        flag[t] = 0;
        return;
    }
    const uint64_t u = U[t];
    uint64_t lo = 0, hi = na;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (A[mid] < u) lo = mid + 1; else hi = mid;
    }
    const bool present = lo < na && A[lo] == u;
    flag[t] = (del ? present : !present) ? 1u : 0u;
}

__global__ void k_csr_compact(const uint64_t *__restrict__ U, const uint32_t *__restrict__ nu,
                              const uint32_t *__restrict__ flag, const uint32_t *__restrict__ pos,
                              uint64_t *__restrict__ out) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < *nu && flag[t]) out[pos[t]] = U[t];
}

// row offsets of the sorted edge array E (n edges): thread i writes the
// starts of the rows from src(E[i-1])+1 through src(E[i]); the last thread
// closes the rows after the final edge
__global__ void k_csr_rows(const uint64_t *__restrict__ E, uint64_t n, uint32_t V, uint64_t *__restrict__ row_ptr) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const uint64_t lo = i == 0 ? 0 : (uint64_t)key_src(E[i - 1]) + 1;
    const uint64_t hi = i == n ? (uint64_t)V : (uint64_t)key_src(E[i]);
    for (uint64_t u = lo; u <= hi; u++) row_ptr[u] = i;
}

}  // namespace

struct gpma_csr {
    uint32_t V = 0;
    uint64_t n = 0, cap = 0;
    uint64_t *E = nullptr, *E2 = nullptr;   // edges, and the rebuild target
    uint64_t *row_ptr = nullptr;           // V + 1
    uint64_t bcap = 0;
    uint64_t *kA = nullptr, *kB = nullptr, *kC = nullptr;
    uint32_t *flag = nullptr, *tmp = nullptr, *cnt = nullptr;   // flag: 2 x batch; cnt: [unique, effective]
    uint32_t *cnt_h = nullptr;
    Ctl *ctl = nullptr;
};

namespace {

template <typename T>
int alloc(T **p, uint64_t count) {
    *p = nullptr;
    if (hipMalloc((void **)p, (count ? count : 1) * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return GPMA_ENOMEM;
    }
    return GPMA_OK;
}
template <typename T>
void release(T *&p) {
    if (p) hipFree((void *)p);
    p = nullptr;
}

uint32_t bits_for(uint32_t V) {
    uint32_t b = 0;
    for (uint64_t x = V ? V - 1 : 0; x; x >>= 1) b++;
    return b;
}

int ensure_edges(gpma_csr *c, uint64_t need) {
    if (need <= c->cap) return GPMA_OK;
    const uint64_t want = need + need / 4 + 1024;
    uint64_t *e = nullptr, *e2 = nullptr;
    if (alloc(&e, want) || alloc(&e2, want)) {
        release(e);
        release(e2);
        return GPMA_ENOMEM;
    }
    if (c->n) hipMemcpy(e, c->E, c->n * sizeof(uint64_t), hipMemcpyDeviceToDevice);
    release(c->E);
    release(c->E2);
    c->E = e;
    c->E2 = e2;
    c->cap = want;
    return GPMA_OK;
}

int ensure_scratch(gpma_csr *c, uint64_t b) {
    if (b <= c->bcap) return GPMA_OK;
    release(c->kA); release(c->kB); release(c->kC); release(c->flag); release(c->tmp);
    c->bcap = 0;
    const uint64_t n = std::max<uint64_t>(b, 4096);
    const size_t tw = std::max(gpma_host::radix_tmp_words(n), gpma_host::scan_tmp_words(n + 1));
    int e = GPMA_OK;
    e |= alloc(&c->kA, n); e |= alloc(&c->kB, n); e |= alloc(&c->kC, n);
    e |= alloc(&c->flag, 2 * n + 2); e |= alloc(&c->tmp, tw);
    if (e) return GPMA_ENOMEM;
    c->bcap = n;
    return GPMA_OK;
}

void build_rows(gpma_csr *c, hipStream_t s) {
    hipLaunchKernelGGL(k_csr_rows, dim3((uint32_t)div_up(c->n + 1, 256)), dim3(256), 0, s, c->E, c->n, c->V,
                       c->row_ptr);
}

}  // namespace

extern "C" {

int gpma_csr_create(gpma_csr_t **out, uint32_t V, const uint64_t *keys, uint64_t n, hipStream_t s) {
    if (!out) return GPMA_EINVAL;
    *out = nullptr;
    if (V == 0 || V > (1u << 31) || (n && !keys)) return GPMA_EINVAL;
    gpma_csr *c = new (std::nothrow) gpma_csr();
    if (!c) return GPMA_ENOMEM;
    c->V = V;
    int e = alloc(&c->row_ptr, (uint64_t)V + 1) | alloc(&c->cnt, 2) | alloc(&c->ctl, 1);
    if (!e && hipHostMalloc((void **)&c->cnt_h, 2 * sizeof(uint32_t), 0) != hipSuccess) e = GPMA_ENOMEM;
    if (!e) e = ensure_edges(c, std::max<uint64_t>(n, 1));
    if (!e && n) {
        // the initial set: one rebuild from empty
        c->n = 0;
        e = gpma_csr_update(c, keys, n, 0, s);
    } else if (!e) {
        build_rows(c, s);
        hipStreamSynchronize(s);
    }
    if (e) {
        gpma_csr_destroy(c);
        return e;
    }
    *out = c;
    return GPMA_OK;
}

void gpma_csr_destroy(gpma_csr_t *c) {
    if (!c) return;
    release(c->E); release(c->E2); release(c->row_ptr);
    release(c->kA); release(c->kB); release(c->kC); release(c->flag); release(c->tmp); release(c->cnt);
    release(c->ctl);
    if (c->cnt_h) hipHostFree(c->cnt_h);
    delete c;
}

int gpma_csr_update(gpma_csr_t *c, const uint64_t *keys, uint64_t b, int del, hipStream_t s) {
    if (!c || (b && !keys) || b >= (1ull << 31)) return GPMA_EINVAL;
    if (b == 0) return GPMA_OK;
    int e = ensure_scratch(c, b);
    if (e) return e;
    const uint32_t sb = bits_for(c->V);
    // validation rides on the sort's first pass
    hipMemsetAsync(c->ctl, 0, sizeof(Ctl), s);
    const uint64_t *sorted =
        gpma_host::radix_sort_keys(keys, b, sb, sb, c->V, c->kA, c->kB, c->tmp, s, nullptr, c->ctl);
    uint64_t *uq = sorted == c->kA ? c->kB : c->kA;
    gpma_host::unique_sorted(sorted, b, uq, &c->cnt[0], c->flag, c->tmp, s);
    hipMemcpyAsync(c->cnt_h, &c->ctl->err, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    hipStreamSynchronize(s);
    if (c->cnt_h[0]) return GPMA_EINVAL;
    // drop no-ops, then merge or remove over the whole edge array
    hipLaunchKernelGGL(k_csr_effective, dim3((uint32_t)div_up(b, 256)), dim3(256), 0, s, c->E, c->n, uq,
                       &c->cnt[0], b, del, c->flag);
    gpma_host::scan_u32(c->flag, c->flag + b, b, &c->cnt[1], c->tmp, s);
    hipLaunchKernelGGL(k_csr_compact, dim3((uint32_t)div_up(b, 256)), dim3(256), 0, s, uq, &c->cnt[0], c->flag,
                       c->flag + b, c->kC);
    hipMemcpyAsync(c->cnt_h, c->cnt, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    hipStreamSynchronize(s);
    const uint64_t k = c->cnt_h[1];
    const uint64_t n2 = del ? c->n - k : c->n + k;
    e = ensure_edges(c, n2);
    if (e) return e;
    gpma_host::launch_merge_sorted(del != 0, c->E, c->n, c->kC, k, c->E2, s);
    std::swap(c->E, c->E2);
    c->n = n2;
    build_rows(c, s);
    return GPMA_OK;
}

uint64_t gpma_csr_num_edges(const gpma_csr_t *c) { return c ? c->n : 0; }

int gpma_csr_export(const gpma_csr_t *c, uint64_t *keys_out, uint64_t max_keys, uint64_t *row_ptr_out,
                    hipStream_t s) {
    if (!c || (keys_out && max_keys < c->n)) return GPMA_EINVAL;
    if (keys_out && c->n) hipMemcpyAsync(keys_out, c->E, c->n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
    if (row_ptr_out)
        hipMemcpyAsync(row_ptr_out, c->row_ptr, ((uint64_t)c->V + 1) * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
    return GPMA_OK;
}

}  // extern "C"
