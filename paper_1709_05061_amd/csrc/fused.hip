// Device side of fused batching: a sequence of update batches run without
// host synchronisation between batches.
//
// Batches go in windows.  A window's prefix (k_window_fetch, one radix sort,
// unique, k_window_starts) sorts all its batches at once: each key carries its
// batch's place in the window above the source bits, so one sort groups the
// keys by batch and orders them within.  Then, per batch, k_window_select
// takes the batch's keys from the window's unique keys (or nothing when the
// sequence is stopped), the state-dependent steps run (locate, merges,
// compactions), and k_finish either records the batch's statistics and
// advances to the next batch, or stops the sequence when the batch still has
// updates pending above the levels run on the device (those need the
// host-driven tiers: segments larger than LDS, or the root).  Batches that
// follow a stop see an empty batch and change nothing, so the pending state of
// the stopped batch survives until the host completes it.
#include "common.h"
#include "fused.h"

using namespace gpma_dev;

namespace {

__global__ void k_finish(FusedState *__restrict__ st, uint32_t *__restrict__ stop, const Ctl *__restrict__ ctl,
                         const uint32_t *__restrict__ pending, BatchOut *__restrict__ out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    if (*stop) return;   // this replay ran on an empty batch
    const uint32_t b = st->batch;
    if (ctl->err || *pending) {
        st->snap = *ctl;
        st->halted = 1;
        *stop = 1;
        return;
    }
    out[b].applied = ctl->applied;
    out[b].noops = ctl->noops;
    out[b].dn = ctl->dn;
    out[b].segs = ctl->segs;
    out[b].rewritten = ctl->rewritten;
    out[b].misses = ctl->misses;
    out[b].lookups = ctl->n_in;
    st->batch = b + 1;
}

// Window prefix.  Block-local table of the window's batch offsets (w <= 64),
// then a grid-stride copy of every key: validated (src < V, dst < V), the
// mirror's transposed, tagged with its batch's place in the window.  An
// invalid key marks its batch and is stored as the tagged key (0, 0); the
// batch is skipped as a whole later.
__global__ void __launch_bounds__(256)
k_window_fetch(const BatchDesc *__restrict__ desc, FusedState *__restrict__ st, const uint32_t *__restrict__ stop,
               uint32_t w, uint64_t n_max, uint32_t V, uint32_t sb, int transpose, uint64_t *__restrict__ staging,
               uint32_t *__restrict__ wcount, uint32_t *__restrict__ errs) {
    __shared__ uint64_t off[kWindowMax + 1];
    __shared__ const uint64_t *src[kWindowMax];
    const uint32_t b0 = st->batch;
    const uint32_t gen = st->gen;
    if (threadIdx.x == 0) {
        uint64_t o = 0;
        for (uint32_t j = 0; j < w; j++) {
            off[j] = o;
            src[j] = desc[b0 + j].keys;
            o += *stop ? 0 : desc[b0 + j].n;
        }
        off[w] = o < n_max ? o : n_max;
    }
    __syncthreads();
    const uint64_t total = off[w];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *wcount = (uint32_t)total;
        st->wstart = b0;
    }
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        uint32_t j = 0;
        while (j + 1 < w && off[j + 1] <= t) j++;
        uint64_t k = src[j][t - off[j]];
        if (transpose) k = (k << 32) | (k >> 32);
        if (key_src(k) >= V || key_dst(k) >= V) {
            errs[j] = gen;
            k = 0;
        }
        staging[t] = k | ((uint64_t)j << (32 + sb));
    }
}

__global__ void __launch_bounds__(256)
k_window_starts(const uint64_t *__restrict__ ukeys, const uint32_t *__restrict__ nuniq, uint32_t w, uint32_t sb,
                uint32_t *__restrict__ ustart, FusedState *__restrict__ st) {
    const uint32_t j = threadIdx.x;
    if (j == 0) st->gen = st->gen + 1;   // the fetch of this window is done with it
    if (j > w) return;
    const uint32_t n = *nuniq;
    ustart[j] = j == w ? n : lower_bound_u64(ukeys, n, (uint64_t)j << (32 + sb));
}

__global__ void __launch_bounds__(256)
k_window_select(const FusedState *__restrict__ st, const uint32_t *__restrict__ stop, const uint64_t *__restrict__ ukeys,
                const uint32_t *__restrict__ ustart, const uint32_t *__restrict__ errs, uint32_t sb, uint64_t n_max,
                uint64_t *__restrict__ dense, Ctl *__restrict__ ctl) {
    const uint32_t j = st->batch - st->wstart;
    const bool stopped = *stop != 0;
    const uint64_t beg = ustart[j];
    uint64_t n = stopped ? 0 : ustart[j + 1] - beg;
    if (n > n_max) n = n_max;
    const uint64_t tag_mask = ~(((1ull << kWindowTagBits) - 1) << (32 + sb));
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dense[i] = ukeys[beg + i] & tag_mask;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->err = (!stopped && errs[j] == st->gen - 1) ? 1u : 0u;
        ctl->n_in = (uint32_t)n;
        ctl->lvl[0] = 0;
        ctl->lvl[1] = 0;
        ctl->segs = 0;
        ctl->applied = 0;
        ctl->noops = 0;
        ctl->dn = 0;
        ctl->rewritten = 0;
        ctl->misses = 0;
    }
}

}  // namespace

namespace gpma_host {

void launch_finish(FusedState *st, uint32_t *stop, const Ctl *ctl, const uint32_t *pending, BatchOut *out,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, st, stop, ctl, pending, out);
}

static uint32_t copy_blocks(uint64_t n) {
    uint64_t b = (n + 255) / 256;
    return (uint32_t)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

void launch_window_fetch(const BatchDesc *desc, FusedState *st, const uint32_t *stop, uint32_t w, uint64_t n_max,
                         uint32_t V, uint32_t sb, bool transpose, uint64_t *staging, uint32_t *wcount, uint32_t *errs,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_window_fetch, dim3(copy_blocks(n_max)), dim3(256), 0, s, desc, st, stop, w, n_max, V, sb,
                       transpose ? 1 : 0, staging, wcount, errs);
}

void launch_window_starts(const uint64_t *ukeys, const uint32_t *nuniq, uint32_t w, uint32_t sb, uint32_t *ustart,
                          FusedState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_window_starts, dim3(1), dim3(128), 0, s, ukeys, nuniq, w, sb, ustart, st);
}

void launch_window_select(const FusedState *st, const uint32_t *stop, const uint64_t *ukeys, const uint32_t *ustart,
                          const uint32_t *errs, uint32_t sb, uint64_t n_max, uint64_t *dense, Ctl *ctl,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_window_select, dim3(copy_blocks(n_max)), dim3(256), 0, s, st, stop, ukeys, ustart, errs, sb,
                       n_max, dense, ctl);
}

}  // namespace gpma_host
