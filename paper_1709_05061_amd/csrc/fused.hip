// Device side of fused batching: a sequence of update batches replayed from
// captured HIP graphs without host synchronisation between batches.
//
// Every replay of a batch graph starts with k_fetch, which takes the next
// batch from a descriptor table (or nothing when the sequence is stopped),
// and ends with k_finish, which either records the batch's statistics and
// advances to the next descriptor, or stops the sequence when the batch still
// has updates pending above the levels the graph covers (those need the
// host-driven tiers: segments larger than LDS, or the root).  Batches that
// follow a stop see a zero-length batch and change nothing, so the pending
// state of the stopped batch survives until the host completes it.
#include "common.h"
#include "fused.h"

using namespace gpma_dev;

namespace {

__global__ void __launch_bounds__(256)
k_fetch(const BatchDesc *__restrict__ desc, const FusedState *__restrict__ st,
        const uint32_t *__restrict__ stop, uint64_t *__restrict__ staging, uint32_t *__restrict__ cur_n,
        Ctl *__restrict__ ctl, int transpose, uint64_t cap) {
    const bool stopped = *stop != 0;
    const uint32_t b = st->batch;
    uint64_t n = stopped ? 0 : desc[b].n;
    if (n > cap) n = cap;
    const uint64_t *src = desc[b].keys;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t k = src[i];
        staging[i] = transpose ? ((k << 32) | (k >> 32)) : k;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->err = 0;
        ctl->n_in = 0;
        ctl->lvl[0] = 0;
        ctl->lvl[1] = 0;
        ctl->segs = 0;
        ctl->applied = 0;
        ctl->noops = 0;
        ctl->dn = 0;
        ctl->rewritten = 0;
        ctl->misses = 0;
        *cur_n = (uint32_t)n;
    }
}

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

}  // namespace

namespace gpma_host {

void launch_fetch(const BatchDesc *desc, const FusedState *st, const uint32_t *stop, uint64_t *staging,
                  uint32_t *cur_n, Ctl *ctl, bool transpose, uint64_t cap, hipStream_t s) {
    uint64_t blocks = (cap + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_fetch, dim3((uint32_t)blocks), dim3(256), 0, s, desc, st, stop, staging, cur_n, ctl,
                       transpose ? 1 : 0, cap);
}

void launch_finish(FusedState *st, uint32_t *stop, const Ctl *ctl, const uint32_t *pending, BatchOut *out,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, st, stop, ctl, pending, out);
}

}  // namespace gpma_host
