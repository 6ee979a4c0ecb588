// Device side of fused batching: a sequence of update batches run without
// host synchronisation between batches.
//
// Batches go in windows.  A window's prefix (k_window_fetch, then one sort --
// the splitter sort up to 2^20 keys, else the radix sort) sorts all its
// batches at once: each key carries its batch's place in the window above
// the source bits, so one sort groups the keys by batch and orders them
// within; repeats stay, next to each other, and the leaf level takes a key
// equal to the one before it as a no-op.  As every key stays, batch j's keys
// start at the sum of the earlier batches' lengths, which the fetch writes.
// The window generation advances once the fetch is done: in the splitter
// sort's first launch, or in k_window_starts after the radix sort.
// Then, per batch, the locate kernel takes the batch's keys from the window's
// sorted keys (or nothing when the sequence is stopped), the state-dependent
// steps run (locate, merges, compactions; with no level above the leaves on
// the device, the leaf merge counts the batch's statistics and what is left
// itself), and k_finish either records the batch's statistics and advances to
// the next batch, or stops the sequence when the batch still has updates
// pending above the levels run on the device (those need the host-driven
// tiers: segments larger than LDS, or the root).  Batches that follow a stop
// see an empty batch and change nothing, so the pending state of the stopped
// batch survives until the host completes it.
#include "common.h"
#include "fused.h"
#include "bitonic.h"
#include "pair.h"

using namespace gpma_dev;

namespace {

__global__ void k_finish(FusedState *__restrict__ st, uint32_t *__restrict__ stop, Ctl *__restrict__ ctl,
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
    ctl->misses = 0;   // the next batch's locate counts from zero
    out[b].lookups = ctl->n_in;
    st->batch = b + 1;
}

// k_finish after a leaf merge that left per-block figures in part[4*i ..]
// (merged, no-ops, leaves merged, pending) instead of compacting: sum them
// into the control block (reset by the batch's locate), then finish.
// host (optional): the device view of the handle's pinned block, laid out
// like its fused block (state, then the stop flag, `head` bytes in all,
// then the per-batch results at `head`); the finished batch's state, stop
// flag and results are written there too, so the host reads them after the
// stream's synchronisation without a copy of its own.
struct FinishLeafOp {
    struct Args {
        FusedState *st;
        uint32_t *stop;
        Ctl *ctl;
        const uint4 *part;
        uint64_t nparts;
        int del;
        uint32_t lf;
        BatchOut *out;
        uint4 *host;
        uint32_t head;   // bytes, a multiple of 16
    };
    // thread 0, after its own stores to the fused block
    static __device__ __forceinline__ void publish(const Args &a, uint32_t b, bool with_out) {
        if (!a.host) return;
        const uint4 *blk = reinterpret_cast<const uint4 *>(a.st);   // the state opens the fused block
        for (uint32_t i = 0; i < a.head / 16; i++) a.host[i] = blk[i];
        if (with_out) {
            const uint4 *o = reinterpret_cast<const uint4 *>(a.out + b);
            uint4 *h = a.host + a.head / 16 + (uint64_t)b * (sizeof(BatchOut) / 16);
            for (uint32_t i = 0; i < sizeof(BatchOut) / 16; i++) h[i] = o[i];
        }
    }
    static __device__ __forceinline__ void run(const Args &a) {
        FusedState *__restrict__ st = a.st;
        uint32_t *__restrict__ stop = a.stop;
        Ctl *__restrict__ ctl = a.ctl;
        const uint4 *__restrict__ part = a.part;
        uint64_t nparts = a.nparts;
        int del = a.del;
        uint32_t lf = a.lf;
        BatchOut *__restrict__ out = a.out;
        __shared__ uint32_t red[4][1024 / kWave];
        if (*stop) return;   // this replay ran on an empty batch (block-uniform)
        uint32_t v[4] = {0, 0, 0, 0};
#pragma unroll 4
        for (uint64_t i = threadIdx.x; i < nparts; i += blockDim.x) {
            const uint4 p = part[i];
            v[0] += p.x;
            v[1] += p.y;
            v[2] += p.z;
            v[3] += p.w;
        }
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
            for (int d = kWave / 2; d >= 1; d >>= 1) v[q] += __shfl_xor(v[q], d, kWave);
        if (__lane_id() == 0)
#pragma unroll
            for (int q = 0; q < 4; q++) red[q][threadIdx.x / kWave] = v[q];
        __syncthreads();
        if (threadIdx.x != 0) return;
        uint32_t t[4] = {0, 0, 0, 0};
        for (int x = 0; x < 1024 / kWave; x++)
#pragma unroll
            for (int q = 0; q < 4; q++) t[q] += red[q][x];
        ctl->applied = t[0];
        ctl->dn = del ? -(int64_t)t[0] : (int64_t)t[0];
        ctl->noops = t[1];
        ctl->segs = t[2];
        ctl->rewritten = (uint64_t)t[2] * lf;
        ctl->lvl[0] = t[3];
        const uint32_t b = st->batch;
        if (ctl->err || t[3]) {
            st->snap = *ctl;
            st->halted = 1;
            *stop = 1;
            publish(a, b, false);
            return;
        }
        out[b].applied = t[0];
        out[b].noops = t[1];
        out[b].dn = ctl->dn;
        out[b].segs = t[2];
        out[b].rewritten = ctl->rewritten;
        out[b].misses = ctl->misses;
        ctl->misses = 0;
        out[b].lookups = ctl->n_in;
        st->batch = b + 1;
        publish(a, b, true);
    }
};

__global__ void __launch_bounds__(1024)
k_finish_leaf(FusedState *__restrict__ st, uint32_t *__restrict__ stop, Ctl *__restrict__ ctl,
              const uint4 *__restrict__ part, uint64_t nparts, int del, uint32_t lf, BatchOut *__restrict__ out) {
    FinishLeafOp::run(FinishLeafOp::Args{st, stop, ctl, part, nparts, del, lf, out, nullptr, 0});
}

// Window prefix.  Block-local table of the window's batch offsets (w <= 64),
// then a grid-stride copy of every key: validated (src < V, dst < V), the
// mirror's transposed, tagged with its batch's place in the window.  An
// invalid key marks its batch and is stored as the tagged key (0, 0); the
// batch is skipped as a whole later.  Every key of batch j carries tag j and
// the sort keeps repeats, so batch j's keys will start at offset j of the
// sorted window: the first block writes the offsets to ustart[0 .. w].
// With spl set (1024-thread blocks), the last block does not copy: it takes
// the splitter sort's regular sample of the window's keys straight from the
// batches, sorts it and writes the B-1 splitters, as the sort's own sampling
// launch would from the copied keys, while the other blocks copy.

// the window's key at position t (batch j = its tag); bad: src or dst >= V
__device__ __forceinline__ uint64_t window_key(const uint64_t *const *src, const uint64_t *off, uint32_t j,
                                               uint64_t t, int transpose, uint32_t V, uint32_t sb, bool &bad) {
    uint64_t k = src[j][t - off[j]];
    if (transpose) k = (k << 32) | (k >> 32);
    bad = key_src(k) >= V || key_dst(k) >= V;
    if (bad) k = 0;
    return k | ((uint64_t)j << (32 + sb));
}

template <int R>
__device__ void window_splitters(const uint64_t *const *src, const uint64_t *off, uint32_t w, uint64_t n,
                                 int transpose, uint32_t V, uint32_t sb, uint32_t B, uint64_t *spl, uint64_t *lds) {
    constexpr uint32_t S = 1024u * R;
    uint64_t k[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint64_t t = ((uint64_t)((uint32_t)r * 1024u + threadIdx.x) * n) / S;
        uint32_t j = 0;
        while (j + 1 < w && off[j + 1] <= t) j++;
        bool bad;
        k[r] = window_key(src, off, j, t, transpose, V, sb, bad);
    }
    block_bitonic<R>(k, lds, S);
#pragma unroll
    for (int r = 0; r < R; r++) lds[(uint32_t)r * 1024u + threadIdx.x] = k[r];
    __syncthreads();
    for (uint32_t j = threadIdx.x; j + 1 < B; j += blockDim.x) spl[j] = lds[((uint64_t)(j + 1) * S) / B];
}

struct WindowFetchOp {
    struct Args {
        const BatchDesc *desc;
        FusedState *st;
        const uint32_t *stop;
        uint32_t w;
        uint64_t n_max;
        uint32_t V;
        uint32_t sb;
        int transpose;
        uint64_t *staging;
        uint32_t *wcount;
        uint32_t *errs;
        uint32_t *ustart;
        uint64_t *spl;      // optional: the splitters, sampled by the last block
        uint32_t B;         // with spl: buckets of the splitter sort
        uint32_t S;         // with spl: its sample size (1024, 2048 or 4096)
    };
    static __device__ __forceinline__ void run(const Args &a) {
        const BatchDesc *__restrict__ desc = a.desc;
        FusedState *__restrict__ st = a.st;
        const uint32_t *__restrict__ stop = a.stop;
        uint32_t w = a.w;
        uint64_t n_max = a.n_max;
        uint32_t V = a.V;
        uint32_t sb = a.sb;
        int transpose = a.transpose;
        uint64_t *__restrict__ staging = a.staging;
        uint32_t *__restrict__ wcount = a.wcount;
        uint32_t *__restrict__ errs = a.errs;
        uint32_t *__restrict__ ustart = a.ustart;
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
        if (blockIdx.x == 0 && threadIdx.x <= w) ustart[threadIdx.x] = (uint32_t)off[threadIdx.x];
        const uint32_t copiers = a.spl ? gridDim.x - 1 : gridDim.x;
        if (blockIdx.x == copiers) {   // block-uniform: the sampling block
            __shared__ uint64_t lds[4096];
            if (a.B < 2) return;
            if (total == 0) {
                for (uint32_t j = threadIdx.x; j + 1 < a.B; j += blockDim.x) a.spl[j] = ~0ull;
                return;
            }
            if (a.S == 1024) window_splitters<1>(src, off, w, total, transpose, V, sb, a.B, a.spl, lds);
            else if (a.S == 2048) window_splitters<2>(src, off, w, total, transpose, V, sb, a.B, a.spl, lds);
            else window_splitters<4>(src, off, w, total, transpose, V, sb, a.B, a.spl, lds);
            return;
        }
        const uint64_t stride = (uint64_t)copiers * blockDim.x;
        for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
            uint32_t j = 0;
            while (j + 1 < w && off[j + 1] <= t) j++;
            bool bad;
            const uint64_t k = window_key(src, off, j, t, transpose, V, sb, bad);
            if (bad) errs[j] = gen;
            staging[t] = k;
        }
    }
};

__global__ void __launch_bounds__(256)
k_window_fetch(const BatchDesc *__restrict__ desc, FusedState *__restrict__ st, const uint32_t *__restrict__ stop,
               uint32_t w, uint64_t n_max, uint32_t V, uint32_t sb, int transpose, uint64_t *__restrict__ staging,
               uint32_t *__restrict__ wcount, uint32_t *__restrict__ errs, uint32_t *__restrict__ ustart) {
    WindowFetchOp::run(WindowFetchOp::Args{desc, st, stop, w, n_max, V, sb, transpose, staging, wcount, errs, ustart,
                                           nullptr, 0, 0});
}

struct WindowStartsOp {
    struct Args {
        const uint64_t *ukeys;
        const uint32_t *nuniq;
        uint32_t w;
        uint32_t sb;
        uint32_t *ustart;
        FusedState *st;
        Ctl *ctl;
    };
    static __device__ __forceinline__ void run(const Args &a) {
        const uint64_t *__restrict__ ukeys = a.ukeys;
        const uint32_t *__restrict__ nuniq = a.nuniq;
        uint32_t w = a.w;
        uint32_t sb = a.sb;
        uint32_t *__restrict__ ustart = a.ustart;
        FusedState *__restrict__ st = a.st;
        Ctl *__restrict__ ctl = a.ctl;
        const uint32_t j = threadIdx.x;
        if (j == 0) {
            st->gen = st->gen + 1;   // the fetch of this window is done with it
            ctl->misses = 0;         // the window's first locate counts from zero
        }
        if (j > w) return;
        const uint32_t n = *nuniq;
        ustart[j] = j == w ? n : lower_bound_u64(ukeys, n, (uint64_t)j << (32 + sb));
    }
};

__global__ void __launch_bounds__(256)
k_window_starts(const uint64_t *__restrict__ ukeys, const uint32_t *__restrict__ nuniq, uint32_t w, uint32_t sb,
                uint32_t *__restrict__ ustart, FusedState *__restrict__ st, Ctl *__restrict__ ctl) {
    WindowStartsOp::run(WindowStartsOp::Args{ukeys, nuniq, w, sb, ustart, st, ctl});
}

// Start of a fused call: the batch descriptors copied from the caller's
// pinned table (read over the bus) and each handle's state set to run from
// `batch`, halted and stop flags cleared (the window generation carries on).
__global__ void __launch_bounds__(256)
k_fused_begin(FusedState *__restrict__ st0, uint32_t *__restrict__ stop0, FusedState *__restrict__ st1,
              uint32_t *__restrict__ stop1, uint32_t batch, const BatchDesc *__restrict__ src,
              BatchDesc *__restrict__ dst, uint32_t count) {
    for (uint32_t i = threadIdx.x; i < count; i += blockDim.x) dst[i] = src[i];
    if (threadIdx.x == 0) {
        st0->batch = batch;
        st0->halted = 0;
        *stop0 = 0;
        if (st1) {
            st1->batch = batch;
            st1->halted = 0;
            *stop1 = 0;
        }
    }
}

}  // namespace

namespace gpma_host {

void launch_fused_begin(FusedState *st0, uint32_t *stop0, FusedState *st1, uint32_t *stop1, uint32_t batch,
                        const BatchDesc *src, BatchDesc *dst, uint32_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_fused_begin, dim3(1), dim3(256), 0, s, st0, stop0, st1, stop1, batch, src, dst, count);
}


void launch_finish(FusedState *st, uint32_t *stop, Ctl *ctl, const uint32_t *pending, BatchOut *out,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, st, stop, ctl, pending, out);
}

void launch_finish_leaf(FusedState *st, uint32_t *stop, Ctl *ctl, const uint32_t *part, uint64_t nparts, bool del,
                        uint32_t lf, BatchOut *out, hipStream_t s) {
    hipLaunchKernelGGL(k_finish_leaf, dim3(1), dim3(1024), 0, s, st, stop, ctl, reinterpret_cast<const uint4 *>(part),
                       nparts, del ? 1 : 0, lf, out);
}

static uint32_t copy_blocks(uint64_t n) {
    uint64_t b = (n + 255) / 256;
    return (uint32_t)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

void launch_window_fetch(const BatchDesc *desc, FusedState *st, const uint32_t *stop, uint32_t w, uint64_t n_max,
                         uint32_t V, uint32_t sb, bool transpose, uint64_t *staging, uint32_t *wcount, uint32_t *errs,
                         uint32_t *ustart, hipStream_t s) {
    hipLaunchKernelGGL(k_window_fetch, dim3(copy_blocks(n_max)), dim3(256), 0, s, desc, st, stop, w, n_max, V, sb,
                       transpose ? 1 : 0, staging, wcount, errs, ustart);
}

void launch_window_starts(const uint64_t *ukeys, const uint32_t *nuniq, uint32_t w, uint32_t sb, uint32_t *ustart,
                          FusedState *st, Ctl *ctl, hipStream_t s) {
    hipLaunchKernelGGL(k_window_starts, dim3(1), dim3(128), 0, s, ukeys, nuniq, w, sb, ustart, st, ctl);
}

// ---- paired launches (the array at y = 0, its mirror at y = 1)

void launch_window_fetch2(const BatchDesc *desc, FusedState *const st[2], const uint32_t *const stop[2], uint32_t w,
                          uint64_t n_max, uint32_t V, uint32_t sb, uint64_t *const staging[2],
                          uint32_t *const wcount[2], uint32_t *const errs[2], uint32_t *const ustart[2],
                          uint64_t *const spl[2], uint32_t B, uint32_t S, hipStream_t s) {
    WindowFetchOp::Args a[2];
    for (int k = 0; k < 2; k++)
        a[k] = {desc, st[k], stop[k], w, n_max, V, sb, k, staging[k], wcount[k], errs[k], ustart[k], spl[k], B, S};
    // 1024-thread blocks: the copying ones, then the sampling one
    uint64_t copiers = (n_max + 1023) / 1024;
    if (copiers < 1) copiers = 1;
    if (copiers > 256) copiers = 256;
    launch_pair<WindowFetchOp, 1024>((uint32_t)copiers + 1, a[0], a[1], s);
}

void launch_finish_leaf2(FusedState *const st[2], uint32_t *const stop[2], Ctl *const ctl[2],
                         const uint32_t *const part[2], uint64_t nparts, bool del, uint32_t lf,
                         BatchOut *const out[2], void *const host[2], uint32_t head, hipStream_t s) {
    FinishLeafOp::Args a[2];
    for (int k = 0; k < 2; k++)
        a[k] = {st[k], stop[k], ctl[k], reinterpret_cast<const uint4 *>(part[k]), nparts, del ? 1 : 0, lf, out[k],
                static_cast<uint4 *>(host[k]), head};
    launch_pair<FinishLeafOp, 1024>(1, a[0], a[1], s);
}

}  // namespace gpma_host
