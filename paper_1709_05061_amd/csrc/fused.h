// Shared declarations of fused batching (device descriptors and state).
#pragma once

#include "common.h"

namespace gpma_dev {

// one batch of a fused sequence (device copy of the caller's table)
struct BatchDesc {
    const uint64_t *keys;
    uint64_t n;
};

// per-handle progress through the sequence
struct FusedState {
    uint32_t batch;    // next batch to run
    uint32_t halted;   // 1: stopped at `batch` with work left for the host
    uint32_t wstart;   // first batch of the current window
    uint32_t gen;      // window generation (starts at 1): errs[j] == gen - 1 marks batch j invalid
    Ctl snap;          // control block of the stopped batch
};

// a window's batches are sorted together: batch j of the window carries the
// tag j in the key's source field above the source bits
constexpr uint32_t kWindowTagBits = 6;
constexpr uint32_t kWindowMax = 1u << kWindowTagBits;

// statistics of one completed batch
struct BatchOut {
    uint64_t applied;
    uint64_t noops;
    int64_t dn;
    uint64_t rewritten;
    uint32_t segs;
    uint32_t misses;    // learned-locator fallbacks
    uint32_t lookups;   // keys located (repeats included)
    uint32_t pad;
};
static_assert(sizeof(BatchOut) % 16 == 0, "results are copied in 16-byte words");

}  // namespace gpma_dev

namespace gpma_host {

void launch_finish(gpma_dev::FusedState *st, uint32_t *stop, gpma_dev::Ctl *ctl, const uint32_t *pending,
                   gpma_dev::BatchOut *out, hipStream_t s);
// the same after a leaf merge that wrote per-block figures to part (nparts
// blocks): their sums go into ctl (lvl[0]: the updates left pending) first
void launch_finish_leaf(gpma_dev::FusedState *st, uint32_t *stop, gpma_dev::Ctl *ctl, const uint32_t *part,
                        uint64_t nparts, bool del, uint32_t lf, gpma_dev::BatchOut *out, hipStream_t s);

// window prefix: the w batches from st->batch, validated, tagged and
// concatenated into staging (count to *wcount); errs[j] = st->gen for a
// batch with an invalid key; ustart[j] = where batch j's keys will start in
// the sorted window (j <= w).  n_max bounds the window's total keys.  Before
// the window's first locate, st->gen must advance and ctl->misses be zeroed
// (by launch_window_starts, or by the splitter sort's bookkeeping).
void launch_window_fetch(const gpma_dev::BatchDesc *desc, gpma_dev::FusedState *st, const uint32_t *stop,
                         uint32_t w, uint64_t n_max, uint32_t V, uint32_t sb, bool transpose, uint64_t *staging,
                         uint32_t *wcount, uint32_t *errs, uint32_t *ustart, hipStream_t s);
// first position of each batch's keys in the window's sorted keys (the
// values the fetch wrote); advances st->gen and zeroes ctl->misses
void launch_window_starts(const uint64_t *ukeys, const uint32_t *nuniq, uint32_t w, uint32_t sb, uint32_t *ustart,
                          gpma_dev::FusedState *st, gpma_dev::Ctl *ctl, hipStream_t s);

// The fetch and the finishing step for the array (index 0) and its mirror
// (index 1, keys transposed) in one launch each.  The paired fetch also
// writes the splitter sort's splitters to spl[k] (B buckets, sample size S:
// splitter_buckets, splitter_sample_size, splitter_spl).
void launch_window_fetch2(const gpma_dev::BatchDesc *desc, gpma_dev::FusedState *const st[2],
                          const uint32_t *const stop[2], uint32_t w, uint64_t n_max, uint32_t V, uint32_t sb,
                          uint64_t *const staging[2], uint32_t *const wcount[2], uint32_t *const errs[2],
                          uint32_t *const ustart[2], uint64_t *const spl[2], uint32_t B, uint32_t S, hipStream_t s);
// (host[k]: the device view of side k's pinned block of the fused block's
// layout; each finished batch's state, stop flag and results go there too)
void launch_finish_leaf2(gpma_dev::FusedState *const st[2], uint32_t *const stop[2], gpma_dev::Ctl *const ctl[2],
                         const uint32_t *const part[2], uint64_t nparts, bool del, uint32_t lf,
                         gpma_dev::BatchOut *const out[2], void *const host[2], uint32_t head, hipStream_t s);

// Start of a fused call: count descriptors copied from src (the caller's
// pinned table, device view) to dst, and each handle's state set to run from
// `batch` with its halted and stop flags cleared (st1/stop1 may be null).
void launch_fused_begin(gpma_dev::FusedState *st0, uint32_t *stop0, gpma_dev::FusedState *st1, uint32_t *stop1,
                        uint32_t batch, const gpma_dev::BatchDesc *src, gpma_dev::BatchDesc *dst, uint32_t count,
                        hipStream_t s);

}  // namespace gpma_host

