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
    uint32_t pad[2];
    Ctl snap;          // control block of the stopped batch
};

// statistics of one completed batch
struct BatchOut {
    uint64_t applied;
    uint64_t noops;
    int64_t dn;
    uint64_t rewritten;
    uint32_t segs;
    uint32_t misses;    // learned-locator fallbacks
    uint32_t lookups;   // distinct keys located
    uint32_t pad;
};

}  // namespace gpma_dev

namespace gpma_host {

void launch_fetch(const gpma_dev::BatchDesc *desc, const gpma_dev::FusedState *st, const uint32_t *stop,
                  uint64_t *staging, uint32_t *cur_n, gpma_dev::Ctl *ctl, bool transpose, uint64_t cap,
                  hipStream_t s);
void launch_finish(gpma_dev::FusedState *st, uint32_t *stop, const gpma_dev::Ctl *ctl, const uint32_t *pending,
                   gpma_dev::BatchOut *out, hipStream_t s);

}  // namespace gpma_host
