// Learned segment locator: model parameters and launchers.
#pragma once

#include "common.h"

namespace gpma_dev {

// 2 -> 32 -> 1 MLP with a skip term: position = x + w2 . relu(W1 [x y] + b1) + b2
struct LocModel {
    float w1x[32], w1y[32], b1[32];   // layer 1 (fp32)
    uint16_t w2[32];                  // layer 2 weights (bf16 bit patterns)
    float b2;
    float inv_v, inv_v1;              // feature scales 1/V and 1/(V+1)
    uint32_t V;
    uint32_t L;                       // leaves the model was fitted for
    uint32_t eps;                     // max leaf error over all pivots
    uint32_t valid;
};

}  // namespace gpma_dev

namespace gpma_host {

void launch_locate_learned(const uint64_t *keys, const uint32_t *n_dev, uint64_t n_max, const uint64_t *slots,
                           uint64_t L, uint32_t lf_log2, const gpma_dev::LocModel *model,
                           const gpma_dev::Ctl *ctl, uint32_t *leaf, uint8_t *status, uint32_t *misses,
                           hipStream_t s);
size_t loc_gram_words();
void launch_loc_gram(const uint64_t *slots, uint64_t L, uint32_t lf_log2, uint64_t stride, uint64_t S,
                     const gpma_dev::LocModel *model, double *gram, hipStream_t s);
void launch_loc_eval(const uint64_t *slots, uint64_t L, uint32_t lf_log2, const gpma_dev::LocModel *model,
                     uint32_t *max_err, hipStream_t s);

}  // namespace gpma_host
