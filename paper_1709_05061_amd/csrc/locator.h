// Learned segment locator: model parameters and launchers.
#pragma once

#include "common.h"

namespace gpma_dev {

// The leaf of key (u, v) lies among the leaves spanned by row u, from the
// leaf holding guard u-1 to the leaf holding guard u (the CSR offsets give
// both).  For rows spanning more than kMinSpan leaves a 2 -> 32 -> 1 MLP with
// a skip term predicts how far through that span the key sits:
//   t = y + w2 . relu(W1 [x y] + b1) + b2,  x = u/V, y = v/(V+1),
// leaf = first + floor(t * span).  The window is +-(e + e/4 + 2) leaves,
// e = the largest leaf error over row u's pivots when the model was fitted.
constexpr uint32_t kMinSpan = 8;

struct LocModel {
    float w1x[32], w1y[32], b1[32];   // layer 1 (fp32)
    uint16_t w2[32];                  // layer 2 weights (bf16 bit patterns)
    float b2;
    float inv_v, inv_v1;              // feature scales 1/V and 1/(V+1)
    uint32_t V;
    uint32_t L;                       // leaves the model was fitted for
    uint32_t eps;                     // max leaf error over long-row pivots (report)
    uint32_t valid;
};

}  // namespace gpma_dev

namespace gpma_host {

void launch_locate_learned(const uint64_t *keys, const uint32_t *n_dev, uint64_t n_max, const uint64_t *piv,
                           const uint32_t *row_ptr, const uint32_t *row_eps, uint64_t L, uint32_t lf_log2,
                           const gpma_dev::LocModel *model,
                           const gpma_dev::Ctl *ctl, uint32_t *leaf, uint8_t *status, uint32_t *misses,
                           hipStream_t s, const gpma_dev::WinSrc *ws = nullptr);
// the same for the array (index 0) and its mirror (index 1) in one launch,
// each taking its batch from its window (ws)
void launch_locate_learned2(uint64_t n_max, const uint64_t *const piv[2], const uint32_t *const row_ptr[2],
                            const uint32_t *const row_eps[2],
                            const uint64_t L[2], uint32_t lf_log2, const gpma_dev::LocModel *const model[2],
                            const gpma_dev::Ctl *const ctl[2], uint32_t *const leaf[2], uint8_t *const status[2],
                            uint32_t *const misses[2], const gpma_dev::WinSrc ws[2], hipStream_t s);
size_t loc_gram_words();
void launch_loc_gram(const uint64_t *piv, const uint32_t *row_ptr, uint64_t L, uint32_t lf_log2, uint64_t stride,
                     uint64_t S, const gpma_dev::LocModel *model, double *gram, hipStream_t s);
// *err: the largest leaf error over every long-row pivot; row_eps[u]: the
// largest over row u's (both start at 0)
void launch_loc_eval(const uint64_t *piv, const uint32_t *row_ptr, uint64_t L, uint32_t lf_log2,
                     const gpma_dev::LocModel *model, uint32_t *err, uint32_t *row_eps, hipStream_t s);

}  // namespace gpma_host
