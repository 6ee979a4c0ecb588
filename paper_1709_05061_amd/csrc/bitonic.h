// Workgroup bitonic sort of up to 1024*R 64-bit keys held in registers
// (shared by the splitter sort and the window fetch, which samples the
// splitters itself).
#pragma once

#include "common.h"

namespace gpma_dev {

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, uint32_t m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, (int)m, kWave);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), (int)m, kWave);
    return ((uint64_t)hi << 32) | lo;
}

// Bitonic sort, ascending, of the first P keys (P a power of two, 64 <= P <=
// 1024*R) a 1024-thread workgroup holds: k[r] of thread t is the key at index
// r*1024 + t.  Partners closer than a wave trade through lane shuffles,
// partners in other waves through lds (1024*R words), partners 1024 or more
// apart sit in the same thread.  The sort is bound by vector ALU issue (some
// 20 instructions per key and stage), so waves wholly past P skip the
// arithmetic and only keep to the barriers.
template <int R>
__device__ void block_bitonic(uint64_t (&k)[R], uint64_t *lds, uint32_t P) {
    const uint32_t t = threadIdx.x;
    const bool live = (t & ~(uint32_t)(kWave - 1)) < P;   // wave-uniform
    for (uint32_t kk = 2; kk <= P; kk <<= 1) {
        for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
            if (j >= 1024) {
                const uint32_t rj = j >> 10;
#pragma unroll
                for (int r = 0; r < R; r++) {
                    if (r & rj) continue;
                    const uint32_t idx = (uint32_t)r * 1024u + t;
                    const bool asc = (idx & kk) == 0;
                    const uint64_t a = k[r], b = k[r | rj];
                    const bool sw = asc ? (a > b) : (a < b);
                    k[r] = sw ? b : a;
                    k[r | rj] = sw ? a : b;
                }
            } else if (j >= (uint32_t)kWave) {
                if (live)
#pragma unroll
                    for (int r = 0; r < R; r++) lds[(uint32_t)r * 1024u + t] = k[r];
                __syncthreads();
                if (live)
#pragma unroll
                    for (int r = 0; r < R; r++) {
                        const uint32_t idx = (uint32_t)r * 1024u + t;
                        const uint64_t o = lds[idx ^ j];
                        const bool want_min = ((idx & j) == 0) == ((idx & kk) == 0);
                        k[r] = want_min ? (o < k[r] ? o : k[r]) : (o > k[r] ? o : k[r]);
                    }
                __syncthreads();
            } else if (live) {
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const uint32_t idx = (uint32_t)r * 1024u + t;
                    const uint64_t o = shfl_xor_u64(k[r], j);
                    const bool want_min = ((idx & j) == 0) == ((idx & kk) == 0);
                    k[r] = want_min ? (o < k[r] ? o : k[r]) : (o > k[r] ? o : k[r]);
                }
            }
        }
    }
}


}  // namespace gpma_dev
