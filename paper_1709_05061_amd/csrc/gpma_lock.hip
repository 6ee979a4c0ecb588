// The lock-based GPMA of Section 4.1 (paragraph "Concurrent Insertions in
// GPMA", Algorithm "GPMA Concurrent Insertion"), kept as a comparator for
// GPMA+ (Section 6 compares the two).
//
// Each insertion is handled by its own worker (here a wavefront: the lanes
// share the segment work of one insertion) and climbs the segment tree from
// its leaf.  At every height the worker tries, once, to lock its segment; a
// worker that loses aborts and retries in the next round.  A winner checks
// whether its segment can take one more entry under that height's upper
// bound; if so it merges its key into the segment and re-dispatches the
// segment evenly, else it goes on to the parent at the next height.  The
// heights run one after the other (one launch each), which is the
// synchronisation that keeps a merge at height h from overlapping one at a
// lower height inside the same segment.  A round ends when every height has
// run; the host then compacts the aborted insertions, doubles the root if an
// insertion found even the root full, and starts the next round.
//
// Locks are epochs: a round has a number, and a worker owns node (h, s) when
// an atomicMax of the round number into the node's word returns an older
// number.  Nothing spins and nothing needs resetting between rounds.
//
// Scratch: a segment being merged is staged in a slot-sized scratch array at
// the segment's own offset (segments locked at one height are disjoint), read
// back after an agent-scope fence.
#include "common.h"

using namespace gpma_dev;

namespace {

inline uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

constexpr uint32_t kAborted = 0xFFFFFFFFu;   // leaf id of an insertion that lost a lock this round
constexpr int kLockThreads = 256;             // 4 insertions per workgroup

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// existence probe: an insertion of a live key is a no-op (set semantics)
__global__ void k_lock_probe(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ leaf,
                             uint8_t *__restrict__ status, const uint32_t *__restrict__ n_dev, uint64_t n_max,
                             const uint64_t *__restrict__ slots, const uint16_t *__restrict__ cnt,
                             uint32_t lf_log2, const Ctl *__restrict__ ctl) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_max || i >= *n_dev || ctl->err) return;
    const uint64_t k = keys[i];
    const uint32_t j = leaf[i];
    const uint64_t base = (uint64_t)j << lf_log2;
    uint32_t lo = 0, hi = cnt[j];
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((slots[base + mid] & ~kTomb) < k) lo = mid + 1; else hi = mid;
    }
    status[i] = (lo < cnt[j] && slots[base + lo] == k) ? kNoop : kPending;
}

// One height of one round: a wave per pending insertion.
__global__ void __launch_bounds__(kLockThreads)
k_lock_try(uint32_t h, uint32_t H, const uint64_t *__restrict__ keys, uint32_t *__restrict__ leaf,
           uint8_t *__restrict__ status, uint64_t n, uint64_t *__restrict__ slots, uint64_t *__restrict__ piv,
           uint16_t *__restrict__ cnt,
           uint32_t *__restrict__ dead, uint32_t *__restrict__ row_ptr, uint32_t *__restrict__ deg,
           uint64_t *__restrict__ scratch, uint32_t *__restrict__ locks, uint32_t epoch, uint64_t L,
           uint32_t lf_log2, uint64_t maxh, Ctl *__restrict__ ctl) {
    const uint64_t i = (uint64_t)blockIdx.x * (kLockThreads / kWave) + threadIdx.x / kWave;
    if (i >= n) return;   // wave-uniform
    const uint32_t lane = __lane_id();
    if ((status[i] & kStateMask) != kPending || leaf[i] == kAborted) return;
    const uint64_t k = keys[i];
    const uint64_t s = leaf[i] >> h;
    uint32_t old = 0;
    if (lane == 0) old = atomicMax(&locks[(L >> h) + s], epoch);
    old = __shfl(old, 0, kWave);
    if (old >= epoch) {   // another insertion holds this segment: retry next round
        if (lane == 0) leaf[i] = kAborted;
        return;
    }
    const uint64_t P = 1ull << h;
    const uint64_t first = s << h;
    const uint64_t lf = 1ull << lf_log2;
    const uint64_t base = first << lf_log2;
    // CountSegment (live entries)
    uint32_t ns = 0;
    for (uint64_t j = lane; j < P; j += kWave) ns += cnt[first + j] - (dead ? dead[first + j] : 0u);
    ns = wave_sum(ns);
    if ((uint64_t)ns + 1 > maxh) {   // too dense: the parent next, or a root doubling
        if (h == H && lane == 0) {
            leaf[i] = kAborted;
            atomicAdd(&ctl->root_full, 1u);
        }
        return;
    }
    // Merge: the segment's live entries in order with k in its place, staged
    const uint64_t cap_h = P << lf_log2;
    uint64_t at = 0, below = 0;
    for (uint64_t p0 = 0; p0 < cap_h; p0 += kWave) {   // 64 slots (one or more leaves) per step
        const uint64_t p = p0 + lane;
        uint64_t v = kEmpty;
        if (p < cap_h && (p & (lf - 1)) < cnt[first + (p >> lf_log2)]) v = slots[base + p];
        const bool live = is_live(v);
        const uint64_t m = __ballot(live);
        const uint64_t lt = __ballot(live && v < k);
        if (live) scratch[base + at + __popcll(m & lanemask_lt()) + (v > k ? 1 : 0)] = v;
        at += (uint64_t)__popcll(m);
        below += (uint64_t)__popcll(lt);
    }
    if (lane == 0) scratch[base + below] = k;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    // re-dispatch N entries evenly over the P leaves
    const uint64_t N = at + 1;
    for (uint64_t p = lane; p < cap_h; p += kWave) {
        const uint64_t j = p >> lf_log2, o = p & (lf - 1);
        const uint64_t st = leaf_start(j, N, h);
        const uint64_t cj = leaf_start(j + 1, N, h) - st;
        const uint64_t v = o < cj ? scratch[base + st + o] : kEmpty;
        slots[base + p] = v;
        if (o == 0) {
            piv[first + j] = v & ~kTomb;
            cnt[first + j] = (uint16_t)cj;
            if (dead) dead[first + j] = 0;
        }
        if (o < cj && is_guard(v)) row_ptr[key_src(v) + 1] = (uint32_t)(base + p + 1);
    }
    if (lane == 0) {
        atomicAdd(&deg[key_src(k)], 1u);
        status[i] = (uint8_t)(kDone | kHead);
    }
}

}  // namespace

namespace gpma_host {

void launch_lock_probe(const uint64_t *keys, const uint32_t *leaf, uint8_t *status, const uint32_t *n_dev,
                       uint64_t n_max, const uint64_t *slots, const uint16_t *cnt, uint32_t lf_log2, const Ctl *ctl,
                       hipStream_t s) {
    if (!n_max) return;
    hipLaunchKernelGGL(k_lock_probe, dim3((uint32_t)div_up(n_max, 256)), dim3(256), 0, s, keys, leaf, status, n_dev,
                       n_max, slots, cnt, lf_log2, ctl);
}

void launch_lock_try(uint32_t h, uint32_t H, const uint64_t *keys, uint32_t *leaf, uint8_t *status, uint64_t n,
                     uint64_t *slots, uint64_t *piv, uint16_t *cnt, uint32_t *dead, uint32_t *row_ptr, uint32_t *deg,
                     uint64_t *scratch, uint32_t *locks, uint32_t epoch, uint64_t L, uint32_t lf_log2, uint64_t maxh,
                     Ctl *ctl, hipStream_t s) {
    if (!n) return;
    hipLaunchKernelGGL(k_lock_try, dim3((uint32_t)div_up(n, kLockThreads / kWave)), dim3(kLockThreads), 0, s, h, H,
                       keys, leaf, status, n, slots, piv, cnt, dead, row_ptr, deg, scratch, locks, epoch, L, lf_log2, maxh,
                       ctl);
}

}  // namespace gpma_host
