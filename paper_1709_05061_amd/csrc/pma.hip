// PMA kernels of the GPMA+ update (Section 5.2, Algorithm "GPMA+ Segment-
// Oriented Insertion", and its dual for deletions) for gfx950.
//
// Layout (HBM): slots[cap] uint64 sorted keys with gaps (kEmpty); leaf j is
// slots[j*lf, (j+1)*lf) and always holds a packed prefix of cnt[j] >= 1
// occupied entries followed by gaps; row_ptr[V+1] uint32 CSR offsets (row u
// ends with its guard); deg[V] uint32 out-degrees.
//
// Lazy deletion (the GPMA/GPMA+ setup of Section 6): a delete marks its entry
// in place (bit 63) and counts it in dead[j] of its leaf; nothing moves.  A
// marked entry keeps ordering the array by its masked key, so the leaf
// pivots and the locate rule see it like a live one, but every density test
// counts live entries only (cnt - dead) and every merge drops the marked
// entries of the segments it rewrites (and clears their dead counts).  With
// lazy deletion off, dead is null and nothing below changes.
//
// Tiers of TryInsert+ (Section 5.2 and Appendix A, warp / block / device):
//   level 0   k_leaf_merge: a group of lf/SPL lanes of one wave per leaf, the
//             leaf staged through a per-group LDS slice (no workgroup barrier);
//   level h   k_seg_merge: one workgroup per segment, the segment staged in
//             LDS (up to what one workgroup may allocate);
//   above     host-driven device tier: gather -> merge -> dispatch kernels.
#include "common.h"
#include "pair.h"

using namespace gpma_dev;

namespace {

inline uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// batch validation: every key needs src < V and dst < V

__global__ void k_validate(const uint64_t *__restrict__ keys, uint64_t n, const uint32_t *__restrict__ n_dev,
                           uint32_t V, Ctl *__restrict__ ctl) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n_dev && *n_dev < n) n = *n_dev;
    bool bad = false;
    if (i < n) {
        uint64_t k = keys[i];
        bad = key_src(k) >= V || key_dst(k) >= V;
    }
    if (__ballot(bad) && __lane_id() == 0) atomicOr(&ctl->err, 1u);
}

__global__ void k_append_guards(uint64_t *__restrict__ dst, uint32_t V) {
    uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < V) dst[u] = (u << 32) | kGuardDst;
}

// ---------------------------------------------------------------------------
// BinarySearchLeafSegments: the leaf of key k is the leaf holding the
// greatest stored key <= k, leaf 0 when there is none.  No leaf is ever empty,
// so the first slot of every leaf is its smallest key and those pivots
// ascend strictly: a plain binary search over them (a marked entry orders by
// its masked key).  The pivots sit in their own dense array, piv[j] = the
// first slot of leaf j with the mark cleared, which every kernel that writes
// a leaf's first slot keeps; the search then touches one 8-byte word per step
// where the slots would cost a 256-byte leaf apart each (at 2^24 leaves the
// array is 128 MiB, and its last four steps share a cache line).

struct LocateOp {
    struct Args {
        const uint64_t *keys;
        const uint32_t *n_dev;
        uint64_t n_max;
        const uint64_t *piv;
        uint64_t L;
        const Ctl *ctl;
        uint32_t *leaf;
        uint8_t *status;
        WinSrc ws;
    };
    static __device__ __forceinline__ void run(const Args &args) {
        const uint64_t *__restrict__ keys = args.keys;
        const uint32_t *__restrict__ n_dev = args.n_dev;
        uint64_t n_max = args.n_max;
        const uint64_t *__restrict__ piv = args.piv;
        uint64_t L = args.L;
        const Ctl * ctl = args.ctl;
        uint32_t *__restrict__ leaf = args.leaf;
        uint8_t *__restrict__ status = args.status;
        WinSrc ws = args.ws;
        uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
        const BatchView bv = batch_view(ws, keys, n_dev, n_max, ctl);
        if (i >= bv.n || bv.err) return;
        uint64_t k = bv.keys[i] & bv.mask;
        if (ws.ukeys) ws.dense[i] = k;
        uint64_t lo = 0, hi = L;   // count of leaves whose pivot is <= k
        while (lo < hi) {
            uint64_t mid = (lo + hi) >> 1;
            if (piv[mid] <= k) lo = mid + 1; else hi = mid;
        }
        leaf[i] = (uint32_t)(lo ? lo - 1 : 0);
        status[i] = kPending;
    }
};

__global__ void __launch_bounds__(256)
k_locate(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ n_dev,
                         uint64_t n_max, const uint64_t *__restrict__ piv, uint64_t L,
                         const Ctl *ctl, uint32_t *__restrict__ leaf,
                         uint8_t *__restrict__ status, WinSrc ws) {
    LocateOp::run(LocateOp::Args{keys, n_dev, n_max, piv, L, ctl, leaf, status, ws});
}

// ---------------------------------------------------------------------------
// sub-wave group helpers (G lanes, G a power of two <= 64, group-aligned)

template <int G>
__device__ __forceinline__ uint32_t group_sum(uint32_t v) {
#pragma unroll
    for (int d = G / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, G);
    return v;
}

template <int G>
__device__ __forceinline__ uint32_t group_excl_scan(uint32_t v, uint32_t gl) {
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        uint32_t y = __shfl_up(x, d, G);
        if (gl >= (uint32_t)d) x += y;
    }
    return x - v;
}

// end of the run of equal leaf>>h values starting at i (exclusive), in [i+1, n]
__device__ __forceinline__ uint32_t run_end(const uint32_t *__restrict__ leaf, uint32_t i,
                                            uint32_t n, uint32_t s, uint32_t h) {
    uint32_t lo = i + 1, hi = n;
    // small runs are the common case: probe a few neighbours first
    if (lo < hi && (leaf[lo] >> h) != s) return lo;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if ((leaf[mid] >> h) == s) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Level 0: TryInsert+ / TryDelete+ on leaf segments, fused with the existence
// probe that turns present inserts and absent deletes into no-ops (the probe
// reads the same leaf, and at level 0 no other group writes that leaf).
// Group = G lanes, each holding SPL consecutive slots of the leaf (lf = G*SPL).

// What one group's run came to: updates merged, no-ops, merged leaves (0/1)
// and updates left pending for the level above.
struct RunStats {
    uint32_t done, noop, head, pend;
};

// A run of one update into a leaf holding no marked entries (at 2^16 updates
// over 2^24 leaves almost every run), done in registers: the update's rank
// comes from two ballots per slot column, and the entries from that rank on
// shift one place (insert: right, delete: left), each lane taking its
// neighbour's boundary entry by a shuffle.  Only the shifted slots are
// written; the rest of the leaf, the pivot (unless slot 0 moved) and the
// row offsets of guards that stay put are unchanged.  The outcome is the
// general run merge's for a run of one.
template <int G, int SPL, bool DEL>
__device__ __forceinline__ RunStats
leaf_single(uint64_t key, uint32_t i, uint32_t lf_i, uint32_t c, const uint64_t (&mine)[SPL], uint32_t gl,
            uint8_t *__restrict__ status, uint64_t *__restrict__ slots, uint64_t *__restrict__ piv,
            uint16_t *__restrict__ cnt, uint32_t *__restrict__ row_ptr, uint32_t *__restrict__ deg, uint32_t min0,
            uint32_t max0) {
    constexpr uint32_t LF = G * SPL;
    const uint32_t gbase = __lane_id() & ~(uint32_t)(G - 1);
    const uint64_t gmask = G == 64 ? ~0ull : ((1ull << G) - 1);
    uint32_t below = 0;   // entries < key
    bool present = false;
#pragma unroll
    for (int q = 0; q < SPL; q++) {
        const uint32_t x = gl * SPL + q;
        below += (uint32_t)__popcll((__ballot(x < c && mine[q] < key) >> gbase) & gmask);
        present |= ((__ballot(x < c && mine[q] == key) >> gbase) & gmask) != 0;
    }
    RunStats rs{0, 0, 0, 0};
    if (DEL ? !present : present) {
        if (gl == 0) status[i] = kNoop;
        rs.noop = 1;
        return rs;
    }
    if (DEL ? (c < 1 + min0) : (c + 1 > max0)) {   // the leaf fails its bound
        if (gl == 0) status[i] = kPending;
        rs.pend = 1;
        return rs;
    }
    const uint32_t N = DEL ? c - 1 : c + 1;
    const uint32_t end = DEL ? c : N;   // slots below .. end-1 change
    const uint64_t base = (uint64_t)lf_i * LF;
    const uint64_t prev = __shfl_up(mine[SPL - 1], 1, G);   // the entry before the lane's first
    const uint64_t next = __shfl_down(mine[0], 1, G);       // the entry after the lane's last
#pragma unroll
    for (int q = 0; q < SPL; q++) {
        const uint32_t x = gl * SPL + q;
        if (x < below || x >= end) continue;
        uint64_t v;
        if (DEL) v = x + 1 < c ? (q + 1 < SPL ? mine[q + 1] : next) : kEmpty;
        else v = x == below ? key : (q > 0 ? mine[q - 1] : prev);
        slots[base + x] = v;
        if (x == 0) piv[lf_i] = v & ~kTomb;
        if (x < N && is_guard(v)) row_ptr[key_src(v) + 1] = (uint32_t)(base + x + 1);
    }
    if (gl == 0) {
        cnt[lf_i] = (uint16_t)N;
        status[i] = (uint8_t)(kDone | kHead);
        atomicAdd(&deg[key_src(key)], DEL ? 0xFFFFFFFFu : 1u);
    }
    rs.done = 1;
    rs.head = 1;
    return rs;
}

template <int G, int SPL, bool DEL>
__device__ __forceinline__ RunStats
leaf_merge_group(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ leaf,
                 uint8_t *__restrict__ status, const uint32_t *__restrict__ n_dev, uint64_t n_max,
                 uint64_t *__restrict__ slots, uint64_t *__restrict__ piv, uint16_t *__restrict__ cnt,
                 uint32_t *__restrict__ row_ptr, uint32_t *__restrict__ deg, uint32_t *__restrict__ dead,
                 uint32_t min0, uint32_t max0, const Ctl *__restrict__ ctl, uint64_t *lb, uint64_t *ub,
                 uint64_t *ob) {
    constexpr int LF = G * SPL;
    constexpr int GPB = 256 / G;   // groups per block
    const uint32_t gib = threadIdx.x / G;          // group in block
    const uint32_t gl = threadIdx.x & (G - 1);     // lane in group
    const uint64_t gi = (uint64_t)blockIdx.x * GPB + gib;
    RunStats rs{0, 0, 0, 0};
    if (gi >= n_max) return rs;
    const uint32_t i = (uint32_t)gi;
    // One round trip for what a run's head needs first: the batch size and
    // error flag, the lane's first update of the run, and the leaf ids of the
    // update and both neighbours (a run of one, the common case, then needs
    // no search for its end).  The arrays hold n_max entries; those past the
    // batch size are stale and dropped once it is known.
    const uint32_t n = *n_dev;
    const uint32_t err = ctl->err;
    const uint64_t kpre = i + gl < n_max ? keys[i + gl] : 0;
    const uint32_t lf_i = leaf[i];
    const uint32_t lf_prev = i > 0 ? leaf[i - 1] : ~0u;   // leaf ids are < 2^32 - 1
    const uint32_t lf_nx = i + 1 < n_max ? leaf[i + 1] : ~0u;
    if (gi >= n || err) return rs;
    const uint32_t lf_next = i + 1 < n ? lf_nx : ~0u;
    if (lf_prev == lf_i) return rs;   // not the head of its run
    const uint32_t e = lf_next != lf_i ? i + 1 : run_end(leaf, i, n, lf_i, 0);
    const uint32_t k = e - i;
    const uint64_t base = (uint64_t)lf_i * LF;
    uint64_t mine[SPL];
#pragma unroll
    for (int q = 0; q < SPL; q++) mine[q] = slots[base + gl * SPL + q];
    // the leaf's entry count from its slots (a packed prefix, marked entries
    // included, then gaps): the same as cnt[lf_i] without a load of its own
    // cache line (a third of the merge's fetched bytes)
    uint32_t c = 0;
    {
        const uint32_t gbase = __lane_id() & ~(uint32_t)(G - 1);
        const uint64_t gmask = G == 64 ? ~0ull : ((1ull << G) - 1);
#pragma unroll
        for (int q = 0; q < SPL; q++) c += (uint32_t)__popcll((__ballot(mine[q] != kEmpty) >> gbase) & gmask);
    }
    const bool marked = dead && dead[lf_i];
    if (k == 1 && !marked)
        return leaf_single<G, SPL, DEL>(__shfl(kpre, 0, G), i, lf_i, c, mine, gl, status, slots, piv, cnt, row_ptr,
                                        deg, min0, max0);
    if (marked) {
        // the leaf holds marked entries: stage its live entries only, packed
        // in order (the merge below drops the marked ones)
        uint32_t nl = 0;
#pragma unroll
        for (int q = 0; q < SPL; q++) nl += (gl * SPL + q < c && is_live(mine[q])) ? 1u : 0u;
        uint32_t pos = group_excl_scan<G>(nl, gl);
        const uint32_t live = group_sum<G>(nl);
#pragma unroll
        for (int q = 0; q < SPL; q++)
            if (gl * SPL + q < c && is_live(mine[q])) lb[pos++] = mine[q];
        c = live;
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < SPL; q++) mine[q] = lb[gl * SPL + q];
    } else {
#pragma unroll
        for (int q = 0; q < SPL; q++) lb[gl * SPL + q] = mine[q];
    }
    wave_lds_sync();

    // classify the run: applicable updates are compacted (in key order) into ub
    uint32_t kapp = 0;
    bool app0 = false;   // the lane's first update is applicable
    for (uint32_t r0 = 0; r0 < k; r0 += G) {
        const uint32_t t = r0 + gl;
        const bool valid = t < k;
        const uint64_t key = valid ? (r0 == 0 ? kpre : keys[i + t]) : 0;
        // a key equal to the one before it (keys are sorted; a run head's
        // predecessor lies in another leaf) is a repeat, a no-op
        const uint64_t prev = r0 == 0 ? (uint64_t)__shfl_up((unsigned long long)kpre, 1, G)
                                      : (valid ? keys[i + t - 1] : 0);
        const bool rep = valid && t > 0 && prev == key;
        const bool present = valid && !rep && contains_u64(lb, c, key);
        const bool app = valid && !rep && (DEL ? present : !present);
        if (r0 == 0) app0 = app;
        const uint32_t pos = kapp + group_excl_scan<G>(app ? 1u : 0u, gl);
        if (app && pos < LF) ub[pos] = key;
        if (valid) status[i + t] = app ? kPending : kNoop;
        kapp += group_sum<G>(app ? 1u : 0u);
    }
    rs.noop = k - kapp;
    if (kapp == 0) return rs;
    const bool pass = DEL ? (c >= kapp + min0) : (c + kapp <= max0);
    if (!pass) {
        rs.pend = kapp;
        return rs;
    }
    rs.done = kapp;
    rs.head = 1;
    wave_lds_sync();

    // Merge + even re-dispatch: a leaf is one segment of one leaf, so the
    // merged run is simply packed at the front
    const uint32_t N = DEL ? c - kapp : c + kapp;
#pragma unroll
    for (int q = 0; q < SPL; q++) {
        const uint32_t x = gl * SPL + q;
        if (x < c) {
            const uint64_t a = mine[q];
            const uint32_t below = lower_bound_u64(ub, kapp, a);
            if (DEL) {
                if (!(below < kapp && ub[below] == a)) ob[x - below] = a;
            } else {
                ob[x + below] = a;
            }
        }
    }
    if (!DEL) {
        for (uint32_t t = gl; t < kapp; t += G) {
            const uint64_t uk = ub[t];
            ob[t + lower_bound_u64(lb, c, uk)] = uk;
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < SPL; q++) {
        const uint32_t p = gl * SPL + q;
        const uint64_t v = p < N ? ob[p] : kEmpty;
        slots[base + p] = v;
        if (p == 0) piv[lf_i] = v & ~kTomb;
        if (p < N && is_guard(v)) row_ptr[key_src(v) + 1] = (uint32_t)(base + p + 1);
    }
    if (gl == 0) {
        cnt[lf_i] = (uint16_t)N;
        if (dead) dead[lf_i] = 0;
    }
    // statuses of the run were written by the same lanes in the classify
    // loop; the lane's first update is still in registers
    for (uint32_t t = gl; t < k; t += G) {
        const bool first = t < (uint32_t)G;
        uint8_t st = first ? (app0 ? kPending : kNoop) : status[i + t];
        if (st == kPending) {
            st = kDone;
            atomicAdd(&deg[key_src(first ? kpre : keys[i + t])], DEL ? 0xFFFFFFFFu : 1u);
        }
        status[i + t] = t == 0 ? (uint8_t)(st | kHead) : st;
    }
    return rs;
}

// One group of G lanes per update; the head of each run of updates bound for
// one leaf merges the run.  part (optional): each block writes what its runs
// came to -- updates merged, no-ops, leaves merged, updates left pending --
// to part[4*block .. +3] (plain stores: per-block atomics on one control
// block serialise at the L2), for a finishing kernel to sum in place of a
// compaction's count.
struct LeafMergeArgs {
    const uint64_t *keys;
    const uint32_t *leaf;
    uint8_t *status;
    const uint32_t *n_dev;
    uint64_t n_max;
    uint64_t *slots;
    uint64_t *piv;
    uint16_t *cnt;
    uint32_t *row_ptr;
    uint32_t *deg;
    uint32_t *dead;
    uint32_t min0, max0;
    Ctl *ctl;
    uint32_t *part;
};

template <int G, int SPL, bool DEL>
struct LeafMergeOp {
    using Args = LeafMergeArgs;
    static __device__ __forceinline__ void run(const Args &args) {
        const uint64_t *__restrict__ keys = args.keys;
        const uint32_t *__restrict__ leaf = args.leaf;
        uint8_t *__restrict__ status = args.status;
        const uint32_t *__restrict__ n_dev = args.n_dev;
        const uint64_t n_max = args.n_max;
        uint64_t *__restrict__ slots = args.slots;
        uint64_t *__restrict__ piv = args.piv;
        uint16_t *__restrict__ cnt = args.cnt;
        uint32_t *__restrict__ row_ptr = args.row_ptr;
        uint32_t *__restrict__ deg = args.deg;
        uint32_t *__restrict__ dead = args.dead;
        const uint32_t min0 = args.min0, max0 = args.max0;
        Ctl *__restrict__ ctl = args.ctl;
        uint32_t *__restrict__ part = args.part;
        constexpr int LF = G * SPL;
        constexpr int GPB = 256 / G;   // groups per block
        __shared__ uint64_t s_leaf[GPB][LF];
        __shared__ uint64_t s_upd[GPB][LF];
        __shared__ uint64_t s_out[GPB][LF];
        __shared__ uint32_t s_red[4][256 / kWave];
        const uint32_t gib = threadIdx.x / G;
        RunStats rs = leaf_merge_group<G, SPL, DEL>(keys, leaf, status, n_dev, n_max, slots, piv, cnt, row_ptr, deg, dead,
                                                    min0, max0, ctl, s_leaf[gib], s_upd[gib], s_out[gib]);
        if (!part) return;   // grid-uniform
        // every lane of a group holds the group's figures: count lane 0's
        uint32_t v[4] = {rs.done, rs.noop, rs.head, rs.pend};
        const bool lead = (threadIdx.x & (G - 1)) == 0;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            v[q] = lead ? v[q] : 0u;
#pragma unroll
            for (int d = kWave / 2; d >= 1; d >>= 1) v[q] += __shfl_xor(v[q], d, kWave);
        }
        const uint32_t w = threadIdx.x / kWave;
        if (__lane_id() == 0)
#pragma unroll
            for (int q = 0; q < 4; q++) s_red[q][w] = v[q];
        __syncthreads();
        if (threadIdx.x < 4) {
            uint32_t t = 0;
            for (int x = 0; x < 256 / kWave; x++) t += s_red[threadIdx.x][x];
            part[4 * (uint64_t)blockIdx.x + threadIdx.x] = t;
        }
    }
};

template <int G, int SPL, bool DEL>
__global__ void __launch_bounds__(256)
k_leaf_merge(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ leaf,
             uint8_t *__restrict__ status, const uint32_t *__restrict__ n_dev, uint64_t n_max,
             uint64_t *__restrict__ slots, uint64_t *__restrict__ piv, uint16_t *__restrict__ cnt,
             uint32_t *__restrict__ row_ptr, uint32_t *__restrict__ deg, uint32_t *__restrict__ dead,
             uint32_t min0, uint32_t max0, Ctl *__restrict__ ctl, uint32_t *__restrict__ part) {
    LeafMergeOp<G, SPL, DEL>::run(LeafMergeArgs{keys, leaf, status, n_dev, n_max, slots, piv, cnt, row_ptr, deg,
                                                dead, min0, max0, ctl, part});
}

// ---------------------------------------------------------------------------
// Level h >= 1, workgroup tier: one workgroup per segment of P = 2^h leaves.
// CountSegment sums the leaf counts; a passing segment is staged (compacted)
// in LDS, merged with its updates by rank, and written back evenly.

constexpr int kSegThreads = 256;

__device__ __forceinline__ void block_scan_counts(uint32_t *v, uint32_t P, uint32_t *total,
                                                  uint32_t *lds_w) {
    // exclusive scan of v[0..P) in place; P <= a few thousand
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < P; b0 += blockDim.x) {
        uint32_t j = b0 + threadIdx.x;
        uint32_t x0 = j < P ? v[j] : 0;
        uint32_t x = x0;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            uint32_t y = __shfl_up(x, d, kWave);
            if (lane >= d) x += y;
        }
        if (lane == kWave - 1) lds_w[wid] = x;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t run = 0;
            for (int w = 0; w < nw; w++) {
                uint32_t t = lds_w[w];
                lds_w[w] = run;
                run += t;
            }
            lds_w[nw] = run;
        }
        __syncthreads();
        if (j < P) v[j] = carry + lds_w[wid] + x - x0;
        carry += lds_w[nw];
        __syncthreads();
    }
    *total = carry;
}

// One segment of the workgroup tier (head update i).  Block-uniform control
// flow: every early return is taken by the whole workgroup.
template <bool DEL>
__device__ __forceinline__ void seg_merge_one(uint32_t i, uint32_t n, uint32_t h,
                                              const uint64_t *__restrict__ keys,
                                              const uint32_t *__restrict__ leaf,
                                              uint8_t *__restrict__ status, uint64_t *__restrict__ slots,
                                              uint64_t *__restrict__ piv,
                                              uint16_t *__restrict__ cnt, uint32_t *__restrict__ row_ptr,
                                              uint32_t *__restrict__ deg, uint32_t *__restrict__ dead,
                                              uint32_t lf_log2, uint64_t minh, uint64_t maxh, uint64_t *dyn,
                                              uint32_t *s_misc) {
    const uint32_t s = leaf[i] >> h;
    if (i > 0 && (leaf[i - 1] >> h) == s) return;
    const uint32_t e = run_end(leaf, i, n, s, h);
    const uint32_t k = e - i;
    const uint32_t lf = 1u << lf_log2;
    const uint32_t P = 1u << h;
    const uint64_t cap_h = (uint64_t)P << lf_log2;
    const uint64_t first_leaf = (uint64_t)s << h;
    const uint64_t base = first_leaf << lf_log2;

    // LDS: E[cap_h] entries, U[cap_h] updates, off[P] leaf offsets
    uint64_t *E = dyn;
    uint64_t *U = dyn + cap_h;
    uint32_t *off = (uint32_t *)(dyn + 2 * cap_h);
    // CountSegment: live entries per leaf (marked ones are free space)
    for (uint32_t j = threadIdx.x; j < P; j += blockDim.x)
        off[j] = cnt[first_leaf + j] - (dead ? dead[first_leaf + j] : 0u);
    __syncthreads();
    uint32_t ns;
    block_scan_counts(off, P, &ns, s_misc);
    const bool pass = DEL ? ((uint64_t)ns >= (uint64_t)k + minh) : ((uint64_t)ns + k <= maxh);
    if (!pass) return;

    if (dead) {
        // marked entries may sit anywhere in a leaf's prefix: one wave per
        // leaf keeps the live ones, in order, by ballot
        const uint32_t lane = threadIdx.x & (kWave - 1);
        for (uint32_t j = threadIdx.x / kWave; j < P; j += blockDim.x / kWave) {
            const uint32_t cj = cnt[first_leaf + j];
            uint32_t at = off[j];
            for (uint32_t o0 = 0; o0 < cj; o0 += kWave) {
                const uint32_t o = o0 + lane;
                const uint64_t v = o < cj ? slots[base + ((uint64_t)j << lf_log2) + o] : kEmpty;
                const uint64_t m = __ballot(is_live(v));
                if (is_live(v)) E[at + __popcll(m & lanemask_lt())] = v;
                at += (uint32_t)__popcll(m);
            }
        }
    } else {
        for (uint64_t p = threadIdx.x; p < cap_h; p += blockDim.x) {
            uint32_t j = (uint32_t)(p >> lf_log2), o = (uint32_t)(p & (lf - 1));
            uint32_t cj = (j + 1 < P ? off[j + 1] : ns) - off[j];
            if (o < cj) E[off[j] + o] = slots[base + p];
        }
    }
    for (uint32_t t = threadIdx.x; t < k; t += blockDim.x) U[t] = keys[i + t];
    __syncthreads();

    const uint64_t N = DEL ? (uint64_t)ns - k : (uint64_t)ns + k;
    auto put = [&](uint64_t r, uint64_t v) {
        uint64_t j = rank_leaf(r, N, h);
        const uint64_t o = r - leaf_start(j, N, h);
        uint64_t pos = base + (j << lf_log2) + o;
        slots[pos] = v;
        if (o == 0) piv[first_leaf + j] = v & ~kTomb;
        if (is_guard(v)) row_ptr[key_src(v) + 1] = (uint32_t)(pos + 1);
    };
    for (uint32_t x = threadIdx.x; x < ns; x += blockDim.x) {
        const uint64_t a = E[x];
        const uint32_t below = lower_bound_u64(U, k, a);
        if (DEL) {
            if (!(below < k && U[below] == a)) put(x - below, a);
        } else {
            put((uint64_t)x + below, a);
        }
    }
    if (!DEL) {
        for (uint32_t t = threadIdx.x; t < k; t += blockDim.x) {
            const uint64_t uk = U[t];
            put((uint64_t)t + lower_bound_u64(E, ns, uk), uk);
        }
    }
    for (uint64_t p = threadIdx.x; p < cap_h; p += blockDim.x) {
        uint64_t j = p >> lf_log2, o = p & (lf - 1);
        uint64_t cj = leaf_start(j + 1, N, h) - leaf_start(j, N, h);
        if (o >= cj) slots[base + p] = kEmpty;
        if (o == 0) {
            if (cj == 0) piv[first_leaf + j] = kEmpty & ~kTomb;
            cnt[first_leaf + j] = (uint16_t)cj;
            if (dead) dead[first_leaf + j] = 0;
        }
    }
    for (uint32_t t = threadIdx.x; t < k; t += blockDim.x) {
        status[i + t] = t == 0 ? (uint8_t)(kDone | kHead) : (uint8_t)kDone;
        atomicAdd(&deg[key_src(U[t])], DEL ? 0xFFFFFFFFu : 1u);
    }
}

template <bool DEL>
__global__ void __launch_bounds__(kSegThreads)
k_seg_merge(uint32_t h, const uint64_t *__restrict__ keys, const uint32_t *__restrict__ leaf,
            uint8_t *__restrict__ status, const uint32_t *__restrict__ n_dev,
            uint64_t *__restrict__ slots, uint64_t *__restrict__ piv, uint16_t *__restrict__ cnt,
            uint32_t *__restrict__ row_ptr, uint32_t *__restrict__ deg, uint32_t *__restrict__ dead,
            uint32_t lf_log2, uint64_t minh, uint64_t maxh, Ctl *__restrict__ ctl) {
    extern __shared__ uint64_t dyn[];
    __shared__ uint32_t s_misc[kSegThreads / kWave + 4];
    const uint32_t n = *n_dev;
    if (ctl->err) return;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x)
        seg_merge_one<DEL>(i, n, h, keys, leaf, status, slots, piv, cnt, row_ptr, deg, dead, lf_log2, minh, maxh,
                           dyn, s_misc);
}

// ---------------------------------------------------------------------------
// device tier (large segments, root rebuild, bulk load)

// live entries per leaf
__global__ void k_leaf_counts_u32(const uint16_t *__restrict__ cnt, const uint32_t *__restrict__ dead,
                                  uint64_t first_leaf, uint64_t P, uint32_t *__restrict__ out) {
    uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < P) out[j] = cnt[first_leaf + j] - (dead ? dead[first_leaf + j] : 0u);
}

// compacted entries of the segment, in order: leaf j's prefix goes to
// out[leaf_off[j] - leaf_off[0] ..] (leaf_off: an exclusive scan of live
// counts that may start anywhere)
__global__ void k_gather_segment(const uint64_t *__restrict__ slots, const uint16_t *__restrict__ cnt,
                                 uint64_t first_leaf, uint64_t P, uint32_t lf_log2,
                                 const uint32_t *__restrict__ leaf_off, uint64_t *__restrict__ out) {
    uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (P << lf_log2)) return;
    uint64_t j = p >> lf_log2, o = p & ((1u << lf_log2) - 1);
    if (o < cnt[first_leaf + j]) out[leaf_off[j] - leaf_off[0] + o] = slots[(first_leaf << lf_log2) + p];
}

// The live entries of each segment of P = 2^h leaves that a run of pending
// updates falls in, written at the run's head: pre is the exclusive scan of
// all L live leaf counts, *total their sum.
__global__ void k_seg_live(const uint32_t *__restrict__ leaf, uint64_t rem, uint32_t h,
                           const uint32_t *__restrict__ pre, uint64_t L, const uint32_t *__restrict__ total,
                           uint32_t *__restrict__ ns_out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rem) return;
    const uint32_t seg = leaf[i] >> h;
    if (i > 0 && (leaf[i - 1] >> h) == seg) return;
    const uint64_t first = (uint64_t)seg << h;
    const uint64_t last = first + (1ull << h);
    ns_out[i] = (last < L ? pre[last] : *total) - pre[first];
}

// the same with marked entries dropped: one wave per leaf, live entries
// placed by ballot (leaf_off holds live-count offsets)
__global__ void __launch_bounds__(256)
k_gather_live(const uint64_t *__restrict__ slots, const uint16_t *__restrict__ cnt, uint64_t first_leaf,
              uint64_t P, uint32_t lf_log2, const uint32_t *__restrict__ leaf_off, uint64_t *__restrict__ out) {
    const uint64_t j = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (j >= P) return;   // wave-uniform
    const uint32_t lane = __lane_id();
    const uint32_t cj = cnt[first_leaf + j];
    const uint64_t base = (first_leaf + j) << lf_log2;
    uint64_t at = leaf_off[j] - leaf_off[0];
    for (uint32_t o0 = 0; o0 < cj; o0 += kWave) {
        const uint32_t o = o0 + lane;
        const uint64_t v = o < cj ? slots[base + o] : kEmpty;
        const uint64_t m = __ballot(is_live(v));
        if (is_live(v)) out[at + __popcll(m & lanemask_lt())] = v;
        at += (uint64_t)__popcll(m);
    }
}

// Merge(s, U_s) by rank: every element finds its output rank with one binary
// search in the other list (both sorted, disjoint for insert; U a subset of
// A for delete).
__global__ void k_merge_rank_a(bool del, const uint64_t *__restrict__ A, uint64_t na,
                               const uint64_t *__restrict__ U, uint64_t k, uint64_t *__restrict__ out) {
    uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= na) return;
    uint64_t a = A[x];
    uint64_t lo = 0, hi = k;
    while (lo < hi) {
        uint64_t mid = (lo + hi) >> 1;
        if (U[mid] < a) lo = mid + 1; else hi = mid;
    }
    if (del) {
        if (!(lo < k && U[lo] == a)) out[x - lo] = a;
    } else {
        out[x + lo] = a;
    }
}

__global__ void k_merge_rank_u(const uint64_t *__restrict__ A, uint64_t na,
                               const uint64_t *__restrict__ U, uint64_t k, uint64_t *__restrict__ out) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= k) return;
    uint64_t u = U[t];
    uint64_t lo = 0, hi = na;
    while (lo < hi) {
        uint64_t mid = (lo + hi) >> 1;
        if (A[mid] < u) lo = mid + 1; else hi = mid;
    }
    out[t + lo] = u;
}

// even re-dispatch of M[0..N) over leaves first_leaf .. first_leaf+P-1
__global__ void k_dispatch(const uint64_t *__restrict__ M, uint64_t N, uint64_t *__restrict__ slots,
                           uint64_t *__restrict__ piv, uint16_t *__restrict__ cnt, uint32_t *__restrict__ dead,
                           uint32_t *__restrict__ row_ptr, uint64_t first_leaf, uint64_t P, uint32_t lf_log2) {
    uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (P << lf_log2)) return;
    uint64_t j = p >> lf_log2, o = p & ((1u << lf_log2) - 1);
    const uint32_t h = 63 - __clzll(P);   // P is a power of two
    uint64_t st = leaf_start(j, N, h);
    uint64_t cj = leaf_start(j + 1, N, h) - st;
    uint64_t pos = (first_leaf << lf_log2) + p;
    uint64_t v = o < cj ? M[st + o] : kEmpty;
    slots[pos] = v;
    if (o == 0) {
        piv[first_leaf + j] = v & ~kTomb;
        cnt[first_leaf + j] = (uint16_t)cj;
        if (dead) dead[first_leaf + j] = 0;
    }
    if (o < cj && is_guard(v)) row_ptr[key_src(v) + 1] = (uint32_t)(pos + 1);
}

// Lazy deletion: mark each key of the batch in its leaf.  A key is deleted
// when its leaf holds it live; the mark keeps the entry's place and the
// leaf's dead count grows by one.  Absent and already marked keys, and
// repeats of a key (the batch is sorted; its first copy marks), are no-ops,
// so no two threads touch one slot.  part (optional): each block writes its
// marked and no-op counts to part[4*block], 0 and 0 after them (no leaf is
// rewritten and nothing is left pending), the leaf merge's figures for a
// finishing kernel to sum.
struct MarkOp {
    struct Args {
        const uint64_t *keys;
        const uint32_t *leaf;
        uint8_t *status;
        const uint32_t *n_dev;
        uint64_t n_max;
        uint64_t *slots;
        const uint16_t *cnt;
        uint32_t *dead;
        uint32_t *deg;
        uint32_t lf_log2;
        const Ctl *ctl;
        uint32_t *part;
    };
    static __device__ __forceinline__ void run(const Args &a) {
        const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
        bool marked = false, noop = false;
        if (i < a.n_max && i < *a.n_dev && !a.ctl->err) {
            const uint64_t k = a.keys[i];
            if (i > 0 && a.keys[i - 1] == k) {
                noop = true;
            } else {
                const uint32_t j = a.leaf[i];
                const uint64_t base = (uint64_t)j << a.lf_log2;
                const uint32_t c = a.cnt[j];
                uint32_t lo = 0, hi = c;   // occupied prefix: first masked key >= k
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if ((a.slots[base + mid] & ~kTomb) < k) lo = mid + 1; else hi = mid;
                }
                marked = lo < c && a.slots[base + lo] == k;   // a marked copy differs in bit 63
                noop = !marked;
                if (marked) {
                    a.slots[base + lo] = k | kTomb;
                    atomicAdd(&a.dead[j], 1u);
                    atomicAdd(&a.deg[key_src(k)], 0xFFFFFFFFu);
                }
            }
            a.status[i] = marked ? kDone : kNoop;
        }
        if (!a.part) return;   // grid-uniform
        __shared__ uint32_t s_red[2][1024 / kWave];
        const uint32_t w = threadIdx.x / kWave;
        const uint32_t nm = (uint32_t)__popcll(__ballot(marked));
        const uint32_t nn = (uint32_t)__popcll(__ballot(noop));
        if (__lane_id() == 0) {
            s_red[0][w] = nm;
            s_red[1][w] = nn;
        }
        __syncthreads();
        if (threadIdx.x < 4) {
            uint32_t t = 0;
            if (threadIdx.x < 2)
                for (uint32_t x = 0; x < blockDim.x / kWave; x++) t += s_red[threadIdx.x][x];
            a.part[4 * (uint64_t)blockIdx.x + threadIdx.x] = t;
        }
    }
};

__global__ void __launch_bounds__(256)
k_leaf_mark(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ leaf, uint8_t *__restrict__ status,
            const uint32_t *__restrict__ n_dev, uint64_t n_max, uint64_t *__restrict__ slots,
            const uint16_t *__restrict__ cnt, uint32_t *__restrict__ dead, uint32_t *__restrict__ deg,
            uint32_t lf_log2, const Ctl *__restrict__ ctl) {
    MarkOp::run(MarkOp::Args{keys, leaf, status, n_dev, n_max, slots, cnt, dead, deg, lf_log2, ctl, nullptr});
}

__global__ void k_mark_done(bool del, const uint64_t *__restrict__ keys, uint8_t *__restrict__ status,
                            uint64_t first, uint64_t count, uint32_t *__restrict__ deg,
                            Ctl *__restrict__ ctl, uint64_t cap_seg, int count_stats) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) {
        status[first + t] = t == 0 ? (uint8_t)(kDone | kHead) : (uint8_t)kDone;
        atomicAdd(&deg[key_src(keys[first + t])], del ? 0xFFFFFFFFu : 1u);
    }
    if (t == 0 && count_stats) {
        atomicAdd((unsigned long long *)&ctl->applied, (unsigned long long)count);
        atomicAdd((unsigned long long *)&ctl->dn, (unsigned long long)(del ? -(int64_t)count : (int64_t)count));
        atomicAdd((unsigned long long *)&ctl->rewritten, (unsigned long long)cap_seg);
        atomicAdd(&ctl->segs, 1u);
    }
}

// degrees at bulk load: guard positions in the sorted unique array
__global__ void k_guard_pos(const uint64_t *__restrict__ a, uint64_t n, uint32_t *__restrict__ gpos) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && is_guard(a[i])) gpos[key_src(a[i])] = (uint32_t)i;
}

__global__ void k_deg_from_gpos(const uint32_t *__restrict__ gpos, uint32_t V, uint32_t *__restrict__ deg) {
    uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= V) return;
    int64_t prev = u ? (int64_t)gpos[u - 1] : -1;
    deg[u] = (uint32_t)((int64_t)gpos[u] - prev - 1);
}

uint32_t log2_u32(uint32_t x) {
    uint32_t r = 0;
    while (x > 1) { x >>= 1; r++; }
    return r;
}

}  // namespace

namespace gpma_host {

void launch_validate(const uint64_t *keys, uint64_t n, uint32_t V, Ctl *ctl, hipStream_t s,
                     const uint32_t *n_dev) {
    if (!n) return;
    hipLaunchKernelGGL(k_validate, dim3((uint32_t)div_up(n, 256)), dim3(256), 0, s, keys, n, n_dev, V, ctl);
}

void launch_append_guards(uint64_t *dst, uint32_t V, hipStream_t s) {
    hipLaunchKernelGGL(k_append_guards, dim3((uint32_t)div_up(V, 256)), dim3(256), 0, s, dst, V);
}

void launch_locate(const uint64_t *keys, const uint32_t *n_dev, uint64_t n_max, const uint64_t *piv,
                   uint64_t L, const Ctl *ctl, uint32_t *leaf, uint8_t *status,
                   hipStream_t s, const WinSrc *ws) {
    if (!n_max) return;
    const WinSrc w = ws ? *ws : WinSrc{};
    hipLaunchKernelGGL(k_locate, dim3((uint32_t)div_up(n_max, 256)), dim3(256), 0, s, keys, n_dev,
                       n_max, piv, L, ctl, leaf, status, w);
}

template <int G, int SPL>
static void leaf_merge_t(bool del, const uint64_t *keys, const uint32_t *leaf, uint8_t *status,
                         const uint32_t *n_dev, uint64_t n_max, uint64_t *slots, uint64_t *piv, uint16_t *cnt,
                         uint32_t *row_ptr, uint32_t *deg, uint32_t *dead, uint32_t min0, uint32_t max0,
                         Ctl *ctl, uint32_t *part, hipStream_t s) {
    constexpr int GPB = 256 / G;
    dim3 grid((uint32_t)div_up(n_max, GPB));
    if (del)
        hipLaunchKernelGGL((k_leaf_merge<G, SPL, true>), grid, dim3(256), 0, s, keys, leaf, status,
                           n_dev, n_max, slots, piv, cnt, row_ptr, deg, dead, min0, max0, ctl, part);
    else
        hipLaunchKernelGGL((k_leaf_merge<G, SPL, false>), grid, dim3(256), 0, s, keys, leaf, status,
                           n_dev, n_max, slots, piv, cnt, row_ptr, deg, dead, min0, max0, ctl, part);
}

// groups of one leaf merge launch: G = lf / SPL lanes each, 256 / G per block
static uint32_t leaf_group_lanes(uint32_t lf) {
    switch (lf) {
        case 16: return 8;
        case 32: return 16;
        case 64: return 32;
        default: return 64;
    }
}

uint64_t leaf_merge_blocks(uint32_t lf, uint64_t n_max) { return div_up(n_max, 256 / leaf_group_lanes(lf)); }

void launch_leaf_merge(bool del, const uint64_t *keys, const uint32_t *leaf, uint8_t *status,
                       const uint32_t *n_dev, uint64_t n_max, uint64_t *slots, uint64_t *piv, uint16_t *cnt,
                       uint32_t *row_ptr, uint32_t *deg, uint32_t *dead, uint32_t lf, uint64_t min0,
                       uint64_t max0, Ctl *ctl, hipStream_t s, uint32_t *part) {
    if (!n_max) return;
    uint32_t mn = (uint32_t)min0, mx = (uint32_t)max0;
    switch (lf) {
        case 16: leaf_merge_t<8, 2>(del, keys, leaf, status, n_dev, n_max, slots, piv, cnt, row_ptr, deg, dead, mn, mx, ctl, part, s); break;
        case 32: leaf_merge_t<16, 2>(del, keys, leaf, status, n_dev, n_max, slots, piv, cnt, row_ptr, deg, dead, mn, mx, ctl, part, s); break;
        case 64: leaf_merge_t<32, 2>(del, keys, leaf, status, n_dev, n_max, slots, piv, cnt, row_ptr, deg, dead, mn, mx, ctl, part, s); break;
        case 128: leaf_merge_t<64, 2>(del, keys, leaf, status, n_dev, n_max, slots, piv, cnt, row_ptr, deg, dead, mn, mx, ctl, part, s); break;
        case 256: leaf_merge_t<64, 4>(del, keys, leaf, status, n_dev, n_max, slots, piv, cnt, row_ptr, deg, dead, mn, mx, ctl, part, s); break;
        default: leaf_merge_t<64, 8>(del, keys, leaf, status, n_dev, n_max, slots, piv, cnt, row_ptr, deg, dead, mn, mx, ctl, part, s); break;
    }
}

// ---- paired launches (the array at y = 0, its mirror at y = 1)

void launch_locate2(uint64_t n_max, const uint64_t *const piv[2], const uint64_t L[2],
                    const Ctl *const ctl[2], uint32_t *const leaf[2], uint8_t *const status[2], const WinSrc ws[2],
                    hipStream_t s) {
    if (!n_max) return;
    LocateOp::Args a[2];
    for (int k = 0; k < 2; k++)
        a[k] = {nullptr, nullptr, n_max, piv[k], L[k], ctl[k], leaf[k], status[k], ws[k]};
    launch_pair<LocateOp, 256>((uint32_t)div_up(n_max, 256), a[0], a[1], s);
}

template <int G, int SPL>
static void leaf_merge2_t(bool del, const LeafMergeArgs (&a)[2], hipStream_t s) {
    constexpr int GPB = 256 / G;
    const uint32_t gx = (uint32_t)div_up(a[0].n_max, GPB);
    if (del) launch_pair<LeafMergeOp<G, SPL, true>, 256>(gx, a[0], a[1], s);
    else launch_pair<LeafMergeOp<G, SPL, false>, 256>(gx, a[0], a[1], s);
}

void launch_leaf_merge2(bool del, const uint64_t *const keys[2], const uint32_t *const leaf[2],
                        uint8_t *const status[2], const uint32_t *const n_dev[2], uint64_t n_max,
                        uint64_t *const slots[2], uint64_t *const piv[2], uint16_t *const cnt[2],
                        uint32_t *const row_ptr[2], uint32_t *const deg[2], uint32_t *const dead[2], uint32_t lf,
                        const uint64_t min0[2], const uint64_t max0[2], Ctl *const ctl[2], uint32_t *const part[2],
                        hipStream_t s) {
    if (!n_max) return;
    LeafMergeArgs a[2];
    for (int k = 0; k < 2; k++)
        a[k] = {keys[k], leaf[k], status[k], n_dev[k], n_max, slots[k], piv[k], cnt[k], row_ptr[k], deg[k], dead[k],
                (uint32_t)min0[k], (uint32_t)max0[k], ctl[k], part[k]};
    switch (lf) {
        case 16: leaf_merge2_t<8, 2>(del, a, s); break;
        case 32: leaf_merge2_t<16, 2>(del, a, s); break;
        case 64: leaf_merge2_t<32, 2>(del, a, s); break;
        case 128: leaf_merge2_t<64, 2>(del, a, s); break;
        case 256: leaf_merge2_t<64, 4>(del, a, s); break;
        default: leaf_merge2_t<64, 8>(del, a, s); break;
    }
}

// LDS the workgroup tier may use: what the device grants a workgroup, once
// both merge kernels are allowed that much dynamic LDS (64 KiB otherwise)
int seg_merge_max_lds() {
    static int bytes = -1;
    if (bytes < 0) {
        int dev = 0, max_lds = 65536;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        bytes = 65536;
        if (max_lds > 65536 &&
            hipFuncSetAttribute((const void *)k_seg_merge<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                max_lds) == hipSuccess &&
            hipFuncSetAttribute((const void *)k_seg_merge<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                max_lds) == hipSuccess)
            bytes = max_lds;
        (void)hipGetLastError();
    }
    return bytes;
}

size_t seg_merge_lds_bytes(uint32_t lf, uint32_t h) {
    uint64_t cap_h = (uint64_t)lf << h;
    return 2 * cap_h * sizeof(uint64_t) + ((uint64_t)1 << h) * sizeof(uint32_t);
}

void launch_seg_merge(bool del, uint32_t h, const uint64_t *keys, const uint32_t *leaf,
                      uint8_t *status, const uint32_t *n_dev, uint64_t n_max, uint64_t *slots, uint64_t *piv,
                      uint16_t *cnt, uint32_t *row_ptr, uint32_t *deg, uint32_t *dead, uint32_t lf,
                      uint64_t minh, uint64_t maxh, Ctl *ctl, hipStream_t s) {
    if (!n_max) return;
    size_t lds = seg_merge_lds_bytes(lf, h);
    const uint32_t grid = (uint32_t)(n_max < 512 ? n_max : 512);   // grid-stride over segments
    if (del)
        hipLaunchKernelGGL(k_seg_merge<true>, dim3(grid), dim3(kSegThreads), lds, s, h,
                           keys, leaf, status, n_dev, slots, piv, cnt, row_ptr, deg, dead, log2_u32(lf), minh,
                           maxh, ctl);
    else
        hipLaunchKernelGGL(k_seg_merge<false>, dim3(grid), dim3(kSegThreads), lds, s, h,
                           keys, leaf, status, n_dev, slots, piv, cnt, row_ptr, deg, dead, log2_u32(lf), minh,
                           maxh, ctl);
}

void launch_leaf_counts_u32(const uint16_t *cnt, const uint32_t *dead, uint64_t first_leaf, uint64_t P,
                            uint32_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_leaf_counts_u32, dim3((uint32_t)div_up(P, 256)), dim3(256), 0, s, cnt, dead,
                       first_leaf, P, out);
}

void launch_gather_segment(const uint64_t *slots, const uint16_t *cnt, const uint32_t *dead,
                           uint64_t first_leaf, uint64_t P, uint32_t lf, const uint32_t *leaf_off,
                           uint64_t *out, hipStream_t s) {
    if (dead) {
        hipLaunchKernelGGL(k_gather_live, dim3((uint32_t)div_up(P, 256 / kWave)), dim3(256), 0, s, slots,
                           cnt, first_leaf, P, log2_u32(lf), leaf_off, out);
        return;
    }
    uint64_t total = P * lf;
    hipLaunchKernelGGL(k_gather_segment, dim3((uint32_t)div_up(total, 256)), dim3(256), 0, s, slots,
                       cnt, first_leaf, P, log2_u32(lf), leaf_off, out);
}

void launch_seg_live(const uint32_t *leaf, uint64_t rem, uint32_t h, const uint32_t *pre, uint64_t L,
                     const uint32_t *total, uint32_t *ns_out, hipStream_t s) {
    if (rem)
        hipLaunchKernelGGL(k_seg_live, dim3((uint32_t)div_up(rem, 256)), dim3(256), 0, s, leaf, rem, h, pre, L,
                           total, ns_out);
}

void launch_merge_sorted(bool del, const uint64_t *A, uint64_t na, const uint64_t *U, uint64_t k,
                         uint64_t *out, hipStream_t s) {
    if (na)
        hipLaunchKernelGGL(k_merge_rank_a, dim3((uint32_t)div_up(na, 256)), dim3(256), 0, s, del, A,
                           na, U, k, out);
    if (!del && k)
        hipLaunchKernelGGL(k_merge_rank_u, dim3((uint32_t)div_up(k, 256)), dim3(256), 0, s, A, na, U,
                           k, out);
}

void launch_dispatch(const uint64_t *M, uint64_t N, uint64_t *slots, uint64_t *piv, uint16_t *cnt, uint32_t *dead,
                     uint32_t *row_ptr, uint64_t first_leaf, uint64_t P, uint32_t lf, hipStream_t s) {
    uint64_t total = P * lf;
    hipLaunchKernelGGL(k_dispatch, dim3((uint32_t)div_up(total, 256)), dim3(256), 0, s, M, N, slots, piv,
                       cnt, dead, row_ptr, first_leaf, P, log2_u32(lf));
}

void launch_leaf_mark2(const uint64_t *const keys[2], const uint32_t *const leaf[2], uint8_t *const status[2],
                       const uint32_t *const n_dev[2], uint64_t n_max, uint64_t *const slots[2],
                       const uint16_t *const cnt[2], uint32_t *const dead[2], uint32_t *const deg[2], uint32_t lf,
                       const Ctl *const ctl[2], uint32_t *const part[2], hipStream_t s) {
    if (!n_max) return;
    MarkOp::Args a[2];
    for (int k = 0; k < 2; k++)
        a[k] = {keys[k], leaf[k], status[k], n_dev[k], n_max, slots[k], cnt[k], dead[k], deg[k], log2_u32(lf), ctl[k],
                part[k]};
    launch_pair<MarkOp, 256>((uint32_t)div_up(n_max, 256), a[0], a[1], s);
}

uint64_t leaf_mark_blocks(uint64_t n_max) { return div_up(n_max, 256); }

void launch_leaf_mark(const uint64_t *keys, const uint32_t *leaf, uint8_t *status, const uint32_t *n_dev,
                      uint64_t n_max, uint64_t *slots, const uint16_t *cnt, uint32_t *dead, uint32_t *deg,
                      uint32_t lf, const Ctl *ctl, hipStream_t s) {
    if (!n_max) return;
    hipLaunchKernelGGL(k_leaf_mark, dim3((uint32_t)div_up(n_max, 256)), dim3(256), 0, s, keys, leaf, status, n_dev,
                       n_max, slots, cnt, dead, deg, log2_u32(lf), ctl);
}

void launch_mark_done(bool del, const uint64_t *keys, uint8_t *status, uint64_t first, uint64_t count,
                      uint32_t *deg, Ctl *ctl, uint64_t cap_seg, bool count_stats, hipStream_t s) {
    hipLaunchKernelGGL(k_mark_done, dim3((uint32_t)div_up(count ? count : 1, 256)), dim3(256), 0, s,
                       del, keys, status, first, count, deg, ctl, cap_seg, count_stats ? 1 : 0);
}

void launch_degrees_from_sorted(const uint64_t *sorted, uint64_t n, uint32_t V, uint32_t *gpos,
                                uint32_t *deg, hipStream_t s) {
    hipLaunchKernelGGL(k_guard_pos, dim3((uint32_t)div_up(n, 256)), dim3(256), 0, s, sorted, n, gpos);
    hipLaunchKernelGGL(k_deg_from_gpos, dim3((uint32_t)div_up(V, 256)), dim3(256), 0, s, gpos, V, deg);
}

}  // namespace gpma_host
