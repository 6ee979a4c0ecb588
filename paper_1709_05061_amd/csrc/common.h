// Internal declarations shared by the HIP sources of the GPMA+ library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gpma.h"

namespace gpma_dev {

constexpr uint64_t kEmpty = 0xFFFFFFFFFFFFFFFFull;
constexpr uint32_t kGuardDst = 0xFFFFFFFFu;
constexpr int kWave = 64;

// status of one update inside a batch; kHead marks the first update of a
// segment that merged (the compaction pass counts merged segments with it)
enum : uint8_t { kPending = 0, kDone = 1, kNoop = 2, kStateMask = 0x7F, kHead = 0x80 };

// Device-side control block of one batch.  The host reads it back once per
// level (one small copy) to decide whether to climb further.
struct Ctl {
    uint32_t err;        // an invalid key was seen: the batch is a no-op
    uint32_t n_in;       // distinct updates of the batch
    uint32_t lvl[2];     // pending updates after alternate levels (compactions)
    uint32_t segs;       // segments merged so far in the batch
    uint64_t applied;    // updates merged so far in the batch
    uint64_t noops;      // updates dropped as no-ops
    int64_t dn;          // change of the stored entry count so far
    uint64_t rewritten;  // sum of capacities of merged segments
    uint32_t misses;     // learned-locator lookups that fell back to full search
    uint32_t root_full;  // lock-based comparator: insertions that found even the root full
};

// Where a locate kernel takes its batch from.  ukeys == nullptr: the keys
// passed to it, n from *n_dev, err from ctl->err.  Else the current batch of
// a fused window: batch j (pos when set, else *batch - *wstart) of the window's sorted
// keys ukeys[ustart[j] .. ustart[j+1]), tag bits cleared (none while *stop
// is set; err when errs[j] == *gen - 1); the kernel writes them to dense[]
// for the kernels after it, and its first thread resets the batch's control
// block (n_in, err, level counts, statistics; `misses` is reset by the
// kernels that read it).
struct WinSrc {
    const uint32_t *batch, *wstart, *gen, *stop;
    const uint64_t *ukeys;
    const uint32_t *ustart, *errs;
    uint64_t tag_mask;
    uint64_t *dense;
    Ctl *ctl;
    int32_t pos = -1;   // >= 0: the batch's place in its window, fixed when the launch was made
};

struct BatchView {
    const uint64_t *keys;
    uint64_t n;
    bool err;
    uint64_t mask;
};

__device__ __forceinline__ BatchView batch_view(const WinSrc &w, const uint64_t *keys, const uint32_t *n_dev,
                                                uint64_t n_max, const Ctl *ctl) {
    if (!w.ukeys) {
        const uint64_t n = *n_dev < n_max ? *n_dev : n_max;
        return BatchView{keys, n, ctl->err != 0, ~0ull};
    }
    const uint32_t j = w.pos >= 0 ? (uint32_t)w.pos : *w.batch - *w.wstart;
    const bool stopped = *w.stop != 0;
    const uint64_t beg = w.ustart[j];
    uint64_t n = stopped ? 0 : w.ustart[j + 1] - beg;
    if (n > n_max) n = n_max;
    const bool err = !stopped && w.errs[j] == *w.gen - 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Ctl *c = w.ctl;
        c->err = err ? 1u : 0u;
        c->n_in = (uint32_t)n;
        c->lvl[0] = 0;
        c->lvl[1] = 0;
        c->segs = 0;
        c->applied = 0;
        c->noops = 0;
        c->dn = 0;
        c->rewritten = 0;
    }
    return BatchView{w.ukeys + beg, n, err, w.tag_mask};
}

__device__ __forceinline__ bool is_guard(uint64_t k) {
    return (uint32_t)k == kGuardDst;
}

// Lazy deletion marks an entry in place by setting bit 63 (keys and guards
// have src < 2^31, so the bit is free).  Gaps (all ones) and marked entries
// are exactly the slots whose top bit is set.
constexpr uint64_t kTomb = 1ull << 63;
__device__ __forceinline__ bool is_live(uint64_t k) { return (int64_t)k >= 0; }
// a live edge: not a gap, not marked, not a guard
__device__ __forceinline__ bool is_edge_entry(uint64_t k) { return is_live(k) && !is_guard(k); }
// the key an occupied slot orders by (a marked entry keeps its place)
__device__ __forceinline__ uint64_t order_key(uint64_t k) { return k == kEmpty ? k : (k & ~kTomb); }
__device__ __forceinline__ uint32_t key_src(uint64_t k) { return (uint32_t)(k >> 32); }
__device__ __forceinline__ uint32_t key_dst(uint64_t k) { return (uint32_t)k; }

// number of a[0..n) that are < k (a sorted)
template <typename PtrT>
__device__ __forceinline__ uint32_t lower_bound_u64(PtrT a, uint32_t n, uint64_t k) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < k) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <typename PtrT>
__device__ __forceinline__ bool contains_u64(PtrT a, uint32_t n, uint64_t k) {
    uint32_t i = lower_bound_u64(a, n, k);
    return i < n && a[i] == k;
}

// Even re-dispatch of N ranked entries over P = 2^h leaves: leaf j holds
// ranks [floor(jN/P), floor((j+1)N/P)).  Rank r therefore sits in leaf
// ceil((r+1)P/N) - 1 at offset r - floor(leaf*N/P).  P is a power of two,
// so the leaf starts are shifts (j*N < 2^58: j < 2^27 leaves, N < 2^31).
__device__ __forceinline__ uint64_t leaf_start(uint64_t j, uint64_t N, uint32_t h) {
    return (j * N) >> h;
}
// The leaf of rank r: an fp64 quotient (relative error ~2^-52 on a value
// below 2^27, so off by at most one) corrected against the leaf starts.
__device__ __forceinline__ uint64_t rank_leaf(uint64_t r, uint64_t N, uint32_t h) {
    const uint64_t num = ((r + 1) << h) - 1;
    uint64_t j = (uint64_t)((double)num / (double)N);
    const uint64_t P = 1ull << h;
    if (j >= P) j = P - 1;
    while (j > 0 && leaf_start(j, N, h) > r) j--;
    while (j + 1 < P && leaf_start(j + 1, N, h) <= r) j++;
    return j;
}

// wave-level ordering of LDS traffic between lanes of one wave
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// exclusive scan of one value per thread over the workgroup (blockDim a
// multiple of the wave size); lds holds blockDim/64 + 1 words
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *total, uint32_t *lds) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    if (lane == kWave - 1) lds[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < nw; w++) {
            uint32_t t = lds[w];
            lds[w] = run;
            run += t;
        }
        lds[nw] = run;
    }
    __syncthreads();
    uint32_t excl = x - v + lds[wid];
    *total = lds[nw];
    __syncthreads();
    return excl;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    uint32_t lane = __lane_id();
    return lane ? ((~0ull) >> (64 - lane)) : 0ull;
}

}  // namespace gpma_dev

// ---------------------------------------------------------------------------
// launchers (host side), implemented in prims.hip / pma.hip / analytics.hip

namespace gpma_host {

struct Device {
    int max_lds = 65536;   // bytes of LDS one workgroup may allocate
    int cus = 256;
};

// ---- primitives (prims.hip)
// exclusive scan of n uint32 in place-safe (in may equal out); the total is
// written to *total_dev when non-null.  tmp needs scan_tmp_words(n) words.
size_t scan_tmp_words(uint64_t n);
void scan_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *total_dev,
              uint32_t *tmp, hipStream_t s);

// the same in one workgroup (one launch; for up to ~2^16 words)
void scan_u32_one_block(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *total_dev, hipStream_t s);

// keys-only LSD radix sort of n uint64 keys on the bits of the compressed
// key (src << dbits) | dst', where dst' = dst, or V for a guard.  Result in
// *out (one of buf_a/buf_b); `in` is not modified.  tmp: radix_tmp_words(n).
size_t radix_tmp_words(uint64_t n);
// n_dev (optional): the actual count, on the device (<= n, which sizes grids).
// check (optional): the first pass also validates the keys (src < V and
// dst < V) and sets check->err on a bad one.  small_chunks: 64-key chunks
// per wave in the tiles of inputs up to 2^20 keys (2, 4 or 8: tiles of 512,
// 1024 or 2048 keys); larger inputs use 4096-key tiles.
const uint64_t *radix_sort_keys(const uint64_t *in, uint64_t n, uint32_t sbits, uint32_t dbits,
                                uint32_t V, uint64_t *buf_a, uint64_t *buf_b, uint32_t *tmp,
                                hipStream_t s, const uint32_t *n_dev = nullptr, gpma_dev::Ctl *check = nullptr,
                                int small_chunks = 4);

// splitter sort (splitter_sort.hip): the order of radix_sort_keys for up to
// 2^20 keys in five launches; n from *n_dev when non-null (<= n_max).  The
// result is in the buffer radix_sort_keys would return for the same bit
// counts (buf_a for an odd number of 8-bit passes); the other buffer is
// overwritten.  tmp: splitter_tmp_words(n_max) words.  bump/clear
// (optional, for a caller's bookkeeping): the counting launch, once the
// input is in place, adds one to *bump and zeroes *clear.
bool splitter_sort_fits(uint64_t n_max);
size_t splitter_tmp_words(uint64_t n_max);
// For a caller that samples the splitters itself (the paired sort below): the
// bucket count, the sample size (a regular sample of that many keys, sorted,
// gives splitter j = sample[(j+1)*S/B], j < B-1) and where they go in tmp.
uint32_t splitter_buckets(uint64_t n_max);
uint32_t splitter_sample_size(uint64_t n_max);
uint64_t *splitter_spl(uint32_t *tmp);
const uint64_t *splitter_sort_keys(const uint64_t *in, uint64_t n_max, const uint32_t *n_dev, uint32_t sbits,
                                   uint32_t dbits, uint32_t V, uint64_t *buf_a, uint64_t *buf_b, uint32_t *tmp,
                                   hipStream_t s, uint32_t *bump = nullptr, uint32_t *clear = nullptr);
// two sorts of n_max-key inputs in one set of launches (the array's and its
// mirror's window), while the bucket counts need no separate scan; the
// caller has written each side's splitters (splitter_spl(tmp[k]), from a
// regular sample of splitter_sample_size keys); returns 0 when the results
// are in buf_a, 1 for buf_b
bool splitter_sort_pairable(uint64_t n_max);
int splitter_sort_keys2(const uint64_t *const in[2], uint64_t n_max, const uint32_t *const n_dev[2], uint32_t sbits,
                        uint32_t dbits, uint64_t *const buf_a[2], uint64_t *const buf_b[2], uint32_t *const tmp[2],
                        hipStream_t s, uint32_t *const bump[2] = nullptr, uint32_t *const clear[2] = nullptr);

// unique of a sorted array: out receives the distinct keys, *count_dev their
// number.  flags/tmp scratch: n+1 words / scan_tmp_words(n).
void unique_sorted(const uint64_t *in, uint64_t n, uint64_t *out, uint32_t *count_dev,
                   uint32_t *flags, uint32_t *tmp, hipStream_t s);
// same, reading n from a device counter (upper bound n_max on the host)
void unique_sorted_dyn(const uint64_t *in, const uint32_t *n_dev, uint64_t n_max, uint64_t *out,
                       uint32_t *count_dev, uint32_t *flags, uint32_t *tmp, hipStream_t s);


// keep (key, leaf) pairs whose status is pending; n from *n_dev (<= n_max);
// the number kept goes to *count_dev and the kept pairs get status pending.
// Also accumulates the level's statistics into ctl (one atomic per block):
// applied / dn (+-merged updates), noops, merged segments and their slots
// (cap_h each); no statistics when ctl is null.
void compact_pending(const uint64_t *keys, const uint32_t *leaf, const uint8_t *status,
                     const uint32_t *n_dev, uint64_t n_max, uint64_t *keys_out,
                     uint32_t *leaf_out, uint8_t *status_out, uint32_t *count_dev,
                     uint32_t *flags, uint32_t *tmp, bool del, uint64_t cap_h,
                     gpma_dev::Ctl *ctl, hipStream_t s);

// stored edges (not empty, not guard) of slots[0..cap) in order
void compact_edges(const uint64_t *slots, uint64_t cap, uint64_t *out, uint32_t *count_dev,
                   uint32_t *flags, uint32_t *tmp, hipStream_t s);

// ---- PMA kernels (pma.hip)
void launch_validate(const uint64_t *keys, uint64_t n, uint32_t V, gpma_dev::Ctl *ctl,
                     hipStream_t s, const uint32_t *n_dev = nullptr);
void launch_append_guards(uint64_t *dst, uint32_t V, hipStream_t s);
// (piv: each leaf's first slot with the mark bit cleared, L words; every
// kernel below that writes a leaf's first slot writes its pivot too)
void launch_locate(const uint64_t *keys, const uint32_t *n_dev, uint64_t n_max,
                   const uint64_t *piv, uint64_t L, const gpma_dev::Ctl *ctl,
                   uint32_t *leaf, uint8_t *status, hipStream_t s, const gpma_dev::WinSrc *ws = nullptr);
void launch_leaf_merge(bool del, const uint64_t *keys, const uint32_t *leaf, uint8_t *status,
                       const uint32_t *n_dev, uint64_t n_max, uint64_t *slots, uint64_t *piv, uint16_t *cnt,
                       uint32_t *row_ptr, uint32_t *deg, uint32_t *dead, uint32_t lf, uint64_t min0,
                       uint64_t max0, gpma_dev::Ctl *ctl, hipStream_t s, uint32_t *part = nullptr);
// blocks of one leaf merge launch over n_max updates (4 words of `part` each)
uint64_t leaf_merge_blocks(uint32_t lf, uint64_t n_max);
// binary-search locate and the leaf merge for the array (index 0) and its
// mirror (index 1) in one launch each; the locate takes each side's batch
// from its window (ws)
void launch_locate2(uint64_t n_max, const uint64_t *const piv[2], const uint64_t L[2],
                    const gpma_dev::Ctl *const ctl[2], uint32_t *const leaf[2], uint8_t *const status[2],
                    const gpma_dev::WinSrc ws[2], hipStream_t s);
void launch_leaf_merge2(bool del, const uint64_t *const keys[2], const uint32_t *const leaf[2],
                        uint8_t *const status[2], const uint32_t *const n_dev[2], uint64_t n_max,
                        uint64_t *const slots[2], uint64_t *const piv[2], uint16_t *const cnt[2],
                        uint32_t *const row_ptr[2], uint32_t *const deg[2], uint32_t *const dead[2], uint32_t lf,
                        const uint64_t min0[2], const uint64_t max0[2], gpma_dev::Ctl *const ctl[2],
                        uint32_t *const part[2], hipStream_t s);
// workgroup tier at height h >= 1; needs seg_merge_lds_bytes(lf, h) <= max LDS
size_t seg_merge_lds_bytes(uint32_t lf, uint32_t h);
int seg_merge_max_lds();
void launch_seg_merge(bool del, uint32_t h, const uint64_t *keys, const uint32_t *leaf,
                      uint8_t *status, const uint32_t *n_dev, uint64_t n_max, uint64_t *slots, uint64_t *piv,
                      uint16_t *cnt, uint32_t *row_ptr, uint32_t *deg, uint32_t *dead, uint32_t lf,
                      uint64_t minh, uint64_t maxh, gpma_dev::Ctl *ctl, hipStream_t s);
// device tier pieces (one segment at a time; also the root rebuild and bulk load)
// (dead: per-leaf marked counts of a lazy-deletion array, else null; the
// counts and the gather then cover live entries only)
// (leaf_off: exclusive scan of the segment's live leaf counts, or the part
// of one over more leaves that starts at the segment: offsets are taken
// relative to leaf_off[0])
void launch_gather_segment(const uint64_t *slots, const uint16_t *cnt, const uint32_t *dead,
                           uint64_t first_leaf, uint64_t P, uint32_t lf, const uint32_t *leaf_off,
                           uint64_t *out, hipStream_t s);
// live entries of the level-h segment of each run of pending updates, at the
// run's head in ns_out (pre: exclusive scan of all L live leaf counts, *total
// their sum)
void launch_seg_live(const uint32_t *leaf, uint64_t rem, uint32_t h, const uint32_t *pre, uint64_t L,
                     const uint32_t *total, uint32_t *ns_out, hipStream_t s);
void launch_merge_sorted(bool del, const uint64_t *A, uint64_t na, const uint64_t *U, uint64_t k,
                         uint64_t *out, hipStream_t s);
void launch_dispatch(const uint64_t *M, uint64_t N, uint64_t *slots, uint64_t *piv, uint16_t *cnt, uint32_t *dead,
                     uint32_t *row_ptr, uint64_t first_leaf, uint64_t P, uint32_t lf,
                     hipStream_t s);
void launch_leaf_counts_u32(const uint16_t *cnt, const uint32_t *dead, uint64_t first_leaf, uint64_t P,
                            uint32_t *out, hipStream_t s);
// lock-based GPMA comparator (gpma_lock.hip)
void launch_lock_probe(const uint64_t *keys, const uint32_t *leaf, uint8_t *status, const uint32_t *n_dev,
                       uint64_t n_max, const uint64_t *slots, const uint16_t *cnt, uint32_t lf_log2,
                       const gpma_dev::Ctl *ctl, hipStream_t s);
void launch_lock_try(uint32_t h, uint32_t H, const uint64_t *keys, uint32_t *leaf, uint8_t *status, uint64_t n,
                     uint64_t *slots, uint64_t *piv, uint16_t *cnt, uint32_t *dead, uint32_t *row_ptr, uint32_t *deg,
                     uint64_t *scratch, uint32_t *locks, uint32_t epoch, uint64_t L, uint32_t lf_log2, uint64_t maxh,
                     gpma_dev::Ctl *ctl, hipStream_t s);
// lazy deletion: mark the located keys in place (status kDone/kNoop); the
// paired form writes per-block figures to part (4 words a block,
// leaf_mark_blocks(n_max) blocks) for the finishing kernel
void launch_leaf_mark2(const uint64_t *const keys[2], const uint32_t *const leaf[2], uint8_t *const status[2],
                       const uint32_t *const n_dev[2], uint64_t n_max, uint64_t *const slots[2],
                       const uint16_t *const cnt[2], uint32_t *const dead[2], uint32_t *const deg[2], uint32_t lf,
                       const gpma_dev::Ctl *const ctl[2], uint32_t *const part[2], hipStream_t s);
uint64_t leaf_mark_blocks(uint64_t n_max);
void launch_leaf_mark(const uint64_t *keys, const uint32_t *leaf, uint8_t *status, const uint32_t *n_dev,
                      uint64_t n_max, uint64_t *slots, const uint16_t *cnt, uint32_t *dead, uint32_t *deg,
                      uint32_t lf, const gpma_dev::Ctl *ctl, hipStream_t s);
// count=true: also add to ctl (used by the root rebuild, after which no
// compaction pass runs)
void launch_mark_done(bool del, const uint64_t *keys, uint8_t *status, uint64_t first,
                      uint64_t count, uint32_t *deg, gpma_dev::Ctl *ctl, uint64_t cap_seg,
                      bool count_stats, hipStream_t s);
void launch_degrees_from_sorted(const uint64_t *sorted, uint64_t n, uint32_t V, uint32_t *gpos,
                                uint32_t *deg, hipStream_t s);

// ---- analytics (analytics.hip)
void launch_pr_prep(const float *x, const uint32_t *deg, uint32_t V, bool uniform,
                    double *contrib, double *y, double *dangling, hipStream_t s);
void launch_pr_push(const uint64_t *slots, const uint16_t *cnt, uint64_t cap, uint32_t lf_log2,
                    const double *contrib, double *y, hipStream_t s);
void launch_pr_pull(const uint64_t *slots, const uint16_t *cnt, uint64_t cap, uint32_t lf_log2,
                    const double *contrib, double *y, hipStream_t s);
void launch_transpose_keys(const uint64_t *in, uint64_t n, uint64_t *out, hipStream_t s);
void launch_pr_combine(const double *y, const double *dangling, uint32_t V, double damping,
                       float *out, hipStream_t s);

// ---- PageRank SpMV by destination bins (spmv_binned.hip)
struct PbLayout {
    uint32_t nb = 0;           // destination bins of 8192 vertices
    uint32_t nc = 0;           // coarse bins of 64 bins (0: bins are written directly)
    uint32_t W = 0;            // slot ranges (one workgroup each)
    uint64_t spw = 0;          // slots per range
    uint64_t max_pieces = 0;   // bound on accumulation pieces
    uint64_t count_words = 0;  // nb * W
    uint64_t coarse_words = 0; // nc * W
};
bool pb_supported(uint32_t V);
PbLayout pb_layout(uint32_t V, uint64_t cap, uint32_t lf_log2, uint64_t n_entries, bool coarse);
// per call: count matrix, its scan (offs, total edges), the piece table, the
// scanned coarse count matrix (coffs, when nc > 0), and each slot range's
// edges packed at keys[w*spw ..] (cap words), ne[w] of them (W words)
void launch_pb_structure(const uint64_t *slots, const PbLayout &L, uint64_t *keys, uint32_t *ne,
                         uint32_t *offs, uint32_t *total, uint32_t *scan_tmp, uint4 *pieces, uint32_t *npieces,
                         uint32_t *coffs, hipStream_t s);
// per iteration: y (zeroed beforehand) += A^T contrib; rec2 is used when nc > 0
void launch_pb_spmv(const uint64_t *keys, const uint32_t *ne, const PbLayout &L,
                    const uint32_t *offs, const uint32_t *total, const uint4 *pieces, const uint32_t *npieces,
                    const uint32_t *coffs, const double *contrib, uint64_t *rec, uint64_t *rec2, uint32_t V,
                    double *y, hipStream_t s);
// the bin pass alone (fine bins, nc == 0): records of contributions, or
// (src_records) of source vertices, written once per call
void launch_pb_bin(const uint64_t *keys, const uint32_t *ne, const PbLayout &L, const uint32_t *offs,
                   const uint32_t *total, const double *contrib, uint64_t *rec, bool src_records, hipStream_t s);
// per iteration over source records: y (zeroed beforehand) += A^T contrib
void launch_pb_gather(const PbLayout &L, const uint4 *pieces, const uint32_t *npieces, const double *contrib,
                      const uint64_t *rec, uint32_t V, double *y, hipStream_t s);
void launch_bfs_init(int32_t *dist, uint32_t V, uint32_t source, uint32_t *queue,
                     uint32_t *qcount, hipStream_t s);
void launch_bfs_row_len(const uint32_t *row_ptr, const uint32_t *front, uint32_t nfront, uint32_t *len,
                        hipStream_t s);
void launch_bfs_expand(const uint64_t *slots, const uint32_t *row_ptr, const uint32_t *front,
                       const uint32_t *offs, uint32_t nfront, const uint32_t *total, uint64_t max_total,
                       int32_t level, int32_t *dist, uint32_t *next, uint32_t *next_count,
                       hipStream_t s);
void launch_bfs_bottom_up(const uint64_t *mslots, const uint32_t *mrow, uint32_t V, int32_t level,
                          int32_t *dist, uint32_t *next, uint32_t *next_count, hipStream_t s);
void launch_cc_init(uint32_t *label, uint32_t V, hipStream_t s);
void launch_cc_hook(const uint64_t *slots, uint64_t cap, uint32_t *label, hipStream_t s);
void launch_cc_sample(const uint64_t *slots, const uint32_t *row_ptr, uint32_t V, uint32_t lf, uint32_t *label,
                      hipStream_t s);
void launch_cc_hook_skip(const uint64_t *slots, uint64_t cap, uint32_t *label, uint32_t c, hipStream_t s);
void launch_cc_pick(const uint32_t *label, uint64_t stride, uint32_t n, uint32_t *out, hipStream_t s);
void launch_cc_compress(uint32_t *label, uint32_t V, hipStream_t s);

}  // namespace gpma_host
