/*
 * gpma.h -- C ABI of the MI355X (gfx950) GPMA+ dynamic-graph library.
 *
 * A directed graph lives on the GPU as a packed memory array (PMA): sorted
 * 64-bit edge keys src<<32 | dst with bounded gaps, leaf segments of
 * `leaf_size` slots and an implicit tree of segments over the leaves
 * (Sha, Li, He, Tan, "Accelerating Dynamic Graph Analytics on GPUs",
 * Section 4.1).  Each vertex u also owns a guard entry u<<32 | 0xFFFFFFFF
 * that closes its row, so CSR row offsets stay valid while entries move
 * (Section 4.2, "CSR as a case study").  Batches of insertions and deletions
 * are applied by the lock-free, level-by-level GPMA+ update (Section 5.2,
 * Algorithm "GPMA+ Segment-Oriented Insertion", and its dual for
 * deletions).  PageRank, BFS and connected components (Section 6.1,
 * "Applications") read the array in place.
 *
 * Conventions for every call:
 *   - Pointers named *_dev are device pointers (HBM of the current device);
 *     everything else is host memory.  The caller keeps ownership of every
 *     buffer it passes; the library keeps no pointer to it after the call
 *     returns, and reads/writes it only in work ordered on `stream`.
 *   - Calls are ordered on the caller's `stream`.  They return to the host
 *     once their work is enqueued, except where noted (each update batch
 *     synchronises with the host once per tree level it climbs; resizes,
 *     BFS levels and the CC component pick also read small counters back).
 *   - A handle must be used by one host thread at a time; handles are
 *     independent.  Return value 0 = GPMA_OK, negative = error.
 *   - Device memory comes from the allocator given to gpma_create (hipMalloc
 *     and hipFree when none is given).  The library hands a block back only
 *     after the device has finished the library's work on it.
 *   - Errors: GPMA_EINVAL changes nothing (an invalid key makes its whole
 *     batch a no-op).  GPMA_ENOMEM changes nothing either: an update call
 *     reserves everything it may need (batch scratch, the merge workspace of
 *     the upper levels and the root, and the arrays of a root resize when
 *     one is possible) on the array and its mirror before either changes.
 *     After GPMA_EDEVICE the handle's contents are undefined: destroy it.
 */
#ifndef GPMA_H
#define GPMA_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gpma gpma_t;

enum {
    GPMA_OK = 0,
    GPMA_EINVAL = -1,   /* bad argument or key; nothing was changed */
    GPMA_ENOMEM = -2,   /* device allocation failed (see the conventions above) */
    GPMA_EDEVICE = -3,  /* a HIP call failed */
};

/* empty slot (key 0 is the real edge (0,0), so a gap is all ones) */
#define GPMA_EMPTY 0xFFFFFFFFFFFFFFFFull
/* the column of a guard entry ("infinity", Section 4.2) */
#define GPMA_GUARD_DST 0xFFFFFFFFu

/* Density bounds of the segment tree (Section 4.1, figure "PMA insertion
 * example"): rho (lower) and tau (upper) at the leaves and at the root, in
 * per mille, interpolated linearly in the height in between.  An insertion
 * merges into a segment iff (n_s + |U_s|)/capacity < tau_h, a deletion iff
 * (n_s - |D_s|)/capacity > rho_h.
 * Requirements (else GPMA_EINVAL): leaf_size a power of two in [16, 512]
 * (0 picks one: the next power of two >= log2 of the capacity, at least 16,
 * Section 4.1 "leaf segments with O(log N) length"); 0 < rho_leaf <= rho_root
 * < tau_root <= tau_leaf < 1000; 2*rho_root <= tau_root; and
 * rho_leaf * leaf_size >= 1000 (no leaf can ever become empty).
 * Defaults are the figure's: tau .92/.80, rho .08/.40. */
typedef struct {
    uint32_t leaf_size;
    uint32_t tau_leaf_pm, tau_root_pm;
    uint32_t rho_leaf_pm, rho_root_pm;
    uint32_t flags;           /* GPMA_FLAG_* below; other bits must be 0 */
    uint32_t sort_tile_keys;  /* keys per workgroup tile of the batch radix sort
                                 for batches up to 2^20: 512, 1024 or 2048
                                 (0 = 1024); a tuning knob, results identical */
    uint32_t fused_levels;    /* gpma_apply_batches: tree levels above the
                                 leaves that a batch runs on the device before
                                 handing updates still pending to the
                                 host-driven path, 0..3 (default 1); a tuning
                                 knob, results identical */
    uint32_t lds_tier_bytes;  /* LDS bytes a workgroup of the segment tier may
                                 use (0 = all the device grants, 160 KiB on
                                 gfx950); a smaller cap hands smaller
                                 segments to the host-driven device tier,
                                 results identical */
    uint32_t spmv_form;       /* PageRank's SpMV, GPMA_SPMV_* below */
} gpma_params;

/* The SpMV of gpma_pagerank.  AUTO: BINNED_GATHER while V <= 2^26, else
 * pull over the mirror when there is one, else push.  BINNED and
 * BINNED_COARSE (the bins filled through 64 coarse bins first) write the
 * contributions into destination bins every iteration; BINNED_GATHER bins
 * the edges once per call (each record names its source) and every
 * iteration fetches the sources' contributions.  The binned forms need
 * V <= 2^26, PULL needs GPMA_FLAG_MIRROR (else gpma_create returns
 * GPMA_EINVAL).  The forms agree within the fp32 rounding of the result. */
enum {
    GPMA_SPMV_AUTO = 0,
    GPMA_SPMV_BINNED = 1,
    GPMA_SPMV_BINNED_COARSE = 2,
    GPMA_SPMV_PULL = 3,
    GPMA_SPMV_PUSH = 4,
    GPMA_SPMV_BINNED_GATHER = 5,
};

/* Device memory provider.  alloc returns `bytes` of device memory of the
 * current device for use on `stream` (the stream of the call that needs it),
 * or NULL when it cannot; free takes back a block with the size it was
 * allocated with.  ctx is passed through.  The torch binding passes the
 * caching allocator of PyTorch. */
typedef struct {
    void *(*alloc)(size_t bytes, hipStream_t stream, void *ctx);
    void (*free)(void *ptr, size_t bytes, hipStream_t stream, void *ctx);
    void *ctx;
} gpma_allocator;

/* Keep a second, dst-major PMA (keys dst<<32 | src, one guard per vertex)
 * updated by the same GPMA+ batches.  It holds every vertex's in-edges as a
 * contiguous row, so PageRank pulls (a segmented reduction, no per-edge
 * atomics) instead of pushing.  Costs a second update per batch and a second
 * array.  Not in the paper (its SpMV reads a CSR copy); a design addition. */
#define GPMA_FLAG_MIRROR 1u

/* Learned segment locator.  The row offsets bound the leaf of key (u, v) to
 * the leaves spanned by row u; in rows spanning more than 8 leaves a
 * 2 -> 32 -> 1 MLP over (u/V, v/(V+1)) with a skip term predicts how far
 * through that span the key sits (layer 2 on MFMA, bf16 weights, fp32
 * accumulation), and an exact search inside the measured error window
 * corrects it, checked against the window's bracketing pivots, with a binary
 * search over the span as fallback, so the leaf (and every later result) is
 * identical to the binary-search locate of Algorithm "GPMA+ Segment-Oriented
 * Insertion".  Refitted after every rebuild or resize of the array, and when
 * more than 1/16 of a call's lookups fall back.  A design addition. */
#define GPMA_FLAG_LEARNED_LOCATOR 2u

/* gpma_apply_batches enqueues each batch's kernels on the stream directly
 * instead of replaying a captured HIP graph per (size class, operation).
 * The device-side control is the same; which is faster depends on the
 * runtime's graph launch cost (the autotuner measures both). */
#define GPMA_FLAG_FUSED_DIRECT 4u

/* Lazy deletion, the way GPMA and GPMA+ handle deletions in the experiments
 * of Section 6: a delete marks its entry in place (bit 63 of the slot set)
 * and moves nothing, so a delete batch never climbs the tree and the array
 * never shrinks.  A marked entry still orders the array by its key with the
 * bit cleared (leaf pivots, the locate rule), counts as free space in every
 * density test, and is dropped by the next merge, rebuild or resize that
 * rewrites its leaf; re-inserting a marked key merges it like any absent
 * key.  Exported slots show the marks; exported keys, degrees, row offsets
 * and the analytics see live edges only; gpma_export_leaf_counts counts
 * occupied slots (live and marked).  Mirrors are marked alike.  Costs one
 * uint32 per leaf. */
#define GPMA_FLAG_LAZY_DELETE 8u

/* gpma_apply_batches with a mirror: run both pipelines on streams of the
 * handle, forked from and joined to the caller's stream, instead of keeping
 * the array's on the caller's stream (a test knob; results identical). */
#define GPMA_FLAG_FUSED_LIB_STREAMS 16u

/* gpma_apply_batches sorts the keys of a window of batches with the LSD
 * radix sort (two launches per 8-bit digit) instead of the splitter sort
 * (five launches, windows of up to 2^20 keys); a test knob, results
 * identical. */
#define GPMA_FLAG_WINDOW_RADIX 32u

/* Per-batch statistics; filled when a non-NULL pointer is passed. */
typedef struct {
    uint64_t requested;      /* keys passed in */
    uint64_t applied;        /* edges actually inserted / deleted */
    uint64_t noops;          /* repeats, present inserts, absent deletes */
    int32_t  top_level;      /* highest level with a merge, -1 if none */
    uint32_t resized;        /* 1 when the root was rebuilt at a new capacity */
    uint64_t segments_merged[40];  /* per level */
    uint64_t slots_rewritten;      /* sum of capacities of merged segments */
    uint64_t mirror_slots_rewritten;  /* the same over the mirror's merges */
} gpma_stats;

/* Fill *p with the defaults above. */
void gpma_default_params(gpma_params *p);

/* Build the PMA for `num_vertices` vertices (1 <= V <= 2^31) holding the set
 * of `n` keys at init_keys_dev (unsorted; repeats collapse) plus V guards:
 * the sliding window's initial graph of the problem statement (Section 3)
 * laid out as CSR on a PMA (Section 4.2, "CSR as a case study", one guard
 * per row).  Keys need src < V and dst < V.  The capacity is the smallest
 * leaf_size*2^k whose root upper bound admits every entry (at most 2^31
 * slots); entries are spread evenly over all leaves ("re-dispatch evenly",
 * Section 4.1).  `params` NULL = gpma_default_params; `alloc` NULL =
 * hipMalloc / hipFree (the allocator is copied, and used for the mirror and
 * for snapshots too).  Synchronises with the host once.  *out receives the
 * handle (NULL on error).  GPMA_EINVAL: bad parameters, V out of range, an
 * invalid key, more than 2^31 slots needed; GPMA_ENOMEM; GPMA_EDEVICE. */
int gpma_create(gpma_t **out, uint32_t num_vertices, const uint64_t *init_keys_dev,
                uint64_t n, const gpma_params *params, const gpma_allocator *alloc, hipStream_t stream);

/* Free every device buffer of the handle (after `stream`-ordered work on it
 * has finished: the call synchronises the device). */
int gpma_destroy(gpma_t *h);

/* Set union with the b keys at keys_dev (Algorithm "GPMA+ Segment-Oriented
 * Insertion"): sort, locate each key's leaf, then merge level by level; the
 * root doubles when it cannot absorb what is left.  Keys already present and
 * repeats are no-ops.  Any key with src >= V or dst >= V makes the whole
 * batch a no-op and returns GPMA_EINVAL. */
int gpma_insert_batch(gpma_t *h, const uint64_t *keys_dev, uint64_t b,
                      hipStream_t stream, gpma_stats *stats);

/* Set difference (the dual of insertion, Section 4.1): a segment absorbs
 * its deletions iff it stays above its lower bound; the root halves when it
 * falls below its own.  Absent keys are no-ops; guards cannot be named
 * (dst must be < V).  With GPMA_FLAG_LAZY_DELETE each present key is marked
 * in its leaf instead (no merge, no resize). */
int gpma_delete_batch(gpma_t *h, const uint64_t *keys_dev, uint64_t b,
                      hipStream_t stream, gpma_stats *stats);

/* Fused batching: apply `count` batches in order (ops[i] = 0 insert, 1
 * delete; keys_dev[i] device pointers with sizes[i] keys; the three arrays
 * are host arrays).  The result is the one of the same sequence of
 * gpma_insert_batch / gpma_delete_batch calls, slot for slot.  Batches run
 * in windows of up to 64 whose keys are sorted together; each batch then
 * runs with device-side control up to the highest level the workgroup tier
 * covers (fused_levels).  The host synchronises once per window, plus once
 * for each batch that climbs above those levels (its remaining levels and
 * the root are then completed on the host-driven path).  Not in the paper;
 * the answer to its observation that GPMA+ pays for many kernel calls on
 * small batches.  On an invalid key in batch i, batches before i stay
 * applied, batch i and later are not, and GPMA_EINVAL is returned;
 * *completed (if non-NULL) receives the number of batches applied.  Memory
 * for the whole sequence (its insertions and deletions summed) is reserved
 * before the first batch runs: GPMA_ENOMEM applies nothing.  `total` (if
 * non-NULL) receives summed statistics (per-level counts are not filled).
 * With a mirror, while the array and the mirror stand at the same batch and
 * take the same kernels (no level above the leaves on the device), every
 * step of a window runs for both in one launch and the whole window is one
 * captured HIP graph on `stream`.  Otherwise each window's sort and each
 * batch replay graphs captured once per shape (or are enqueued directly,
 * GPMA_FLAG_FUSED_DIRECT), and the mirror's batches run on a stream of the
 * handle, forked from and joined to `stream` by events; the first such call
 * on a given `stream` synchronises it once more to pick that stream (a
 * ~0.4 ms probe: the handle's stream must run beside `stream`, not behind
 * it on one hardware queue). */
int gpma_apply_batches(gpma_t *h, uint32_t count, const uint8_t *ops, const uint64_t *const *keys_dev,
                       const uint64_t *sizes, hipStream_t stream, gpma_stats *total,
                       uint32_t *completed);
/* Which arrangement gpma_apply_batches uses with a mirror on caller stream
 * `stream`: 1 = the array's pipeline on `stream` and the mirror's on a
 * handle stream that runs beside it, 0 = both on handle streams (forked and
 * joined), GPMA_EINVAL = no mirror or no fused call on `stream` yet. */
int gpma_fused_pairing(gpma_t *h, hipStream_t stream);

/* PageRank by power iteration (Section 6.1): exactly `iters` steps of
 *   x'[v] = (1-d)/V + d * ( sum_{u->v} x[u]/outdeg(u) + D/V ),
 * D = sum of x over vertices without out-edges (self-loops count).
 * init_dev: V floats, or NULL for the uniform 1/V; out_dev: V floats, may
 * alias init_dev (warm start from the previous result).  Contributions
 * x[u]/outdeg(u) are formed in fp64 and summed in fp64 (the destination-bin
 * form, used while V <= 2^26, carries them with 38 mantissa bits); each step
 * rounds once to fp32.  The summation order is not fixed, so repeated calls
 * may differ in the last fp32 bit.
 * GPMA_EINVAL if iters == 0 or damping is not in (0,1). */
int gpma_pagerank(gpma_t *h, const float *init_dev, float *out_dev, uint32_t iters,
                  float damping, hipStream_t stream);

/* BFS hop distances from `source` along out-edges (Section 4.2, Algorithm
 * "Breadth-First Search"; rows are read through the CSR offsets and gaps
 * and guards are skipped).  dist_dev: V int32, -1 = unreachable.
 * GPMA_EINVAL if source >= V. */
int gpma_bfs(gpma_t *h, uint32_t source, int32_t *dist_dev, hipStream_t stream);

/* gpma_bfs for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same result as gpma_bfs, bit for bit, but the frontier queues, the
 * row-length scan and the level counters live in a fixed device array of
 * the library (about 48 MiB, one per GPU, held until the process ends)
 * instead of the handle's lazily allocated scratch, so the call allocates
 * nothing.  Limit: V <= 2^22 (else GPMA_EINVAL, nothing written).  Every
 * call on one GPU shares that array: calls that overlap on one GPU (from
 * several threads, or on several streams before the earlier ones finish)
 * race and must not be made; each call synchronises `stream` once per BFS
 * level, so consecutive calls from one thread do not overlap.
 * GPMA_EINVAL if source >= V; GPMA_EDEVICE if the array's address cannot be
 * had. */
int gpma_bfs_noalloc(gpma_t *h, uint32_t source, int32_t *dist_dev, hipStream_t stream);

/* Connected components with edge direction ignored (Section 6.1); every
 * vertex gets the smallest vertex id of its component.  label_dev: V uint32. */
int gpma_cc(gpma_t *h, uint32_t *label_dev, hipStream_t stream);

/* Snapshots for concurrent analytics (the streaming service): a read-only
 * handle holding device copies of the arrays the analytics read (slots, leaf
 * counts, row offsets, degrees, and the mirror's), taken in `stream` order,
 * i.e. of the graph as left by the work enqueued on `stream` before it.
 * gpma_pagerank / gpma_bfs / gpma_cc / exports work on it (one host thread and
 * one stream per snapshot at a time); updates return GPMA_EINVAL.  Free with
 * gpma_destroy.  gpma_snapshot_refresh copies a newer state into an existing
 * snapshot (reallocating only if the capacity changed).  Not in the paper: it
 * lets queries on version v overlap the updates that make version v+1. */
int gpma_snapshot(gpma_t *h, gpma_t **snap_out, hipStream_t stream);
int gpma_snapshot_refresh(gpma_t *h, gpma_t *snap, hipStream_t stream);
/* Device bytes of the arrays a snapshot copies (the budget unit of a query). */
uint64_t gpma_device_bytes(const gpma_t *h);

/* The leaf of each of n keys (BinarySearchLeafSegments: the leaf holding the
 * greatest stored key <= k, leaf 0 if none), through the learned locator when
 * the handle has one.  Keys need src < V, dst < V (else GPMA_EINVAL).
 * leaf_out_dev: n uint32.  Synchronises. */
int gpma_locate(gpma_t *h, const uint64_t *keys_dev, uint64_t n, uint32_t *leaf_out_dev,
                hipStream_t stream);
/* Refit the learned locator now (GPMA_EINVAL without one). */
int gpma_locator_refit(gpma_t *h, hipStream_t stream);
/* Learned-locator state: current error window (leaves; all ones when the
 * model is unusable), lookups and fallbacks so far, number of fits. */
int gpma_locator_info(const gpma_t *h, uint32_t *eps, uint64_t *lookups, uint64_t *misses,
                      uint64_t *fits);

/* The mirror of a handle created with GPMA_FLAG_MIRROR, else NULL.  A
 * borrowed handle for the read-only calls below (export, introspection); it
 * must not be updated or destroyed directly. */
gpma_t *gpma_get_mirror(gpma_t *h);

/* Comparator: the lock-based GPMA insertion of Section 4.1 (paragraph
 * "Concurrent Insertions in GPMA", Algorithm "GPMA Concurrent Insertion"),
 * which Section 6 measures against GPMA+.  Same set semantics and the same
 * density bounds as gpma_insert_batch, but each insertion climbs the tree on
 * its own: per round, at each height in turn, it tries once to lock its
 * segment (a loser retries next round), and a winner that fits merges its one
 * key and re-dispatches the segment; a root that cannot take an insertion is
 * doubled between rounds.  The resulting slot layout depends on which
 * insertions win their locks, so only the edge set (and the PMA invariants)
 * match gpma_insert_batch.  Not for handles with a mirror (GPMA_EINVAL).
 * Allocates, on first use, a scratch array as large as the slot array and
 * 8 bytes of lock words per leaf.  *rounds_out (if not NULL) receives the
 * number of rounds.  Synchronises with the host once per round. */
int gpma_lock_insert_batch(gpma_t *h, const uint64_t *keys_dev, uint64_t b, hipStream_t stream,
                           gpma_stats *stats, uint32_t *rounds_out);

/* Device bytes the handle (with its mirror) holds from its allocator. */
uint64_t gpma_allocated_bytes(const gpma_t *h);

/* Take now, on the array and its mirror, the memory that update batches of
 * up to b keys need short of a root resize (batch scratch, fused-batching
 * state, the merge workspace of the upper levels and the root), so that
 * later calls allocate only to resize.  For callers that budget device
 * memory (the streaming service admits work against an HBM budget).
 * GPMA_ENOMEM if the allocator refuses (what was taken stays taken). */
int gpma_reserve(gpma_t *h, uint64_t b, hipStream_t stream);

/* Introspection.  Counts are those after the last completed call. */
uint64_t gpma_num_edges(const gpma_t *h);     /* guards excluded */
uint64_t gpma_capacity(const gpma_t *h);      /* slots */
uint32_t gpma_leaf_size(const gpma_t *h);
uint32_t gpma_num_vertices(const gpma_t *h);

/* Copy the raw slot array (capacity uint64, gaps = GPMA_EMPTY, guards
 * included) to out_dev.  GPMA_EINVAL if max < capacity. *cap_out = capacity. */
int gpma_export_slots(gpma_t *h, uint64_t *out_dev, uint64_t max, uint64_t *cap_out,
                      hipStream_t stream);
/* Copy the stored edges in key order (guards dropped).  GPMA_EINVAL if
 * max < number of edges.  Synchronises; *n_out = number of edges. */
int gpma_export_keys(gpma_t *h, uint64_t *out_dev, uint64_t max, uint64_t *n_out,
                     hipStream_t stream);
/* Per-leaf entry counts (capacity/leaf_size uint16). */
int gpma_export_leaf_counts(gpma_t *h, uint16_t *out_dev, uint64_t max, hipStream_t stream);
/* Per-leaf pivots (capacity/leaf_size uint64): the first slot of each leaf
 * with the deletion mark cleared, the array BinarySearchLeafSegments searches
 * (Section 5.1, Algorithm "GPMA+ Segment-Oriented Insertion").  Every update
 * keeps it equal to that definition.  GPMA_EINVAL if max is too small or h is
 * a snapshot (which keeps no pivots). */
int gpma_export_pivots(gpma_t *h, uint64_t *out_dev, uint64_t max, hipStream_t stream);
/* CSR row offsets on the PMA (V+1 uint32): row u spans slots
 * [off[u], off[u+1]) and ends with its guard; off[0] = 0. */
int gpma_export_row_offsets(gpma_t *h, uint32_t *out_dev, uint64_t max, hipStream_t stream);
/* Out-degrees (V uint32), guards excluded. */
int gpma_export_degrees(gpma_t *h, uint32_t *out_dev, uint64_t max, hipStream_t stream);

/* Wait for all work of the handle.  Returns 0. */
int gpma_sync(gpma_t *h);

/* ---- Comparator: CSR rebuilt on every batch ------------------------------
 * A plain CSR (edges sorted, no gaps, 64-bit row offsets) whose updates
 * rebuild the whole format, the role the GPU CSR of cuSparse plays among the
 * paper's baselines (Section 6, "GPU-based CSR": updates by rebuilding).
 * Same set semantics and key rules as the PMA; present for comparison, not
 * used by the PMA. */
typedef struct gpma_csr gpma_csr_t;
/* Build from n keys (device; duplicates allowed).  GPMA_EINVAL as for
 * gpma_create; *out = NULL on error. */
int gpma_csr_create(gpma_csr_t **out, uint32_t num_vertices, const uint64_t *init_keys_dev, uint64_t n,
                    hipStream_t stream);
void gpma_csr_destroy(gpma_csr_t *h);
/* Apply one batch (del = 0 insert, 1 delete): sort, drop no-ops, merge into
 * or remove from the whole edge array, recompute the row offsets.
 * Synchronises with the host twice.  GPMA_EINVAL on an invalid key (nothing
 * changed). */
int gpma_csr_update(gpma_csr_t *h, const uint64_t *keys_dev, uint64_t b, int del, hipStream_t stream);
uint64_t gpma_csr_num_edges(const gpma_csr_t *h);
/* Sorted edges (keys_out, at least num_edges) and/or row offsets (V + 1
 * uint64); either may be NULL. */
int gpma_csr_export(const gpma_csr_t *h, uint64_t *keys_out_dev, uint64_t max_keys, uint64_t *row_ptr_out_dev,
                    hipStream_t stream);

/* Static message for an error code. */
const char *gpma_strerror(int code);

/* Kernel timing for roofline accounting.  When enabled, the library brackets
 * every launch of the kernels below with HIP events on the launch stream and
 * accumulates elapsed time, launch count and algorithmic bytes (what the
 * method must move; see the per-kernel notes in the implementation).
 * gpma_profile_read synchronises the events it reads; with a mirror, the
 * mirror's launches are included. */
enum {
    GPMA_K_SPMV = 0,      /* one PageRank SpMV (all its kernels) */
    GPMA_K_LEAF_MERGE,    /* level-0 fused probe/check/merge */
    GPMA_K_SEG_MERGE,     /* levels >= 1, workgroup tier */
    GPMA_K_SORT,          /* whole batch radix sort (all passes) */
    GPMA_K_LOCATE,        /* leaf search */
    GPMA_K_BFS,           /* frontier expansion */
    GPMA_K_CC,            /* hooking sweep */
    GPMA_K_COUNT
};
int gpma_profile_enable(gpma_t *h, int enable);
int gpma_profile_reset(gpma_t *h);
int gpma_profile_read(gpma_t *h, int kernel, double *ms_total, uint64_t *launches,
                      double *bytes_total);

#ifdef __cplusplus
}
#endif
#endif /* GPMA_H */
