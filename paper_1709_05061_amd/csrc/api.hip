// Host side of the GPMA+ library: the C ABI, the handle, the density bounds,
// the level-by-level driver of the batched update (Section 5.2, Algorithm
// "GPMA+ Segment-Oriented Insertion" and its dual), root resize, and the
// analytics drivers.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "fused.h"
#include "locator.h"

using namespace gpma_dev;
using namespace gpma_host;

namespace {

constexpr uint64_t kMaxCap = 1ull << 31;   // row offsets are uint32
constexpr uint32_t kMaxLeaf = 512;

uint32_t ilog2(uint64_t x) {
    uint32_t r = 0;
    while (x > 1) { x >>= 1; r++; }
    return r;
}
uint32_t bit_width(uint64_t x) {
    uint32_t b = 0;
    while (x) { b++; x >>= 1; }
    return b;
}
uint64_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

struct Prof {
    int kind;
    hipEvent_t a, b;
    double bytes;
};

}  // namespace

struct gpma {
    uint32_t V = 0, lf = 0, lf_log2 = 0;
    uint32_t tau_leaf = 0, tau_root = 0, rho_leaf = 0, rho_root = 0;
    uint64_t cap = 0, L = 0;
    uint32_t H = 0;
    uint64_t n = 0;   // stored entries, guards included
    uint64_t *slots = nullptr;
    uint64_t *piv = nullptr;    // per leaf: its first slot, mark bit cleared (the locate's search array)
    uint16_t *cnt = nullptr;
    uint32_t *row_ptr = nullptr;
    uint32_t *deg = nullptr;
    uint32_t *dead = nullptr;   // lazy deletion: marked entries per leaf (null when off)

    // batch scratch
    uint64_t bcap = 0;
    uint64_t *kA = nullptr, *kB = nullptr, *kC = nullptr, *kD = nullptr;
    uint32_t *leafA = nullptr, *leafB = nullptr;
    uint8_t *stA = nullptr, *stB = nullptr;
    uint32_t *flags = nullptr, *tmp = nullptr;
    Ctl *ctl = nullptr;       // device
    Ctl *ctl_h = nullptr;     // pinned host mirror

    // device-tier scratch (grown on demand)
    uint64_t dt_cap = 0;
    uint64_t *dtA = nullptr, *dtB = nullptr;
    uint64_t dt_off_cap = 0;
    uint32_t *dt_off = nullptr, *dt_tmp = nullptr, *dt_tot = nullptr;

    // dst-major mirror (keys dst<<32|src), kept in step with every batch
    gpma *mir = nullptr;
    uint64_t *tkeys = nullptr;
    uint64_t tkeys_cap = 0;

    // analytics scratch
    double *pr_contrib = nullptr, *pr_y = nullptr, *pr_dang = nullptr;
    // destination-binned SpMV scratch (sized on use, grown as the array grows)
    uint32_t *pb_offs = nullptr, *pb_tmp = nullptr, *pb_small = nullptr;   // pb_small: total, pieces
    uint4 *pb_pieces = nullptr;
    uint64_t *pb_rec = nullptr, *pb_rec2 = nullptr;
    uint64_t *pb_keys = nullptr;   // each slot range's edges, packed once per call (cap words)
    uint32_t *pb_ne = nullptr;     // edges packed per range
    uint64_t pb_keys_cap = 0, pb_ne_cap = 0;
    uint32_t *pb_coffs = nullptr;
    uint64_t pb_offs_words = 0, pb_tmp_words = 0, pb_pieces_cap = 0, pb_rec_cap = 0, pb_rec2_cap = 0;
    uint64_t pb_coffs_words = 0;
    uint32_t *bfs_q0 = nullptr, *bfs_q1 = nullptr, *bfs_off = nullptr, *bfs_tmp = nullptr;
    uint32_t *cc_pick = nullptr;   // 1024 sampled labels
    uint32_t *small = nullptr;
    uint32_t *small_h = nullptr;   // pinned

    // fused batching: cached graphs (valid while geom_version is unchanged)
    struct GraphEntry {
        hipGraphExec_t exec;
        uint64_t cls;
        bool del;
        uint32_t version;
        uint64_t *fin_k;
        uint32_t *fin_l;
        uint8_t *fin_st;
        uint32_t *fin_n;
        uint32_t h_top;
        bool fin_raw;   // the leaf level was the last: pending updates left in place, uncompacted
    };
    std::vector<GraphEntry> graphs;
    // paired windows (this handle with its mirror, one launch per step): one
    // graph per window shape (the window's size class, then each batch's
    // size class and operation), valid while both handles' geom_version are
    // unchanged
    struct PairEntry {
        hipGraphExec_t exec;
        uint64_t wcls;
        std::vector<uint64_t> sig;   // per batch: size class * 2 + delete
        uint32_t vg, vm;             // geom_version of this handle and of its mirror
    };
    std::vector<PairEntry> pgraphs;
    uint32_t geom_version = 1;
    hipStream_t cap_stream = nullptr;
    // fused batching with a mirror: the mirror's batches run on side or
    // side2, whichever a probe found running beside the caller's stream, the
    // array's on the caller's stream.  Two pipelines on one
    // hardware queue run one after the other, and the runtime may put a
    // library stream on the caller's queue; when neither does better, the
    // array's batches take side and the mirror's side2 (created one after
    // the other, so on different queues).
    hipStream_t side = nullptr, side2 = nullptr;
    // probe results: caller stream -> the library stream that runs beside it
    // (nullptr: neither does); the most recent kProbeMemo callers
    std::vector<std::pair<hipStream_t, hipStream_t>> probes;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join2 = nullptr;
    uint64_t *kS = nullptr;              // window staging, then the current batch's keys
    FusedState *fs = nullptr;            // device
    uint32_t *werrs = nullptr;           // device: per window batch, generation of its invalid key
    uint32_t *wcount = nullptr;          // device: window keys
    uint32_t *ustart = nullptr;          // device: window batch starts in the sorted keys
    uint64_t *wukeys = nullptr;          // which sort buffer holds the window's sorted keys
    struct WindowEntry {
        hipGraphExec_t exec;
        uint32_t w;
        uint64_t cls;
        uint32_t version;
    };
    std::vector<WindowEntry> wgraphs;
    uint32_t *stop = nullptr;            // device stop flag of this handle's sequence
    BatchDesc *desc = nullptr;           // device table of the current chunk
    BatchOut *outs = nullptr;            // device per-batch results
    // fs, stop and outs live in one device block, mirrored by one pinned
    // block, so a window's results come back in one copy per handle
    uint64_t *fblk = nullptr;            // device block
    void *fblk_h = nullptr;              // pinned block
    void *fblk_hd = nullptr;             // its device view (kernels write the results there)
    FusedState *fs_h = nullptr;          // pinned mirror of *fs
    uint32_t *stop_h = nullptr;          // pinned
    FusedState *reset_h = nullptr;       // pinned source of state resets
    BatchDesc *desc_h = nullptr;         // pinned staging of the descriptor table
    BatchDesc *desc_hd = nullptr;        // its device view (read by the call's first kernel)
    BatchOut *outs_h = nullptr;          // pinned copy of the per-batch results

    bool readonly = false;   // a snapshot: analytics and exports only

    // learned segment locator
    bool learned = false;
    bool fused_direct = false;     // enqueue fused batches without graph capture
    int sort_chunks = 4;           // 64-key chunks per wave in batch sort tiles
    uint32_t fused_levels = 1;     // levels above the leaves in a fused batch
    LocModel *loc = nullptr;       // device
    LocModel loc_h{};              // host copy
    double *loc_gram = nullptr;    // device fp64 normal equations
    uint32_t *loc_err = nullptr;   // device
    uint32_t *loc_row_eps = nullptr;   // device, V: each row's leaf error bound
    uint32_t batches_since_fit = 0;
    uint64_t loc_lookups = 0, loc_misses = 0, loc_fits = 0;
    uint64_t acc_lookups = 0, acc_misses = 0;   // fused batches since the last check

    // lock-based GPMA comparator (allocated on first use, sized to the array)
    uint64_t *lk_scratch = nullptr;   // cap slots
    uint32_t *lk_locks = nullptr;     // 2L epoch words, node (h, s) at (L >> h) + s
    uint64_t lk_cap = 0;              // capacity the lock words were reset for
    uint64_t lk_buf = 0;              // capacity the two buffers hold
    uint32_t lk_epoch = 0;

    // device memory: the caller's allocator (hipMalloc/hipFree when none),
    // the stream of the call in progress (handed to the allocator), the size
    // of every live block and their total
    gpma_allocator alloc{};
    hipStream_t astream = nullptr;
    std::unordered_map<void *, size_t> blocks;
    uint64_t held_bytes = 0;
    // arrays for a root resize, reserved before a batch changes anything;
    // after a resize the old arrays join them until the call ends
    struct ArrBuf {
        uint64_t *slots;
        uint64_t *piv;
        uint16_t *cnt;
        uint32_t *dead;
        uint64_t cap;   // slots the buffer holds (>= the capacity it serves)
    };
    std::vector<ArrBuf> pool;
    uint64_t slots_buf = 0;    // slots the live arrays' buffers hold (>= cap)
    uint32_t spmv_form = 0;    // GPMA_SPMV_*
    bool lib_streams = false;  // GPMA_FLAG_FUSED_LIB_STREAMS
    bool window_radix = false; // GPMA_FLAG_WINDOW_RADIX

    Device dev;
    int prof_on = 0;
    std::vector<Prof> prof_pending;
    std::vector<hipEvent_t> ev_pool;
    double prof_ms[GPMA_K_COUNT] = {};
    double prof_bytes[GPMA_K_COUNT] = {};
    uint64_t prof_n[GPMA_K_COUNT] = {};
};

namespace {

// Device memory of a handle, through its allocator (hipMalloc / hipFree
// when the caller gave none).  The allocator gets the stream of the call in
// progress; a block goes back to it only after the device has finished every
// piece of the library's work (hipFree synchronises by itself).
template <typename T>
int dev_alloc(gpma *g, T **p, uint64_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    const size_t bytes = (size_t)count * sizeof(T);
    void *q = nullptr;
    if (g->alloc.alloc) {
        q = g->alloc.alloc(bytes, g->astream, g->alloc.ctx);
    } else if (hipMalloc(&q, bytes) != hipSuccess) {
        q = nullptr;
        (void)hipGetLastError();
    }
    if (!q) return GPMA_ENOMEM;
    g->blocks[q] = bytes;
    g->held_bytes += bytes;
    *p = (T *)q;
    return GPMA_OK;
}

template <typename T>
void dev_free(gpma *g, T *&p) {
    if (!p) return;
    size_t bytes = 0;
    auto it = g->blocks.find((void *)p);
    if (it != g->blocks.end()) {
        bytes = it->second;
        g->blocks.erase(it);
        g->held_bytes -= bytes;
    }
    if (g->alloc.free) {
        hipDeviceSynchronize();
        g->alloc.free((void *)p, bytes, g->astream, g->alloc.ctx);
    } else {
        hipFree((void *)p);
    }
    p = nullptr;
}

void set_stream(gpma *g, hipStream_t s) {
    g->astream = s;
    if (g->mir) g->mir->astream = s;
}

// ---------------------------------------------------------------------------
// density bounds (Section 4.1, figure "PMA insertion example")
//
// rho_h and tau_h move linearly with the height h from the leaf values to the
// root values; a one-leaf tree (H = 0) uses the root values.  With
// cap_h = lf * 2^h slots, an insertion passes iff (n+u)/cap_h < tau_h, i.e.
// n+u <= hi = ceil(tau_h*cap_h) - 1, and a deletion iff (n-d)/cap_h > rho_h,
// i.e. n-d >= lo = floor(rho_h*cap_h) + 1.  Exact in 64-bit integers:
// tau_h*cap_h = (tau_leaf*(H-h) + tau_root*h) * cap_h / (1000*H).
void bounds_at(uint32_t lf, uint32_t tl, uint32_t tr, uint32_t rl, uint32_t rr, uint32_t H,
               uint32_t h, uint64_t *lo, uint64_t *hi) {
    const uint64_t cap_h = (uint64_t)lf << h;
    const uint64_t wl = H ? (uint64_t)(H - h) : 0, wr = H ? (uint64_t)h : 1;
    const uint64_t den = 1000ull * (H ? H : 1);
    const uint64_t t = ((uint64_t)tl * wl + (uint64_t)tr * wr) * cap_h;
    const uint64_t r = ((uint64_t)rl * wl + (uint64_t)rr * wr) * cap_h;
    *hi = (t % den ? t / den + 1 : t / den) - 1;
    *lo = r / den + 1;
}

void bounds(const gpma *g, uint32_t H, uint32_t h, uint64_t *lo, uint64_t *hi) {
    bounds_at(g->lf, g->tau_leaf, g->tau_root, g->rho_leaf, g->rho_root, H, h, lo, hi);
}

uint64_t root_hi(const gpma *g, uint64_t cap) {
    uint64_t lo, hi;
    uint32_t H = ilog2(cap / g->lf);
    bounds(g, H, H, &lo, &hi);
    return hi;
}
uint64_t root_lo(const gpma *g, uint64_t cap) {
    uint64_t lo, hi;
    uint32_t H = ilog2(cap / g->lf);
    bounds(g, H, H, &lo, &hi);
    return lo;
}

bool params_valid(const gpma_params *p, bool allow_auto) {
    uint32_t lf = p->leaf_size;
    if (!(allow_auto && lf == 0)) {
        if (lf < 16 || lf > kMaxLeaf || (lf & (lf - 1))) return false;
        if ((uint64_t)p->rho_leaf_pm * lf < 1000) return false;
    }
    if (!(p->rho_leaf_pm > 0 && p->rho_leaf_pm <= p->rho_root_pm && p->rho_root_pm < p->tau_root_pm &&
          p->tau_root_pm <= p->tau_leaf_pm && p->tau_leaf_pm < 1000))
        return false;
    if (2 * p->rho_root_pm > p->tau_root_pm) return false;
    if (p->flags & ~(uint32_t)(GPMA_FLAG_MIRROR | GPMA_FLAG_LEARNED_LOCATOR | GPMA_FLAG_FUSED_DIRECT |
                               GPMA_FLAG_LAZY_DELETE | GPMA_FLAG_FUSED_LIB_STREAMS | GPMA_FLAG_WINDOW_RADIX))
        return false;
    if (p->spmv_form > GPMA_SPMV_BINNED_GATHER) return false;
    if (p->spmv_form == GPMA_SPMV_PULL && !(p->flags & GPMA_FLAG_MIRROR)) return false;
    if (p->sort_tile_keys != 0 && p->sort_tile_keys != 512 && p->sort_tile_keys != 1024 && p->sort_tile_keys != 2048)
        return false;
    if (p->fused_levels > 3) return false;
    return true;
}

// ---------------------------------------------------------------------------
// profiling

hipEvent_t ev_get(gpma *g) {
    if (!g->ev_pool.empty()) {
        hipEvent_t e = g->ev_pool.back();
        g->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    hipEventCreate(&e);
    return e;
}

struct ProfScope {
    gpma *g;
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr;
    ProfScope(gpma *g_, int k, hipStream_t s_) : g(g_), kind(k), s(s_) {
        if (g->prof_on) {
            a = ev_get(g);
            hipEventRecord(a, s);
        }
    }
    void done(double bytes) {
        if (!a) return;
        hipEvent_t b = ev_get(g);
        hipEventRecord(b, s);
        g->prof_pending.push_back(Prof{kind, a, b, bytes});
        a = nullptr;
    }
    ~ProfScope() { done(0.0); }
};

void prof_collect(gpma *g) {
    for (auto &p : g->prof_pending) {
        hipEventSynchronize(p.b);
        float ms = 0.f;
        hipEventElapsedTime(&ms, p.a, p.b);
        g->prof_ms[p.kind] += ms;
        g->prof_bytes[p.kind] += p.bytes;
        g->prof_n[p.kind] += 1;
        g->ev_pool.push_back(p.a);
        g->ev_pool.push_back(p.b);
    }
    g->prof_pending.clear();
}

// ---------------------------------------------------------------------------
// scratch management

void drop_graphs(gpma *g) {
    for (auto &e : g->graphs)
        if (e.exec) hipGraphExecDestroy(e.exec);
    g->graphs.clear();
    for (auto &e : g->wgraphs)
        if (e.exec) hipGraphExecDestroy(e.exec);
    g->wgraphs.clear();
    for (auto &e : g->pgraphs)
        if (e.exec) hipGraphExecDestroy(e.exec);
    g->pgraphs.clear();
    g->geom_version++;
}

void free_batch(gpma *g) {
    drop_graphs(g);
    g->wukeys = nullptr;   // the sort buffers go; the next window prefix picks them again
    dev_free(g, g->kS);
    dev_free(g, g->kA); dev_free(g, g->kB); dev_free(g, g->kC); dev_free(g, g->kD);
    dev_free(g, g->leafA); dev_free(g, g->leafB); dev_free(g, g->stA); dev_free(g, g->stB);
    dev_free(g, g->flags); dev_free(g, g->tmp);
    g->bcap = 0;
}

int ensure_batch(gpma *g, uint64_t b) {
    if (b <= g->bcap) return GPMA_OK;
    free_batch(g);
    uint64_t c = next_pow2(std::max<uint64_t>(b, 4096));
    size_t tw = std::max({radix_tmp_words(c), scan_tmp_words(c + 1), splitter_tmp_words(c)});
    int e = GPMA_OK;
    e |= dev_alloc(g, &g->kS, c);
    e |= dev_alloc(g, &g->kA, c); e |= dev_alloc(g, &g->kB, c);
    e |= dev_alloc(g, &g->kC, c); e |= dev_alloc(g, &g->kD, c);
    e |= dev_alloc(g, &g->leafA, c); e |= dev_alloc(g, &g->leafB, c);
    e |= dev_alloc(g, &g->stA, c); e |= dev_alloc(g, &g->stB, c);
    e |= dev_alloc(g, &g->flags, c + 1); e |= dev_alloc(g, &g->tmp, tw);
    if (e) {
        free_batch(g);
        return GPMA_ENOMEM;
    }
    g->bcap = c;
    return GPMA_OK;
}

int ensure_dt(gpma *g, uint64_t entries, uint64_t leaves) {
    if (entries > g->dt_cap) {
        dev_free(g, g->dtA); dev_free(g, g->dtB);
        g->dt_cap = 0;
        const uint64_t c = entries + entries / 8 + 4096;
        if (dev_alloc(g, &g->dtA, c) || dev_alloc(g, &g->dtB, c)) {
            dev_free(g, g->dtA); dev_free(g, g->dtB);
            return GPMA_ENOMEM;
        }
        g->dt_cap = c;
    }
    if (leaves > g->dt_off_cap) {
        dev_free(g, g->dt_off); dev_free(g, g->dt_tmp);
        g->dt_off_cap = 0;
        uint64_t c = next_pow2(leaves);
        if (dev_alloc(g, &g->dt_off, c) || dev_alloc(g, &g->dt_tmp, scan_tmp_words(c))) {
            dev_free(g, g->dt_off); dev_free(g, g->dt_tmp);
            return GPMA_ENOMEM;
        }
        g->dt_off_cap = c;
    }
    return GPMA_OK;
}

// ---------------------------------------------------------------------------
// reservation before a batch changes anything (so that GPMA_ENOMEM leaves
// the handle as it was)

// Add one set of root arrays holding `cap` slots to the pool.
int pool_add(gpma *g, uint64_t cap) {
    gpma::ArrBuf b{nullptr, nullptr, nullptr, nullptr, cap};
    int e = dev_alloc(g, &b.slots, cap);
    if (!e) e = dev_alloc(g, &b.piv, cap >> g->lf_log2);
    if (!e) e = dev_alloc(g, &b.cnt, cap >> g->lf_log2);
    if (!e && g->dead) e = dev_alloc(g, &b.dead, cap >> g->lf_log2);
    if (e) {
        dev_free(g, b.slots); dev_free(g, b.piv); dev_free(g, b.cnt); dev_free(g, b.dead);
        return GPMA_ENOMEM;
    }
    g->pool.push_back(b);
    return GPMA_OK;
}

// Free the pool: resize arrays that were not needed, and the arrays a resize
// replaced (after the device has finished with them).
void release_pool(gpma *g) {
    for (auto &b : g->pool) {
        dev_free(g, b.slots); dev_free(g, b.piv); dev_free(g, b.cnt); dev_free(g, b.dead);
    }
    g->pool.clear();
}

// Everything batches with at most ins_max insertions and del_max deletions
// in all may allocate below the root and at it: the merge workspace of the
// device tier and of the root (every entry plus the insertions, over the
// leaves of the largest capacity they can reach) and, when the root may be
// resized, `nres` sets of root arrays of the largest capacity a resize can
// pick (one for a single batch; two for a sequence, where the arrays a
// resize frees join the pool and one large set is always free).  A sequence
// whose entries could outgrow the largest array is refused (GPMA_ENOMEM).
int reserve_update(gpma *g, uint64_t ins_max, uint64_t del_max, int nres) {
    const uint64_t entries = g->n + ins_max;
    uint64_t cmax = g->cap;
    while (entries > root_hi(g, cmax)) {
        cmax *= 2;
        if (cmax > kMaxCap) return GPMA_ENOMEM;
    }
    int e = ensure_dt(g, entries, cmax >> g->lf_log2);
    if (e) return e;
    const bool grow = cmax > g->cap;
    const bool shrink = del_max > 0 && !g->dead && g->cap > g->lf &&
                        g->n - std::min(g->n - g->V, del_max) < root_lo(g, g->cap);
    if (!grow && !shrink) return GPMA_OK;
    const uint64_t need = nres > 1 ? cmax : (grow ? cmax : g->cap / 2);
    int have = 0;
    for (auto &b : g->pool)
        if (b.cap >= need) have++;
    for (; have < nres; have++)
        if ((e = pool_add(g, need))) return e;
    return GPMA_OK;
}

void read_ctl(gpma *g, hipStream_t s) {
    hipMemcpyAsync(g->ctl_h, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
    hipStreamSynchronize(s);
}

void drop_graphs(gpma *g);

void set_geometry(gpma *g, uint64_t cap) {
    if (g->cap != cap) drop_graphs(g);   // captured graphs hold the old arrays
    g->cap = cap;
    g->L = cap >> g->lf_log2;
    g->H = ilog2(g->L);
}

// Exclusive prefix of the leaf counts of leaves [first, first+P) into
// g->dt_off; returns the segment's entry count (one host sync).
int segment_offsets(gpma *g, uint64_t first, uint64_t P, uint64_t *ns, hipStream_t s) {
    int e = ensure_dt(g, 0, P);
    if (e) return e;
    launch_leaf_counts_u32(g->cnt, g->dead, first, P, g->dt_off, s);
    scan_u32(g->dt_off, g->dt_off, P, g->small, g->dt_tmp, s);
    hipMemcpyAsync(g->small_h, g->small, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    hipStreamSynchronize(s);
    *ns = g->small_h[0];
    return GPMA_OK;
}

// Root rebuild: merge every stored entry with the k remaining updates U and
// re-dispatch all of them evenly over ncap slots (ncap == cap: in place).  A
// new capacity takes the smallest reserved set of arrays that holds it; the
// replaced arrays join the pool (freed when the call ends).
int rebuild_root(gpma *g, bool del, const uint64_t *U, uint8_t *status, uint64_t k, uint64_t n_now,
                 uint64_t ncap, hipStream_t s) {
    uint64_t ns = 0;
    int e = segment_offsets(g, 0, g->L, &ns, s);
    if (e) return e;
    if (ns != n_now) return GPMA_EDEVICE;   // host and device disagree: refuse to write
    uint64_t N = del ? ns - k : ns + k;
    e = ensure_dt(g, ns + k, 0);
    if (e) return e;
    gpma::ArrBuf nb{g->slots, g->piv, g->cnt, g->dead, g->slots_buf};
    if (ncap != g->cap) {
        int best = -1;
        for (size_t i = 0; i < g->pool.size(); i++)
            if (g->pool[i].cap >= ncap && (best < 0 || g->pool[i].cap < g->pool[(size_t)best].cap)) best = (int)i;
        if (best < 0) {   // nothing reserved (a caller outside the update calls)
            if ((e = pool_add(g, ncap))) return e;
            best = (int)g->pool.size() - 1;
        }
        nb = g->pool[(size_t)best];
        g->pool.erase(g->pool.begin() + best);
    }
    launch_gather_segment(g->slots, g->cnt, g->dead, 0, g->L, g->lf, g->dt_off, g->dtA, s);
    launch_merge_sorted(del, g->dtA, ns, U, k, g->dtB, s);
    launch_dispatch(g->dtB, N, nb.slots, nb.piv, nb.cnt, nb.dead, g->row_ptr, 0, ncap >> g->lf_log2, g->lf, s);
    launch_mark_done(del, U, status, 0, k, g->deg, g->ctl, ncap, true, s);
    if (ncap != g->cap) {
        g->pool.push_back(gpma::ArrBuf{g->slots, g->piv, g->cnt, g->dead, g->slots_buf});
        g->slots = nb.slots;
        g->piv = nb.piv;
        g->cnt = nb.cnt;
        g->dead = nb.dead;
        g->slots_buf = nb.cap;
        set_geometry(g, ncap);
    }
    return GPMA_OK;
}


struct LevelArrays {
    uint64_t *k;
    uint32_t *l;
    uint8_t *st;
    uint32_t *n;   // device count of pending updates
};

// Host-driven device tier at height h: the remaining updates' leaves come
// back to the host, are grouped by segment, and every segment is counted,
// checked and (if it passes) gathered, merged and re-dispatched by kernels.
int device_tier_level(gpma *g, bool del, uint32_t h, const LevelArrays &c, uint64_t rem,
                      uint64_t lo, uint64_t hi, hipStream_t s) {
    // one scan of every leaf's live count, then the live entries of each
    // run's segment from it, read back with the runs' leaves in one round trip
    int e = ensure_dt(g, 0, g->L);
    if (e) return e;
    launch_leaf_counts_u32(g->cnt, g->dead, 0, g->L, g->dt_off, s);
    scan_u32(g->dt_off, g->dt_off, g->L, g->small, g->dt_tmp, s);
    launch_seg_live(c.l, rem, h, g->dt_off, g->L, g->small, g->flags, s);
    std::vector<uint32_t> lh(rem), nsh(rem);
    hipMemcpyAsync(lh.data(), c.l, rem * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    hipMemcpyAsync(nsh.data(), g->flags, rem * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) return GPMA_EDEVICE;
    const uint64_t P = 1ull << h;
    // the merge buffers for the largest passing segment, before any write
    uint64_t need = 0;
    for (uint64_t i = 0; i < rem;) {
        const uint32_t seg = lh[i] >> h;
        uint64_t j = i;
        while (j < rem && (lh[j] >> h) == seg) j++;
        const uint64_t k = j - i, ns = nsh[i];
        if (del ? (ns >= k + lo) : (ns + k <= hi)) need = std::max<uint64_t>(need, ns + k);
        i = j;
    }
    if (need && (e = ensure_dt(g, need, 0))) return e;
    for (uint64_t i = 0; i < rem;) {
        const uint32_t seg = lh[i] >> h;
        uint64_t j = i;
        while (j < rem && (lh[j] >> h) == seg) j++;
        const uint64_t k = j - i, first = (uint64_t)seg << h;
        const uint64_t ns = nsh[i];
        const bool pass = del ? (ns >= k + lo) : (ns + k <= hi);
        if (pass) {
            // the scan's part from this segment's first leaf (segments
            // rewritten earlier in the loop are disjoint from it)
            launch_gather_segment(g->slots, g->cnt, g->dead, first, P, g->lf, g->dt_off + first, g->dtA, s);
            launch_merge_sorted(del, g->dtA, ns, c.k + i, k, g->dtB, s);
            launch_dispatch(g->dtB, del ? ns - k : ns + k, g->slots, g->piv, g->cnt, g->dead, g->row_ptr, first, P,
                            g->lf, s);
            launch_mark_done(del, c.k, c.st, i, k, g->deg, g->ctl, P << g->lf_log2, false, s);
        }
        i = j;
    }
    return GPMA_OK;
}


// ---------------------------------------------------------------------------
// learned locator: fit and dispatch

void do_locate(gpma *g, const uint64_t *keys, const uint32_t *n_dev, uint64_t n_max, uint32_t *leaf,
               uint8_t *status, hipStream_t s, const WinSrc *ws = nullptr) {
    if (g->learned && g->loc)
        launch_locate_learned(keys, n_dev, n_max, g->piv, g->row_ptr, g->loc_row_eps, g->L, g->lf_log2, g->loc,
                              g->ctl, leaf, status, &g->ctl->misses, s, ws);
    else
        launch_locate(keys, n_dev, n_max, g->piv, g->L, g->ctl, leaf, status, s, ws);
}

// Cholesky solve of the (ridge-regularised) n x n normal equations
bool solve_spd(std::vector<double> &A, std::vector<double> &b, int n) {
    double tr = 0;
    for (int i = 0; i < n; i++) tr += A[i * n + i];
    const double ridge = 1e-12 * (tr / n) + 1e-300;
    for (int i = 0; i < n; i++) A[i * n + i] += ridge;
    for (int j = 0; j < n; j++) {
        double d = A[j * n + j];
        for (int k = 0; k < j; k++) d -= A[j * n + k] * A[j * n + k];
        if (!(d > 0)) return false;
        d = std::sqrt(d);
        A[j * n + j] = d;
        for (int i = j + 1; i < n; i++) {
            double v = A[i * n + j];
            for (int k = 0; k < j; k++) v -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = v / d;
        }
    }
    for (int i = 0; i < n; i++) {       // L y = b
        double v = b[i];
        for (int k = 0; k < i; k++) v -= A[i * n + k] * b[k];
        b[i] = v / A[i * n + i];
    }
    for (int i = n - 1; i >= 0; i--) {  // L^T w = y
        double v = b[i];
        for (int k = i + 1; k < n; k++) v -= A[k * n + i] * b[k];
        b[i] = v / A[i * n + i];
    }
    return true;
}

uint16_t host_bf16(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// Fit the model to the current leaf pivots: knots at quantiles of the pivots'
// destinations, layer 2 by least squares on (up to) 2^16 sampled long-row
// pivots, then the error bounds over every long-row pivot with the device
// inference code.  With no long rows the model is the skip term alone.
int locator_fit(gpma *g, hipStream_t s) {
    if (!g->loc) {
        int e = GPMA_OK;
        e |= dev_alloc(g, &g->loc, 1);
        e |= dev_alloc(g, &g->loc_gram, loc_gram_words());
        e |= dev_alloc(g, &g->loc_err, 1);
        e |= dev_alloc(g, &g->loc_row_eps, g->V);
        if (e) return GPMA_ENOMEM;
    }
    const uint64_t L = g->L;
    const uint64_t S = std::min<uint64_t>(L, 1u << 16), stride = L / S;
    // knots: destinations of up to 1024 evenly spaced pivots, sorted
    const uint64_t np = std::min<uint64_t>(1024, L);
    const uint64_t step = L / np;
    std::vector<uint64_t> piv(np);
    hipMemcpy2DAsync(piv.data(), sizeof(uint64_t), g->piv, step * sizeof(uint64_t),
                     sizeof(uint64_t), np, hipMemcpyDeviceToHost, s);
    hipStreamSynchronize(s);
    std::vector<uint32_t> dsts;
    for (uint64_t k : piv)
        if ((uint32_t)k != GPMA_GUARD_DST) dsts.push_back((uint32_t)k);
    std::sort(dsts.begin(), dsts.end());
    LocModel m{};
    m.V = g->V;
    m.inv_v = 1.0f / (float)g->V;
    m.inv_v1 = 1.0f / (float)((double)g->V + 1.0);
    m.L = (uint32_t)L;
    for (int u = 0; u < 31; u++) {
        const float q = dsts.empty() ? (float)u / 31.0f
                                     : (float)dsts[std::min<size_t>((size_t)u * dsts.size() / 31, dsts.size() - 1)] * m.inv_v1;
        m.w1x[u] = 0.0f;
        m.w1y[u] = 1.0f;
        m.b1[u] = -q;
    }
    m.w1x[31] = 1.0f;   // the row: R-MAT destinations depend on the source's bits
    m.w1y[31] = 0.0f;
    m.b1[31] = 0.0f;
    hipMemcpyAsync(g->loc, &m, sizeof(m), hipMemcpyHostToDevice, s);
    hipMemsetAsync(g->loc_gram, 0, loc_gram_words() * sizeof(double), s);
    launch_loc_gram(g->piv, g->row_ptr, L, g->lf_log2, stride, S, g->loc, g->loc_gram, s);
    std::vector<double> gram(loc_gram_words());
    hipMemcpyAsync(gram.data(), g->loc_gram, gram.size() * sizeof(double), hipMemcpyDeviceToHost, s);
    hipStreamSynchronize(s);
    const int F = 33;
    const double samples = gram[32 * F + 32];   // bias x bias: the number of samples used
    if (samples >= 64.0) {
        std::vector<double> A(gram.begin(), gram.begin() + F * F), b(gram.begin() + F * F, gram.end());
        if (solve_spd(A, b, F)) {
            for (int u = 0; u < 32; u++) m.w2[u] = host_bf16((float)b[u]);
            m.b2 = (float)b[32];
        }
    }
    m.eps = 0;
    m.valid = 0;
    hipMemcpyAsync(g->loc, &m, sizeof(m), hipMemcpyHostToDevice, s);
    hipMemsetAsync(g->loc_err, 0, sizeof(uint32_t), s);
    hipMemsetAsync(g->loc_row_eps, 0, (uint64_t)g->V * sizeof(uint32_t), s);
    launch_loc_eval(g->piv, g->row_ptr, L, g->lf_log2, g->loc, g->loc_err, g->loc_row_eps, s);
    uint32_t err = 0;
    hipMemcpyAsync(&err, g->loc_err, sizeof(err), hipMemcpyDeviceToHost, s);
    hipStreamSynchronize(s);
    m.eps = err;
    m.valid = 1;
    hipMemcpyAsync(g->loc, &m, sizeof(m), hipMemcpyHostToDevice, s);
    hipStreamSynchronize(s);
    g->loc_h = m;
    g->batches_since_fit = 0;
    g->loc_fits++;
    return GPMA_OK;
}

// Refit after the array was rebuilt or resized (the pivots all moved), or
// when more than 1/16 of the lookups since the last check fell back to the
// binary search (merges have shifted the pivots the model was fitted to).
// The result never depends on the fit; only the lookup cost does.
int locator_after_batch(gpma *g, uint64_t lookups, uint64_t misses, bool rebuilt, hipStream_t s) {
    if (!g->learned) return GPMA_OK;
    g->loc_lookups += lookups;
    g->loc_misses += misses;
    g->batches_since_fit++;
    if (rebuilt || g->loc_h.L != g->L || misses * 16 > lookups) return locator_fit(g, s);
    return GPMA_OK;
}

// Levels h_start .. H-1 and the root for the updates still pending in `cur`
// (rem of them; g->ctl holds the batch's counters so far).  Shared by the
// plain path and by the completion of a fused batch that stopped.
int finish_levels(gpma *g, bool del, LevelArrays cur, uint64_t rem, uint32_t h_start, uint32_t segs_seen,
                  gpma_stats *st, hipStream_t s) {
    int e = GPMA_OK;
    uint64_t lo, hi;
    hipEvent_t pa = nullptr, pb = nullptr;
    LevelArrays nxt;
    auto other = [&](const LevelArrays &c) {
        LevelArrays o;
        o.k = (c.k == g->kC) ? g->kD : g->kC;
        o.l = (c.l == g->leafB) ? g->leafA : g->leafB;
        o.st = (c.st == g->stB) ? g->stA : g->stB;
        o.n = (c.n == &g->ctl->lvl[0]) ? &g->ctl->lvl[1] : &g->ctl->lvl[0];
        return o;
    };
    nxt = other(cur);

    // levels h_start .. H-1: ascend with whatever is left
    for (uint32_t h = h_start; h < g->H && rem > 0; h++) {
        bounds(g, g->H, h, &lo, &hi);
        if (seg_merge_lds_bytes(g->lf, h) <= (size_t)g->dev.max_lds) {
            pa = pb = nullptr;
            if (g->prof_on) { pa = ev_get(g); hipEventRecord(pa, s); }
            launch_seg_merge(del, h, cur.k, cur.l, cur.st, cur.n, rem, g->slots, g->piv, g->cnt, g->row_ptr,
                             g->deg, g->dead, g->lf, lo, hi, g->ctl, s);
            if (g->prof_on) { pb = ev_get(g); hipEventRecord(pb, s); }
        } else {
            pa = pb = nullptr;
            e = device_tier_level(g, del, h, cur, rem, lo, hi, s);
            if (e) {
                // the merges made so far stand: keep the entry count in step
                read_ctl(g, s);
                g->n = (uint64_t)((int64_t)g->n + g->ctl_h->dn);
                return e;
            }
        }
        compact_pending(cur.k, cur.l, cur.st, cur.n, rem, nxt.k, nxt.l, nxt.st, nxt.n, g->flags,
                        g->tmp, del, (uint64_t)g->lf << h, g->ctl, s);
        read_ctl(g, s);
        const uint32_t segs_h = g->ctl_h->segs - segs_seen;
        segs_seen = g->ctl_h->segs;
        if (pa) g->prof_pending.push_back(Prof{GPMA_K_SEG_MERGE, pa, pb,
                                               16.0 * (double)(g->lf << h) * segs_h + 12.0 * (double)rem});
        if (st) {
            st->segments_merged[h] += segs_h;
            if (segs_h) st->top_level = (int32_t)h;
        }
        rem = (nxt.n == &g->ctl->lvl[0]) ? g->ctl_h->lvl[0] : g->ctl_h->lvl[1];
        cur = nxt;
        nxt = other(cur);
    }

    // the root: absorb in place when the bound holds, else resize
    bool resized = false;
    if (rem > 0) {
        const uint64_t n_now = (uint64_t)((int64_t)g->n + g->ctl_h->dn);
        uint64_t ncap = g->cap;
        if (!del) {
            while (n_now + rem > root_hi(g, ncap)) ncap *= 2;
        } else {
            const uint64_t left = n_now - rem;
            while (ncap > g->lf && left < root_lo(g, ncap) && left <= root_hi(g, ncap / 2)) ncap /= 2;
        }
        // on failure the merges below the root stand: keep n in step with them
        if (ncap > kMaxCap) {
            g->n = n_now;
            return GPMA_ENOMEM;
        }
        const uint32_t Hold = g->H;
        const uint64_t cap_old = g->cap;
        e = rebuild_root(g, del, cur.k, cur.st, rem, n_now, ncap, s);
        if (e) {
            g->n = n_now;
            return e;
        }
        read_ctl(g, s);
        resized = g->cap != cap_old;
        if (st) {
            st->segments_merged[Hold] += 1;
            st->top_level = (int32_t)Hold;
        }
    }
    g->n = (uint64_t)((int64_t)g->n + g->ctl_h->dn);
    if (st) {
        st->applied += g->ctl_h->applied;
        st->slots_rewritten += g->ctl_h->rewritten;
        st->resized |= resized ? 1 : 0;
    }
    return GPMA_OK;
}

int apply_batch(gpma *g, const uint64_t *keys, uint64_t b, bool del, hipStream_t s,
                gpma_stats *st) {
    if (st) {
        memset(st, 0, sizeof(*st));
        st->requested = b;
        st->top_level = -1;
    }
    if (b == 0) return GPMA_OK;
    if (!keys || b >= (1ull << 31)) return GPMA_EINVAL;
    int e = ensure_batch(g, b);
    if (e) return e;

    // Sort(U) and drop repeats
    hipMemsetAsync(g->ctl, 0, sizeof(Ctl), s);
    const uint32_t sb = bit_width(g->V - 1);
    const uint64_t *sorted;
    {
        ProfScope ps(g, GPMA_K_SORT, s);
        sorted = radix_sort_keys(keys, b, sb, sb, g->V, g->kA, g->kB, g->tmp, s, nullptr, g->ctl, g->sort_chunks);
        ps.done(16.0 * (double)b * (double)((2 * sb + 7) / 8));
    }
    uint64_t *ukeys = (sorted == g->kA) ? g->kB : g->kA;
    LevelArrays cur{ukeys, g->leafA, g->stA, &g->ctl->n_in};
    LevelArrays nxt{g->kC, g->leafB, g->stB, &g->ctl->lvl[0]};
    unique_sorted(sorted, b, ukeys, cur.n, g->flags, g->tmp, s);

    // BinarySearchLeafSegments
    {
        ProfScope ps(g, GPMA_K_LOCATE, s);
        do_locate(g, cur.k, cur.n, b, cur.l, cur.st, s);
        ps.done(16.0 * (double)b);
    }

    // level 0 (fused with the no-op probe); with lazy deletion a delete only
    // marks its entry and never reaches the levels
    const bool mark = del && g->dead;
    uint64_t lo, hi;
    bounds(g, g->H, 0, &lo, &hi);
    hipEvent_t pa = nullptr, pb = nullptr;
    if (g->prof_on) { pa = ev_get(g); hipEventRecord(pa, s); }
    if (mark)
        launch_leaf_mark(cur.k, cur.l, cur.st, cur.n, b, g->slots, g->cnt, g->dead, g->deg, g->lf, g->ctl, s);
    else
        launch_leaf_merge(del, cur.k, cur.l, cur.st, cur.n, b, g->slots, g->piv, g->cnt, g->row_ptr, g->deg, g->dead,
                          g->lf, lo, hi, g->ctl, s);
    if (g->prof_on) { pb = ev_get(g); hipEventRecord(pb, s); }
    compact_pending(cur.k, cur.l, cur.st, cur.n, b, nxt.k, nxt.l, nxt.st, nxt.n, g->flags, g->tmp, del,
                    g->lf, g->ctl, s);
    read_ctl(g, s);
    if (g->ctl_h->err) {
        if (pa) { g->ev_pool.push_back(pa); g->ev_pool.push_back(pb); }
        return GPMA_EINVAL;
    }
    const uint64_t distinct = g->ctl_h->n_in;
    uint32_t segs_seen = g->ctl_h->segs;
    if (pa) g->prof_pending.push_back(Prof{GPMA_K_LEAF_MERGE, pa, pb,
                                           mark ? 20.0 * (double)distinct
                                                : 16.0 * g->lf * segs_seen + 12.0 * (double)distinct});
    if (st) {
        st->segments_merged[0] = segs_seen;
        if (segs_seen) st->top_level = 0;
    }
    uint64_t rem = g->ctl_h->lvl[0];
    std::swap(cur, nxt);
    const uint64_t cap_before = g->cap;
    const uint32_t misses = g->ctl_h->misses;
    e = finish_levels(g, del, cur, rem, 1, segs_seen, st, s);
    if (st) st->noops = b - st->applied;
    if (!e) e = locator_after_batch(g, distinct, misses, g->cap != cap_before, s);
    return e;
}

void free_all(gpma *g) {
    release_pool(g);
    free_batch(g);
    dev_free(g, g->loc); dev_free(g, g->loc_gram); dev_free(g, g->loc_err); dev_free(g, g->loc_row_eps);
    dev_free(g, g->tkeys);
    dev_free(g, g->fblk); dev_free(g, g->desc);
    g->fs = nullptr;
    g->stop = nullptr;
    g->outs = nullptr;
    dev_free(g, g->werrs); dev_free(g, g->wcount); dev_free(g, g->ustart);
    if (g->fblk_h) hipHostFree(g->fblk_h);
    g->fblk_h = nullptr;
    if (g->reset_h) hipHostFree(g->reset_h);
    if (g->desc_h) hipHostFree(g->desc_h);
    g->fs_h = nullptr;
    g->stop_h = nullptr;
    g->reset_h = nullptr;
    g->desc_h = nullptr;
    g->desc_hd = nullptr;
    g->fblk_hd = nullptr;
    g->outs_h = nullptr;
    if (g->cap_stream) hipStreamDestroy(g->cap_stream);
    g->cap_stream = nullptr;
    if (g->side) hipStreamDestroy(g->side);
    if (g->side2) hipStreamDestroy(g->side2);
    g->side = g->side2 = nullptr;
    if (g->ev_fork) hipEventDestroy(g->ev_fork);
    if (g->ev_join) hipEventDestroy(g->ev_join);
    if (g->ev_join2) hipEventDestroy(g->ev_join2);
    g->ev_fork = g->ev_join = g->ev_join2 = nullptr;
    dev_free(g, g->slots); dev_free(g, g->piv); dev_free(g, g->cnt); dev_free(g, g->row_ptr); dev_free(g, g->deg);
    dev_free(g, g->dead);
    dev_free(g, g->lk_scratch); dev_free(g, g->lk_locks);
    dev_free(g, g->dtA); dev_free(g, g->dtB); dev_free(g, g->dt_off); dev_free(g, g->dt_tmp);
    dev_free(g, g->pr_contrib); dev_free(g, g->pr_y); dev_free(g, g->pr_dang);
    dev_free(g, g->pb_offs); dev_free(g, g->pb_tmp); dev_free(g, g->pb_small); dev_free(g, g->pb_pieces); dev_free(g, g->pb_rec);
    dev_free(g, g->pb_rec2); dev_free(g, g->pb_coffs); dev_free(g, g->pb_keys); dev_free(g, g->pb_ne);
    g->pb_offs_words = g->pb_tmp_words = g->pb_pieces_cap = g->pb_rec_cap = g->pb_rec2_cap = g->pb_coffs_words = 0;
    g->pb_keys_cap = g->pb_ne_cap = 0;
    dev_free(g, g->bfs_q0); dev_free(g, g->bfs_q1); dev_free(g, g->bfs_off); dev_free(g, g->bfs_tmp);
    dev_free(g, g->cc_pick);
    dev_free(g, g->small);
    dev_free(g, g->ctl);
    if (g->ctl_h) hipHostFree(g->ctl_h);
    if (g->small_h) hipHostFree(g->small_h);
    g->ctl_h = nullptr;
    g->small_h = nullptr;
    for (auto &p : g->prof_pending) { hipEventDestroy(p.a); hipEventDestroy(p.b); }
    g->prof_pending.clear();
    for (auto e : g->ev_pool) hipEventDestroy(e);
    g->ev_pool.clear();
}

// ---------------------------------------------------------------------------
// fused batching (host side)

constexpr uint32_t kFusedChunk = 4096;   // batches per descriptor table

uint64_t batch_class(uint64_t b) { return next_pow2(std::max<uint64_t>(b, 1024)); }

// layout of the fused block: FusedState, the stop flag, the per-batch results
constexpr size_t kFbStop = (sizeof(FusedState) + 15) / 16 * 16;
constexpr size_t kFbOuts = kFbStop + 16;
constexpr size_t kFbBytes = kFbOuts + kFusedChunk * sizeof(BatchOut);

int ensure_fused(gpma *g) {
    if (g->fs) return GPMA_OK;
    int e = GPMA_OK;
    e |= dev_alloc(g, &g->fblk, (kFbBytes + 7) / 8);
    if (!e) {
        uint8_t *b = (uint8_t *)g->fblk;
        g->fs = (FusedState *)b;
        g->stop = (uint32_t *)(b + kFbStop);
        g->outs = (BatchOut *)(b + kFbOuts);
    }
    e |= dev_alloc(g, &g->desc, kFusedChunk);
    // the pinned blocks that kernels read or write over the bus are coherent
    // (not cached on the device), so each side sees the other's latest writes
    constexpr unsigned kBusFlags = hipHostMallocMapped | hipHostMallocCoherent;
    if (hipHostMalloc(&g->fblk_h, kFbBytes, kBusFlags) != hipSuccess) {
        g->fblk_h = nullptr;
        e = GPMA_ENOMEM;
    } else {
        uint8_t *b = (uint8_t *)g->fblk_h;
        g->fs_h = (FusedState *)b;
        g->stop_h = (uint32_t *)(b + kFbStop);
        g->outs_h = (BatchOut *)(b + kFbOuts);
        if (hipHostGetDevicePointer(&g->fblk_hd, g->fblk_h, 0) != hipSuccess) e = GPMA_EDEVICE;
    }
    if (hipHostMalloc((void **)&g->reset_h, sizeof(FusedState), 0) != hipSuccess) e = GPMA_ENOMEM;
    if (hipHostMalloc((void **)&g->desc_h, kFusedChunk * sizeof(BatchDesc), kBusFlags) != hipSuccess) e = GPMA_ENOMEM;
    else if (hipHostGetDevicePointer((void **)&g->desc_hd, g->desc_h, 0) != hipSuccess) e = GPMA_EDEVICE;
    if (!e && hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking) != hipSuccess) e = GPMA_EDEVICE;
    if (!e && hipStreamCreateWithFlags(&g->side, hipStreamNonBlocking) != hipSuccess) e = GPMA_EDEVICE;
    if (!e && hipStreamCreateWithFlags(&g->side2, hipStreamNonBlocking) != hipSuccess) e = GPMA_EDEVICE;
    if (!e && hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming) != hipSuccess) e = GPMA_EDEVICE;
    if (!e && hipEventCreateWithFlags(&g->ev_join, hipEventDisableTiming) != hipSuccess) e = GPMA_EDEVICE;
    if (!e && hipEventCreateWithFlags(&g->ev_join2, hipEventDisableTiming) != hipSuccess) e = GPMA_EDEVICE;
    e |= dev_alloc(g, &g->werrs, kWindowMax);
    e |= dev_alloc(g, &g->wcount, 2);
    e |= dev_alloc(g, &g->ustart, kWindowMax + 1);
    if (!e) {
        // window generations start at 1 so that zeroed error flags mean valid
        memset(g->reset_h, 0, sizeof(FusedState));
        g->reset_h->gen = 1;
        hipMemcpy(g->fs, g->reset_h, sizeof(FusedState), hipMemcpyHostToDevice);
        hipMemset(g->werrs, 0, kWindowMax * sizeof(uint32_t));
    }
    return e;
}

// Tag bits of a window (0: this handle's vertex ids leave no room, windows
// hold one batch).
uint32_t window_tag_bits(const gpma *g) {
    const uint32_t sb = bit_width(g->V - 1);
    return sb + kWindowTagBits <= 32 ? kWindowTagBits : 0;
}

// Enqueue the prefix of a window of w batches from the handle's current batch
// (at most n_max keys in all): fetch, validate and tag, one sort of the whole
// window (batch tag above the source bits), batch starts.  Repeats stay in
// the sorted keys, next to each other: the leaf merge and the mark kernel
// treat a key equal to the one before it as a no-op.
void enqueue_window_prefix(gpma *g, uint32_t w, uint64_t n_max, const BatchDesc *desc, const uint32_t *stop,
                           bool transpose, hipStream_t s) {
    const uint32_t sb = bit_width(g->V - 1);
    const uint32_t tb = window_tag_bits(g);
    launch_window_fetch(desc, g->fs, stop, w, n_max, g->V, sb, transpose, g->kS, g->wcount, g->werrs, g->ustart, s);
    // both sorts leave the keys in the same buffer (fixed by the bit count);
    // the splitter sort's first launch also advances the window generation
    // and zeroes the locate's miss count, the radix sort leaves that to
    // launch_window_starts
    const bool splitter = !g->window_radix && splitter_sort_fits(n_max);
    const uint64_t *sorted =
        splitter ? splitter_sort_keys(g->kS, n_max, g->wcount, sb + tb, sb, g->V, g->kA, g->kB, g->tmp, s,
                                      &g->fs->gen, &g->ctl->misses)
                 : radix_sort_keys(g->kS, n_max, sb + tb, sb, g->V, g->kA, g->kB, g->tmp, s, g->wcount, nullptr,
                                   g->sort_chunks);
    if (!splitter) launch_window_starts(sorted, g->wcount, w, sb, g->ustart, g->fs, g->ctl, s);
    g->wukeys = const_cast<uint64_t *>(sorted);   // the same buffer for every window (fixed pass count)
}

gpma::WindowEntry *get_window_graph(gpma *g, uint32_t w, uint64_t cls, const BatchDesc *desc, const uint32_t *stop,
                                    bool transpose) {
    for (auto &e : g->wgraphs)
        if (e.w == w && e.cls == cls && e.version == g->geom_version) return &e;
    gpma::WindowEntry we{};
    we.w = w;
    we.cls = cls;
    we.version = g->geom_version;
    if (g->fused_direct) {
        g->wgraphs.push_back(we);
        return &g->wgraphs.back();
    }
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    enqueue_window_prefix(g, w, cls, desc, stop, transpose, g->cap_stream);
    if (hipStreamEndCapture(g->cap_stream, &graph) != hipSuccess || !graph) return nullptr;
    hipError_t r = hipGraphInstantiate(&we.exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (r != hipSuccess) return nullptr;
    g->wgraphs.push_back(we);
    return &g->wgraphs.back();
}

// Enqueue one batch of a fused sequence with device-side control only (no
// host reads), for batches of at most `cls` keys: take the batch's keys from
// its window's sorted keys, locate, level 0, then levels 1..h_top of
// the workgroup tier, then finish.  Returns where the pending updates end up.
void enqueue_device_batch(gpma *g, bool del, uint64_t cls, const BatchDesc *desc, uint32_t *stop,
                          bool transpose, hipStream_t s, gpma::GraphEntry *ge) {
    (void)desc;
    (void)transpose;
    const uint32_t sb = bit_width(g->V - 1);
    // the locate kernel takes the batch's keys from the window itself (into
    // kS) and resets the control block
    const WinSrc ws{&g->fs->batch, &g->fs->wstart, &g->fs->gen, stop, g->wukeys, g->ustart, g->werrs,
                    ~(((1ull << kWindowTagBits) - 1) << (32 + sb)), g->kS, g->ctl};
    LevelArrays cur{g->kS, g->leafA, g->stA, &g->ctl->n_in};
    LevelArrays nxt{g->kC, g->leafB, g->stB, &g->ctl->lvl[0]};
    do_locate(g, nullptr, cur.n, cls, cur.l, cur.st, s, &ws);
    uint64_t lo, hi;
    bounds(g, g->H, 0, &lo, &hi);
    const bool mark = del && g->dead;   // lazy deletion: marks only, no levels
    // no level above the leaves on the device: the leaf merge leaves
    // per-block figures (in the batch scratch, free until the next window's
    // sort) that the finishing kernel sums; the host gathers the pending
    // updates only for a batch that stops
    const bool upper = !mark && g->fused_levels >= 1 && g->H > 1 &&
                       seg_merge_lds_bytes(g->lf, 1) <= (size_t)g->dev.max_lds;
    if (!mark && !upper) {
        launch_leaf_merge(del, cur.k, cur.l, cur.st, cur.n, cls, g->slots, g->piv, g->cnt, g->row_ptr, g->deg, g->dead,
                          g->lf, lo, hi, g->ctl, s, g->tmp);
        launch_finish_leaf(g->fs, stop, g->ctl, g->tmp, leaf_merge_blocks(g->lf, cls), del, g->lf, g->outs, s);
        ge->fin_k = cur.k;
        ge->fin_l = cur.l;
        ge->fin_st = cur.st;
        ge->fin_n = nxt.n;
        ge->h_top = 0;
        ge->fin_raw = true;
        return;
    }
    if (mark)
        launch_leaf_mark(cur.k, cur.l, cur.st, cur.n, cls, g->slots, g->cnt, g->dead, g->deg, g->lf, g->ctl, s);
    else
        launch_leaf_merge(del, cur.k, cur.l, cur.st, cur.n, cls, g->slots, g->piv, g->cnt, g->row_ptr, g->deg, g->dead,
                          g->lf, lo, hi, g->ctl, s);
    compact_pending(cur.k, cur.l, cur.st, cur.n, cls, nxt.k, nxt.l, nxt.st, nxt.n, g->flags, g->tmp, del, g->lf,
                    g->ctl, s);
    auto other = [&](const LevelArrays &c) {
        LevelArrays o;
        o.k = (c.k == g->kC) ? g->kD : g->kC;
        o.l = (c.l == g->leafB) ? g->leafA : g->leafB;
        o.st = (c.st == g->stB) ? g->stA : g->stB;
        o.n = (c.n == &g->ctl->lvl[0]) ? &g->ctl->lvl[1] : &g->ctl->lvl[0];
        return o;
    };
    cur = nxt;
    nxt = other(cur);
    uint32_t h_top = 0;
    // levels above the leaves that a batch covers (g->fused_levels); a batch
    // with updates left above them stops the sequence and finishes on the
    // host-driven path
    for (uint32_t h = 1; !mark && h <= g->fused_levels && h < g->H &&
                         seg_merge_lds_bytes(g->lf, h) <= (size_t)g->dev.max_lds;
         h++) {
        bounds(g, g->H, h, &lo, &hi);
        launch_seg_merge(del, h, cur.k, cur.l, cur.st, cur.n, cls, g->slots, g->piv, g->cnt, g->row_ptr, g->deg, g->dead,
                         g->lf, lo, hi, g->ctl, s);
        compact_pending(cur.k, cur.l, cur.st, cur.n, cls, nxt.k, nxt.l, nxt.st, nxt.n, g->flags, g->tmp, del,
                        (uint64_t)g->lf << h, g->ctl, s);
        cur = nxt;
        nxt = other(cur);
        h_top = h;
    }
    launch_finish(g->fs, stop, g->ctl, cur.n, g->outs, s);
    ge->fin_k = cur.k;
    ge->fin_l = cur.l;
    ge->fin_st = cur.st;
    ge->fin_n = cur.n;
    ge->h_top = h_top;
    ge->fin_raw = false;
}

// ---- paired windows: the array g and its mirror m run every step of a
// window in one launch (the grid's y index picks the side), so a window takes
// half the launches.  Used when both sides take the same kernels: the
// splitter sort without a count scan, the leaf level as the last device
// level (merges, or marks for a lazy-deletion delete batch), the same
// locate.

bool pairable_window(const gpma *g, const gpma *m, uint64_t wcls) {
    for (const gpma *h : {g, m})
        if (h->fused_direct || h->window_radix || h->lib_streams || !window_tag_bits(h) || h->bcap != g->bcap)
            return false;
    if (g->lf != m->lf || g->V != m->V || (g->learned && g->loc) != (m->learned && m->loc)) return false;
    if ((g->dead != nullptr) != (m->dead != nullptr)) return false;   // lazy deletion on both sides or neither
    if (!splitter_sort_pairable(wcls)) return false;
    for (const gpma *h : {g, m}) {
        const bool upper = h->fused_levels >= 1 && h->H > 1 && seg_merge_lds_bytes(h->lf, 1) <= (size_t)h->dev.max_lds;
        if (upper) return false;
    }
    return true;
}

void enqueue_window_prefix2(gpma *g, gpma *m, uint32_t w, uint64_t n_max, const BatchDesc *desc, hipStream_t s) {
    const uint32_t sb = bit_width(g->V - 1);
    const uint32_t tb = window_tag_bits(g);
    gpma *h[2] = {g, m};
    FusedState *st[2] = {g->fs, m->fs};
    const uint32_t *stop[2] = {g->stop, m->stop};
    uint64_t *kS[2] = {g->kS, m->kS};
    uint32_t *wcount[2] = {g->wcount, m->wcount};
    uint32_t *errs[2] = {g->werrs, m->werrs};
    uint32_t *ustart[2] = {g->ustart, m->ustart};
    uint32_t *gen[2] = {&g->fs->gen, &m->fs->gen};
    uint32_t *misses[2] = {&g->ctl->misses, &m->ctl->misses};
    // the fetch also samples and sorts the splitters
    uint64_t *spl[2] = {splitter_spl(g->tmp), splitter_spl(m->tmp)};
    launch_window_fetch2(desc, st, stop, w, n_max, g->V, sb, kS, wcount, errs, ustart, spl, splitter_buckets(n_max),
                         splitter_sample_size(n_max), s);
    const uint64_t *in[2] = {g->kS, m->kS};
    const uint32_t *nd[2] = {g->wcount, m->wcount};
    uint64_t *ba[2] = {g->kA, m->kA}, *bb[2] = {g->kB, m->kB};
    uint32_t *tmp[2] = {g->tmp, m->tmp};
    const int which = splitter_sort_keys2(in, n_max, nd, sb + tb, sb, ba, bb, tmp, s, gen, misses);
    for (int k = 0; k < 2; k++) h[k]->wukeys = which ? h[k]->kB : h[k]->kA;
}

void enqueue_device_batch2(gpma *g, gpma *m, bool del, uint64_t cls, uint32_t pos, hipStream_t s) {
    const uint32_t sb = bit_width(g->V - 1);
    const uint64_t tmask = ~(((1ull << kWindowTagBits) - 1) << (32 + sb));
    gpma *h[2] = {g, m};
    WinSrc ws[2];
    const uint64_t *piv_c[2], *keys_c[2];
    uint64_t *slots[2], *piv[2], L[2], lo[2], hi[2];
    const uint32_t *row_ptr_c[2], *reps[2], *leaf_c[2], *nd[2];
    uint32_t *leaf[2], *misses[2], *row_ptr[2], *deg[2], *dead[2], *part[2], *stop[2];
    uint8_t *status[2];
    uint16_t *cnt[2];
    Ctl *ctl[2];
    const Ctl *ctl_c[2];
    const LocModel *model[2];
    FusedState *st[2];
    BatchOut *outs[2];
    const uint32_t *part_c[2];
    for (int k = 0; k < 2; k++) {
        gpma *x = h[k];
        // the window's graph runs its batches in order: this one is at pos
        ws[k] = WinSrc{&x->fs->batch, &x->fs->wstart, &x->fs->gen, x->stop, x->wukeys, x->ustart, x->werrs, tmask,
                       x->kS, x->ctl, (int32_t)pos};
        slots[k] = x->slots;
        piv[k] = x->piv;
        piv_c[k] = x->piv;
        keys_c[k] = x->kS;
        L[k] = x->L;
        bounds(x, x->H, 0, &lo[k], &hi[k]);
        row_ptr[k] = x->row_ptr;
        row_ptr_c[k] = x->row_ptr;
        reps[k] = x->loc_row_eps;
        leaf[k] = x->leafA;
        leaf_c[k] = x->leafA;
        status[k] = x->stA;
        nd[k] = &x->ctl->n_in;
        misses[k] = &x->ctl->misses;
        deg[k] = x->deg;
        dead[k] = x->dead;
        cnt[k] = x->cnt;
        ctl[k] = x->ctl;
        ctl_c[k] = x->ctl;
        model[k] = x->loc;
        part[k] = x->tmp;
        part_c[k] = x->tmp;
        stop[k] = x->stop;
        st[k] = x->fs;
        outs[k] = x->outs;
    }
    if (g->learned && g->loc)
        launch_locate_learned2(cls, piv_c, row_ptr_c, reps, L, g->lf_log2, model, ctl_c, leaf, status, misses, ws,
                               s);
    else
        launch_locate2(cls, piv_c, L, ctl_c, leaf, status, ws, s);
    // a lazy-deletion delete batch marks its keys in place; anything else
    // merges into the leaves
    const bool mark = del && g->dead;
    if (mark)
        launch_leaf_mark2(keys_c, leaf_c, status, nd, cls, slots, cnt, dead, deg, g->lf, ctl_c, part, s);
    else
        launch_leaf_merge2(del, keys_c, leaf_c, status, nd, cls, slots, piv, cnt, row_ptr, deg, dead, g->lf, lo, hi,
                           ctl, part, s);
    // each finished batch also lands in the handle's pinned block
    void *host[2] = {g->fblk_hd, m->fblk_hd};
    const uint64_t nparts = mark ? leaf_mark_blocks(cls) : leaf_merge_blocks(g->lf, cls);
    launch_finish_leaf2(st, stop, ctl, part_c, nparts, del, g->lf, outs, host, (uint32_t)kFbOuts, s);
}

constexpr size_t kPairGraphs = 32;   // window shapes kept per handle

// The cached graph of a whole paired window: its prefix, then every batch.
hipGraphExec_t get_pair_graph(gpma *g, gpma *m, uint64_t wcls, const uint8_t *ops, const uint64_t *sizes,
                              uint32_t from, uint32_t to, const BatchDesc *desc) {
    std::vector<uint64_t> sig;
    for (uint32_t i = from; i < to; i++) sig.push_back(batch_class(sizes[i]) * 2 + (ops[i] ? 1 : 0));
    // entries of an older geometry of either side go first
    for (size_t i = 0; i < g->pgraphs.size();) {
        auto &e = g->pgraphs[i];
        if (e.vg != g->geom_version || e.vm != m->geom_version) {
            if (e.exec) hipGraphExecDestroy(e.exec);
            g->pgraphs.erase(g->pgraphs.begin() + (ptrdiff_t)i);
        } else {
            i++;
        }
    }
    for (auto &e : g->pgraphs)
        if (e.wcls == wcls && e.sig == sig) return e.exec;
    if (g->pgraphs.size() >= kPairGraphs) {   // the oldest shape makes room
        if (g->pgraphs.front().exec) hipGraphExecDestroy(g->pgraphs.front().exec);
        g->pgraphs.erase(g->pgraphs.begin());
    }
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    enqueue_window_prefix2(g, m, to - from, wcls, desc, g->cap_stream);
    for (uint32_t i = from; i < to; i++)
        enqueue_device_batch2(g, m, ops[i] != 0, batch_class(sizes[i]), i - from, g->cap_stream);
    if (hipStreamEndCapture(g->cap_stream, &graph) != hipSuccess || !graph) return nullptr;
    hipGraphExec_t exec = nullptr;
    const hipError_t r = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (r != hipSuccess) return nullptr;
    g->pgraphs.push_back(gpma::PairEntry{exec, wcls, sig, g->geom_version, m->geom_version});
    return exec;
}

gpma::GraphEntry *get_graph(gpma *g, uint64_t cls, bool del, const BatchDesc *desc, uint32_t *stop,
                            bool transpose) {
    for (auto &e : g->graphs)
        if (e.cls == cls && e.del == del && e.version == g->geom_version) return &e;
    // a batch reads its keys from the buffer a window prefix sorted them into
    if (!g->wukeys) return nullptr;
    gpma::GraphEntry ge{};
    ge.cls = cls;
    ge.del = del;
    ge.version = g->geom_version;
    if (g->fused_direct) {   // no capture: the caller enqueues the batch itself
        g->graphs.push_back(ge);
        return &g->graphs.back();
    }
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    enqueue_device_batch(g, del, cls, desc, stop, transpose, g->cap_stream, &ge);
    if (hipStreamEndCapture(g->cap_stream, &graph) != hipSuccess || !graph) return nullptr;
    hipError_t r = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (r != hipSuccess) return nullptr;
    g->graphs.push_back(ge);
    return &g->graphs.back();
}

void read_fused(gpma *g, hipStream_t s) {
    hipMemcpyAsync(g->fs_h, g->fs, sizeof(FusedState), hipMemcpyDeviceToHost, s);
}

void reset_fused(gpma *g, uint32_t batch, hipStream_t s) {
    // the pinned source is rewritten only after the stream has drained the
    // previous copy (every caller synchronises between resets)
    // batch and halted only: the window generation carries on
    g->reset_h->batch = batch;
    g->reset_h->halted = 0;
    hipMemcpyAsync(g->fs, g->reset_h, sizeof(uint32_t) * 2, hipMemcpyHostToDevice, s);
}

// Complete the stopped batch of handle g: restore its control block and run
// the host-driven levels above the graph's, then the root.
int complete_stopped(gpma *g, bool del, hipStream_t s, gpma_stats *st, bool paired = false) {
    const gpma::GraphEntry *ge = nullptr;
    // a paired window ends every batch at the leaf level with its pending
    // updates in place (the level-0 arrays)
    gpma::GraphEntry pe{};
    if (paired) {
        pe.fin_k = g->kS;
        pe.fin_l = g->leafA;
        pe.fin_st = g->stA;
        pe.fin_n = &g->ctl->lvl[0];
        pe.fin_raw = true;
        ge = &pe;
    }
    // else the entry that ran is any with the batch's class/op; its final
    // arrays depend only on H and the tier limit, identical across classes
    for (auto &e : g->graphs)
        if (!ge && e.del == del && e.version == g->geom_version) { ge = &e; break; }
    if (!ge) return GPMA_EDEVICE;
    hipMemcpyAsync(g->ctl, &g->fs->snap, sizeof(Ctl), hipMemcpyDeviceToDevice, s);
    read_ctl(g, s);
    if (g->ctl_h->err) return GPMA_EINVAL;
    const uint64_t rem = (ge->fin_n == &g->ctl->lvl[0]) ? g->ctl_h->lvl[0] : g->ctl_h->lvl[1];
    if (ge->fin_raw) {
        // gather the leaf level's pending updates (its statistics are in the
        // control block already), then the levels above
        LevelArrays nxt{g->kC, g->leafB, g->stB, ge->fin_n};
        compact_pending(ge->fin_k, ge->fin_l, ge->fin_st, &g->ctl->n_in, g->bcap, nxt.k, nxt.l, nxt.st, nxt.n,
                        g->flags, g->tmp, del, g->lf, nullptr, s);
        return finish_levels(g, del, nxt, rem, 1, g->ctl_h->segs, st, s);
    }
    LevelArrays cur{ge->fin_k, ge->fin_l, ge->fin_st, ge->fin_n};
    return finish_levels(g, del, cur, rem, ge->h_top + 1, g->ctl_h->segs, st, s);
}

int apply_chunk(gpma *g, uint32_t count, const uint8_t *ops, const uint64_t *const *keys, const uint64_t *sizes,
                hipStream_t s, gpma_stats *total, uint32_t *done_out);

}  // namespace

namespace {

// Sum the results of batches [from, to) of handle g (already copied to the
// pinned outs_h) into g->n and *total.
void account(gpma *g, uint32_t from, uint32_t to, gpma_stats *total) {
    for (uint32_t b = from; b < to; b++) {
        const BatchOut &x = g->outs_h[b];
        g->n = (uint64_t)((int64_t)g->n + x.dn);
        g->acc_lookups += x.lookups;
        g->acc_misses += x.misses;
        if (total) {
            total->applied += x.applied;
            total->noops += x.noops;
            total->slots_rewritten += x.rewritten;
        }
    }
}

// Probe kernels: a bounded wait (n sleeps of a single wave) and an empty mark.
__global__ void k_probe_wait(uint32_t n) {
    for (uint32_t i = 0; i < n; i++) __builtin_amdgcn_s_sleep(8);
}
__global__ void k_probe_mark() {}

constexpr size_t kProbeMemo = 16;

// Which library stream runs beside caller stream s: a wait of ~0.4 ms goes
// on s, an empty kernel on the candidate; if the candidate's kernel
// completes while s's wait has not, the two sit on different hardware
// queues.  Once per caller stream (the last kProbeMemo streams are
// remembered); nullptr when neither candidate does, or when the handle was
// created with GPMA_FLAG_FUSED_LIB_STREAMS.
hipStream_t pick_pair_stream(gpma *g, hipStream_t s) {
    if (g->lib_streams) return nullptr;
    for (auto &p : g->probes)
        if (p.first == s) return p.second;
    constexpr uint32_t kProbeSleeps = 2000;
    hipEvent_t e_wait = nullptr, e_mark = nullptr;
    hipStream_t pick = nullptr;
    if (hipEventCreateWithFlags(&e_wait, hipEventDisableTiming) == hipSuccess &&
        hipEventCreateWithFlags(&e_mark, hipEventDisableTiming) == hipSuccess) {
        for (hipStream_t c : {g->side, g->side2}) {
            if (hipStreamSynchronize(s) != hipSuccess || hipStreamSynchronize(c) != hipSuccess) break;
            hipLaunchKernelGGL(k_probe_wait, dim3(1), dim3(kWave), 0, s, kProbeSleeps);
            hipEventRecord(e_wait, s);
            hipLaunchKernelGGL(k_probe_mark, dim3(1), dim3(kWave), 0, c);
            hipEventRecord(e_mark, c);
            if (hipEventSynchronize(e_mark) != hipSuccess) break;
            const hipError_t q = hipEventQuery(e_wait);
            // a not-ready query is no error of the caller's next call
            if (q == hipErrorNotReady) (void)hipGetLastError();
            const bool beside = q == hipErrorNotReady;
            if (hipStreamSynchronize(s) != hipSuccess) break;
            if (beside) {
                pick = c;
                break;
            }
        }
    }
    if (e_wait) hipEventDestroy(e_wait);
    if (e_mark) hipEventDestroy(e_mark);
    if (g->probes.size() >= kProbeMemo) g->probes.erase(g->probes.begin());
    g->probes.emplace_back(s, pick);
    return pick;
}

int apply_chunk(gpma *g, uint32_t count, const uint8_t *ops, const uint64_t *const *keys, const uint64_t *sizes,
                hipStream_t s, gpma_stats *total, uint32_t *done_out) {
    gpma *m = g->mir;
    // the mirror's batch results, for its share of the rewritten slots
    gpma_stats mst{};
    gpma_stats *mtot = total ? &mst : nullptr;
    struct MirrorSum {
        gpma_stats *t, *m;
        ~MirrorSum() {
            if (t) t->mirror_slots_rewritten += m->slots_rewritten;
        }
    } msum{total, &mst};
    // the previous call ended with a synchronisation, so the pinned staging
    // buffers are free to rewrite
    for (uint32_t i = 0; i < count; i++) g->desc_h[i] = BatchDesc{keys[i], sizes[i]};
    // The array and its mirror advance independently, each on its own stream
    // with its own stop flag (the mirror's batches are the transposed keys);
    // a handle that stops is completed on the host and resumes after that
    // batch.  Batches are enqueued in windows: a stop wastes at most the rest
    // of its window, and the window grows while batches complete on the
    // device and shrinks after a stop.
    struct Prog {
        gpma *h;
        hipStream_t st;
        bool transpose;
        uint32_t next;
        bool failed;
    };
    // with a mirror: the array's pipeline on the caller's stream and the
    // mirror's on a library stream found running beside it; failing that,
    // both on library streams, forked from and joined to the caller's (the
    // extra hop costs ~10 % of a slide at R-MAT scale 24; a mirror pipeline
    // on the caller's hardware queue cost the overlap: 2.9e8 -> 2.1e8
    // updates/s at scale 22)
    const hipStream_t pair = m ? pick_pair_stream(g, s) : nullptr;
    const bool lib0 = m && !pair;   // the array's pipeline leaves the caller's stream
    Prog P[2] = {{g, lib0 ? g->side : s, false, 0, false}, {m, m ? (pair ? pair : g->side2) : s, true, 0, false}};
    const int nh = m ? 2 : 1;
    // one launch copies the descriptors and clears both handles' state
    launch_fused_begin(g->fs, g->stop, m ? m->fs : nullptr, m ? m->stop : nullptr, 0, g->desc_hd, g->desc, count, s);
    uint32_t window = 8;
    int err = GPMA_OK;
    uint32_t err_at = count;
    auto busy = [&](int k) { return !P[k].failed && P[k].next < count; };
    while (busy(0) || (nh > 1 && busy(1))) {
        uint32_t end[2] = {0, 0};
        // with a mirror at the same batch: one launch per step for both
        bool paired = false;
        if (nh > 1 && busy(0) && busy(1) && P[0].next == P[1].next) {
            const uint32_t wmax = std::min<uint32_t>(window, kWindowMax);
            uint64_t keys_in = 0;
            uint32_t e2 = P[0].next;
            while (e2 < count && e2 - P[0].next < wmax && (e2 == P[0].next || keys_in + sizes[e2] <= g->bcap)) {
                keys_in += sizes[e2];
                e2++;
            }
            const uint64_t wcls = std::min<uint64_t>(batch_class(keys_in), g->bcap);
            if (pairable_window(g, m, wcls)) {
                hipGraphExec_t pw = get_pair_graph(g, m, wcls, ops, sizes, P[0].next, e2, g->desc);
                if (!pw || hipGraphLaunch(pw, s) != hipSuccess) return GPMA_EDEVICE;
                end[0] = end[1] = e2;
                paired = true;
            }
        }
        if (!paired) {
            if (nh > 1) {
                hipEventRecord(g->ev_fork, s);
                if (lib0) hipStreamWaitEvent(P[0].st, g->ev_fork, 0);
                hipStreamWaitEvent(P[1].st, g->ev_fork, 0);
            }
            // a window: at most `window` batches (kWindowMax when tagged,
            // else 1) whose keys fit the staging buffer; its prefix sorts
            // them together
            for (int k = 0; k < nh; k++) {
                end[k] = P[k].next;
                if (!busy(k)) continue;
                gpma *h = P[k].h;
                const uint32_t wmax = window_tag_bits(h) ? std::min<uint32_t>(window, kWindowMax) : 1;
                uint64_t keys_in = 0;
                uint32_t e2 = P[k].next;
                while (e2 < count && e2 - P[k].next < wmax &&
                       (e2 == P[k].next || keys_in + sizes[e2] <= h->bcap)) {
                    keys_in += sizes[e2];
                    e2++;
                }
                end[k] = e2;
                const uint32_t w = e2 - P[k].next;
                const uint64_t wcls = std::min<uint64_t>(batch_class(keys_in), h->bcap);
                gpma::WindowEntry *we = get_window_graph(h, w, wcls, g->desc, h->stop, P[k].transpose);
                if (!we) return GPMA_EDEVICE;
                if (h->fused_direct) enqueue_window_prefix(h, w, wcls, g->desc, h->stop, P[k].transpose, P[k].st);
                else if (hipGraphLaunch(we->exec, P[k].st) != hipSuccess) return GPMA_EDEVICE;
            }
            // interleave the two streams' batches so both have work queued early
            for (uint32_t j = 0; j < window; j++) {
                for (int k = 0; k < nh; k++) {
                    const uint32_t i = P[k].next + j;
                    if (i >= end[k]) continue;
                    gpma *h = P[k].h;
                    const uint64_t cls = batch_class(sizes[i]);
                    gpma::GraphEntry *ge = get_graph(h, cls, ops[i] != 0, g->desc, h->stop, P[k].transpose);
                    if (!ge) return GPMA_EDEVICE;
                    if (h->fused_direct)
                        enqueue_device_batch(h, ops[i] != 0, cls, g->desc, h->stop, P[k].transpose, P[k].st, ge);
                    else if (hipGraphLaunch(ge->exec, P[k].st) != hipSuccess)
                        return GPMA_EDEVICE;
                }
            }
            if (nh > 1) {
                hipEventRecord(g->ev_join, P[1].st);
                hipStreamWaitEvent(s, g->ev_join, 0);
                if (lib0) {
                    hipEventRecord(g->ev_join2, P[0].st);
                    hipStreamWaitEvent(s, g->ev_join2, 0);
                }
            }
        }
        // state, stop flag and results up to the window's end: one copy per
        // handle (a paired window's finishing kernels write them to the host)
        if (!paired)
            for (int k = 0; k < nh; k++) {
                gpma *h = P[k].h;
                hipMemcpyAsync(h->fblk_h, h->fblk, kFbOuts + end[k] * sizeof(BatchOut), hipMemcpyDeviceToHost, s);
            }
        if (hipStreamSynchronize(s) != hipSuccess) return GPMA_EDEVICE;
        bool stopped = false;
        for (int k = 0; k < nh; k++) {
            if (end[k] == P[k].next) continue;   // idle this round
            gpma *h = P[k].h;
            const uint32_t b = h->fs_h->batch;
            account(h, P[k].next, b, k == 0 ? total : mtot);
            if (!*h->stop_h) {
                P[k].next = end[k];
                continue;
            }
            // stopped at batch b with updates left above the device levels
            stopped = true;
            int e = complete_stopped(h, ops[b] != 0, s, k == 0 ? total : mtot, paired);
            if (e == GPMA_EINVAL) {   // an invalid key: batches before b stand
                P[k].failed = true;
                P[k].next = b;
                err = GPMA_EINVAL;
                err_at = std::min(err_at, b);
                continue;
            }
            if (e) {
                *done_out = b;
                return e;
            }
            if (k == 0 && total) total->noops += h->ctl_h->noops;
            hipMemsetAsync(h->stop, 0, sizeof(uint32_t), s);
            if (hipStreamSynchronize(s) != hipSuccess) return GPMA_EDEVICE;   // frees reset_h
            reset_fused(h, b + 1, s);
            P[k].next = b + 1;
        }
        window = stopped ? std::max<uint32_t>(window / 2, 2) : std::min<uint32_t>(2 * window, 64);
    }
    if (err) {
        // both arrays see the same keys, so both stop at the same batch
        if (nh > 1 && (!P[0].failed || !P[1].failed || P[0].next != P[1].next)) return GPMA_EDEVICE;
        *done_out = err_at;
        return err;
    }
    if (m && m->n != g->n) return GPMA_EDEVICE;
    for (gpma *h : {g, m}) {
        if (!h) continue;
        const uint64_t lk = h->acc_lookups, ms = h->acc_misses;
        h->acc_lookups = h->acc_misses = 0;
        if (h->learned) {
            h->batches_since_fit += count > 0 ? count - 1 : 0;   // locator_after_batch adds one
            int e = locator_after_batch(h, lk, ms, false, s);
            if (e) return e;
        }
    }
    *done_out = count;
    return GPMA_OK;
}

}  // namespace

// ===========================================================================
// C ABI

// Snapshots: a read-only copy of the arrays the analytics read (slots, leaf
// counts, row offsets, degrees; the mirror's too), taken in stream order.
static int snapshot_alloc(gpma *src, gpma *c) {
    c->alloc = src->alloc;
    c->astream = src->astream;
    c->V = src->V; c->lf = src->lf; c->lf_log2 = src->lf_log2;
    c->tau_leaf = src->tau_leaf; c->tau_root = src->tau_root;
    c->rho_leaf = src->rho_leaf; c->rho_root = src->rho_root;
    c->cap = src->cap; c->L = src->L; c->H = src->H; c->n = src->n;
    c->dev = src->dev;
    c->readonly = true;
    int e = GPMA_OK;
    e |= dev_alloc(c, &c->slots, src->cap);
    e |= dev_alloc(c, &c->cnt, src->L);
    e |= dev_alloc(c, &c->row_ptr, (uint64_t)src->V + 1);
    e |= dev_alloc(c, &c->deg, src->V);
    if (!c->ctl) e |= dev_alloc(c, &c->ctl, 1);
    if (!c->small) e |= dev_alloc(c, &c->small, 8);
    if (!c->ctl_h && hipHostMalloc((void **)&c->ctl_h, sizeof(Ctl), 0) != hipSuccess) e = GPMA_ENOMEM;
    if (!c->small_h && hipHostMalloc((void **)&c->small_h, 4 * sizeof(uint32_t), 0) != hipSuccess) e = GPMA_ENOMEM;
    return e;
}

static void snapshot_copy(gpma *src, gpma *c, hipStream_t s) {
    hipMemcpyAsync(c->slots, src->slots, src->cap * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
    hipMemcpyAsync(c->cnt, src->cnt, src->L * sizeof(uint16_t), hipMemcpyDeviceToDevice, s);
    hipMemcpyAsync(c->row_ptr, src->row_ptr, ((uint64_t)src->V + 1) * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
    hipMemcpyAsync(c->deg, src->deg, (uint64_t)src->V * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
    c->n = src->n;
}

static int snapshot_refresh_one(gpma *src, gpma *c, hipStream_t s) {
    if (c->cap != src->cap || c->V != src->V) {
        hipStreamSynchronize(s);
        dev_free(c, c->slots); dev_free(c, c->cnt); dev_free(c, c->row_ptr); dev_free(c, c->deg);
        int e = snapshot_alloc(src, c);
        if (e) return e;
    }
    snapshot_copy(src, c, s);
    return GPMA_OK;
}

extern "C" int gpma_snapshot_refresh(gpma_t *src, gpma_t *snap, hipStream_t s);

extern "C" int gpma_snapshot(gpma_t *src, gpma_t **out, hipStream_t s) {
    if (!out) return GPMA_EINVAL;
    *out = nullptr;
    if (!src || src->readonly) return GPMA_EINVAL;
    set_stream(src, s);
    gpma *c = new (std::nothrow) gpma();
    if (!c) return GPMA_ENOMEM;
    int e = snapshot_alloc(src, c);
    if (!e && src->mir) {
        c->mir = new (std::nothrow) gpma();
        e = c->mir ? snapshot_alloc(src->mir, c->mir) : GPMA_ENOMEM;
    }
    if (e) {
        if (c->mir) { free_all(c->mir); delete c->mir; }
        free_all(c);
        delete c;
        return e;
    }
    snapshot_copy(src, c, s);
    if (src->mir) snapshot_copy(src->mir, c->mir, s);
    *out = c;
    return GPMA_OK;
}

extern "C" int gpma_snapshot_refresh(gpma_t *src, gpma_t *snap, hipStream_t s) {
    if (!src || !snap || src->readonly || !snap->readonly) return GPMA_EINVAL;
    if (!src->mir != !snap->mir) return GPMA_EINVAL;
    set_stream(snap, s);
    int e = snapshot_refresh_one(src, snap, s);
    if (!e && src->mir) e = snapshot_refresh_one(src->mir, snap->mir, s);
    return e;
}

extern "C" uint64_t gpma_device_bytes(const gpma_t *g) {
    if (!g) return 0;
    uint64_t b = g->cap * 8 + g->L * 2 + ((uint64_t)g->V + 1) * 4 + (uint64_t)g->V * 4 + (g->dead ? g->L * 4 : 0);
    if (g->mir) b += gpma_device_bytes(g->mir);
    return b;
}


extern "C" {

void gpma_default_params(gpma_params *p) {
    p->leaf_size = 0;
    p->tau_leaf_pm = 920;
    p->tau_root_pm = 800;
    p->rho_leaf_pm = 80;
    p->rho_root_pm = 400;
    p->flags = 0;
    p->sort_tile_keys = 0;
    p->fused_levels = 1;
    p->lds_tier_bytes = 0;
    p->spmv_form = GPMA_SPMV_AUTO;
}

const char *gpma_strerror(int code) {
    switch (code) {
        case GPMA_OK: return "ok";
        case GPMA_EINVAL: return "invalid argument or key";
        case GPMA_ENOMEM: return "device memory allocation failed";
        case GPMA_EDEVICE: return "HIP call failed";
        default: return "unknown error";
    }
}

int gpma_create(gpma_t **out, uint32_t V, const uint64_t *keys, uint64_t n, const gpma_params *params,
                const gpma_allocator *alloc, hipStream_t s) {
    if (!out) return GPMA_EINVAL;
    *out = nullptr;
    gpma_params p;
    if (params) p = *params; else gpma_default_params(&p);
    if (!params_valid(&p, true)) return GPMA_EINVAL;
    if (V == 0 || V > (1u << 31)) return GPMA_EINVAL;
    if (n && !keys) return GPMA_EINVAL;
    if (alloc && (!alloc->alloc || !alloc->free)) return GPMA_EINVAL;
    const uint64_t tot = n + V;
    if (tot >= kMaxCap) return GPMA_EINVAL;
    if ((p.spmv_form == GPMA_SPMV_BINNED || p.spmv_form == GPMA_SPMV_BINNED_COARSE ||
         p.spmv_form == GPMA_SPMV_BINNED_GATHER) && !pb_supported(V))
        return GPMA_EINVAL;

    gpma *g = new (std::nothrow) gpma();
    if (!g) return GPMA_ENOMEM;
    if (alloc) g->alloc = *alloc;
    g->astream = s;
    g->spmv_form = p.spmv_form;
    g->lib_streams = (p.flags & GPMA_FLAG_FUSED_LIB_STREAMS) != 0;
    g->window_radix = (p.flags & GPMA_FLAG_WINDOW_RADIX) != 0;
    g->V = V;
    g->tau_leaf = p.tau_leaf_pm; g->tau_root = p.tau_root_pm;
    g->rho_leaf = p.rho_leaf_pm; g->rho_root = p.rho_root_pm;
    int dev = 0;
    hipGetDevice(&dev);
    g->dev.max_lds = seg_merge_max_lds();
    hipDeviceGetAttribute(&g->dev.cus, hipDeviceAttributeMultiprocessorCount, dev);
    // a cap on the LDS of the workgroup tier sends smaller segments to the
    // host-driven device tier (same results; tests use it to reach that tier)
    if (p.lds_tier_bytes) g->dev.max_lds = std::min<int>(g->dev.max_lds, (int)std::min<uint32_t>(p.lds_tier_bytes, 1u << 30));

    int e = GPMA_OK;
    uint64_t *in = nullptr, *ba = nullptr, *bb = nullptr, *uq = nullptr;
    uint32_t *fl = nullptr, *tmp = nullptr;
    e |= dev_alloc(g, &g->ctl, 1);
    e |= dev_alloc(g, &g->small, 8);
    if (hipHostMalloc((void **)&g->ctl_h, sizeof(Ctl), 0) != hipSuccess) e = GPMA_ENOMEM;
    if (hipHostMalloc((void **)&g->small_h, 4 * sizeof(uint32_t), 0) != hipSuccess) e = GPMA_ENOMEM;
    e |= dev_alloc(g, &in, tot); e |= dev_alloc(g, &ba, tot); e |= dev_alloc(g, &bb, tot);
    e |= dev_alloc(g, &fl, tot + 1);
    e |= dev_alloc(g, &tmp, std::max(radix_tmp_words(tot), scan_tmp_words(tot + 1)));
    if (e) {
        dev_free(g, in); dev_free(g, ba); dev_free(g, bb); dev_free(g, fl); dev_free(g, tmp);
        free_all(g);
        delete g;
        return GPMA_ENOMEM;
    }
    hipMemsetAsync(g->ctl, 0, sizeof(Ctl), s);
    if (n) {
        hipMemcpyAsync(in, keys, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
        launch_validate(keys, n, V, g->ctl, s);
    }
    launch_append_guards(in + n, V, s);
    const uint64_t *sorted = radix_sort_keys(in, tot, bit_width(V - 1), bit_width(V), V, ba, bb, tmp, s);
    uq = (sorted == ba) ? bb : ba;
    unique_sorted(sorted, tot, uq, &g->ctl->n_in, fl, tmp, s);
    read_ctl(g, s);
    const uint64_t nu = g->ctl_h->n_in;
    auto cleanup = [&]() { dev_free(g, in); dev_free(g, ba); dev_free(g, bb); dev_free(g, fl); dev_free(g, tmp); };
    if (g->ctl_h->err) {
        cleanup();
        free_all(g);
        delete g;
        return GPMA_EINVAL;
    }
    // capacity: the smallest power of two (at least one leaf) whose root bound
    // admits every entry; the leaf length then follows it (O(log N), at least 16)
    uint32_t lf = p.leaf_size;
    uint64_t cap = 16;
    g->lf = 16;
    while (nu > root_hi(g, cap)) cap *= 2;
    if (lf == 0) {
        lf = (uint32_t)std::max<uint64_t>(16, next_pow2(ilog2(cap)));
        while ((uint64_t)g->rho_leaf * lf < 1000) lf *= 2;
        lf = std::min(lf, kMaxLeaf);
    }
    g->lf = lf;
    g->lf_log2 = ilog2(lf);
    cap = lf;
    while (nu > root_hi(g, cap)) cap *= 2;
    if (cap > kMaxCap) {
        cleanup();
        free_all(g);
        delete g;
        return GPMA_EINVAL;
    }
    set_geometry(g, cap);
    g->slots_buf = cap;
    e |= dev_alloc(g, &g->slots, cap);
    e |= dev_alloc(g, &g->piv, g->L);
    e |= dev_alloc(g, &g->cnt, g->L);
    e |= dev_alloc(g, &g->row_ptr, (uint64_t)V + 1);
    e |= dev_alloc(g, &g->deg, V);
    if (p.flags & GPMA_FLAG_LAZY_DELETE) e |= dev_alloc(g, &g->dead, g->L);   // zeroed by the dispatch
    if (e) {
        cleanup();
        free_all(g);
        delete g;
        return GPMA_ENOMEM;
    }
    hipMemsetAsync(g->row_ptr, 0, sizeof(uint32_t), s);
    g->learned = (p.flags & GPMA_FLAG_LEARNED_LOCATOR) != 0;
    g->fused_direct = (p.flags & GPMA_FLAG_FUSED_DIRECT) != 0;
    g->sort_chunks = p.sort_tile_keys ? (int)(p.sort_tile_keys / 256) : 4;
    g->fused_levels = p.fused_levels;
    launch_dispatch(uq, nu, g->slots, g->piv, g->cnt, g->dead, g->row_ptr, 0, g->L, lf, s);
    launch_degrees_from_sorted(uq, nu, V, fl, g->deg, s);
    if (hipStreamSynchronize(s) != hipSuccess) {
        cleanup();
        free_all(g);
        delete g;
        return GPMA_EDEVICE;
    }
    cleanup();
    g->n = nu;
    if (g->learned && locator_fit(g, s)) {
        free_all(g);
        delete g;
        return GPMA_ENOMEM;
    }
    if (p.flags & GPMA_FLAG_MIRROR) {
        gpma_params mp = p;
        mp.flags = p.flags & (GPMA_FLAG_LEARNED_LOCATOR | GPMA_FLAG_FUSED_DIRECT | GPMA_FLAG_LAZY_DELETE |
                              GPMA_FLAG_WINDOW_RADIX);
        mp.leaf_size = g->lf;
        mp.spmv_form = GPMA_SPMV_AUTO;
        uint64_t *tk = nullptr;
        if (n && dev_alloc(g, &tk, n)) {
            free_all(g);
            delete g;
            return GPMA_ENOMEM;
        }
        launch_transpose_keys(keys, n, tk, s);
        int e2 = gpma_create(&g->mir, V, tk, n, &mp, alloc, s);
        dev_free(g, tk);
        if (e2) {
            free_all(g);
            delete g;
            return e2;
        }
    }
    *out = g;
    return GPMA_OK;
}

int gpma_destroy(gpma_t *g) {
    if (!g) return GPMA_OK;
    hipDeviceSynchronize();
    if (g->mir) gpma_destroy(g->mir);
    g->mir = nullptr;
    free_all(g);
    delete g;
    return GPMA_OK;
}

// Reserve, on the array and its mirror, everything a batch of b updates may
// allocate, then apply it to both: an allocation failure returns before
// either changes.
static int apply_with_mirror(gpma_t *g, const uint64_t *keys, uint64_t b, bool del, hipStream_t s,
                             gpma_stats *st) {
    if (!g || g->readonly) return GPMA_EINVAL;
    if (b && (!keys || b >= (1ull << 31))) return GPMA_EINVAL;
    set_stream(g, s);
    int e = GPMA_OK;
    if (b) {
        for (gpma *h : {g, g->mir}) {
            if (!h || e) continue;
            e = ensure_batch(h, b);
            if (!e) e = reserve_update(h, del ? 0 : b, del ? b : 0, 1);
        }
        if (!e && g->mir && b > g->tkeys_cap) {
            dev_free(g, g->tkeys);
            g->tkeys_cap = 0;
            e = dev_alloc(g, &g->tkeys, next_pow2(b));
            if (!e) g->tkeys_cap = next_pow2(b);
        }
    }
    if (!e) e = apply_batch(g, keys, b, del, s, st);
    if (!e && g->mir && b) {
        launch_transpose_keys(keys, b, g->tkeys, s);
        gpma_stats mst;
        e = apply_batch(g->mir, g->tkeys, b, del, s, st ? &mst : nullptr);
        if (!e && st) st->mirror_slots_rewritten = mst.slots_rewritten;
        // both arrays hold the same edge set
        if (!e && g->mir->n != g->n) e = GPMA_EDEVICE;
    }
    release_pool(g);
    if (g->mir) release_pool(g->mir);
    return e;
}

int gpma_insert_batch(gpma_t *g, const uint64_t *keys, uint64_t b, hipStream_t s, gpma_stats *st) {
    return apply_with_mirror(g, keys, b, false, s, st);
}

int gpma_delete_batch(gpma_t *g, const uint64_t *keys, uint64_t b, hipStream_t s, gpma_stats *st) {
    return apply_with_mirror(g, keys, b, true, s, st);
}

gpma_t *gpma_get_mirror(gpma_t *g) { return g ? g->mir : nullptr; }

// Lock-based GPMA insertion (the comparator of Section 6; kernels and the
// algorithm's description in gpma_lock.hip): sort, unique, probe, then rounds
// of locate + one launch per height until every insertion has merged.
// The comparator's merge scratch (one slot per slot) and lock words (two
// per leaf), sized for capacities up to cap_max; reset whenever the
// capacity changed since the last batch or round.
static int lock_state(gpma *g, uint64_t cap_max, hipStream_t s) {
    cap_max = std::max(cap_max, g->cap);
    if (g->lk_buf < cap_max) {
        dev_free(g, g->lk_scratch);
        dev_free(g, g->lk_locks);
        g->lk_buf = 0;
        g->lk_cap = 0;
        if (dev_alloc(g, &g->lk_scratch, cap_max) || dev_alloc(g, &g->lk_locks, 2 * (cap_max >> g->lf_log2))) {
            dev_free(g, g->lk_scratch);
            dev_free(g, g->lk_locks);
            return GPMA_ENOMEM;
        }
        g->lk_buf = cap_max;
    }
    if (g->lk_cap != g->cap) {
        hipMemsetAsync(g->lk_locks, 0, 2 * g->L * sizeof(uint32_t), s);
        g->lk_epoch = 0;
        g->lk_cap = g->cap;
    }
    return GPMA_OK;
}

static int lock_rounds(gpma *g, const uint64_t *keys, uint64_t b, hipStream_t s, gpma_stats *st,
                       uint32_t *rounds_out);

int gpma_lock_insert_batch(gpma_t *g, const uint64_t *keys, uint64_t b, hipStream_t s, gpma_stats *st,
                           uint32_t *rounds_out) {
    if (rounds_out) *rounds_out = 0;
    if (st) {
        memset(st, 0, sizeof(*st));
        st->requested = b;
        st->top_level = -1;
    }
    if (!g || g->readonly || g->mir) return GPMA_EINVAL;
    if (b == 0) return GPMA_OK;
    if (!keys || b >= (1ull << 31)) return GPMA_EINVAL;
    set_stream(g, s);
    uint64_t cmax = g->cap;
    while (g->n + b > root_hi(g, cmax) && cmax <= kMaxCap) cmax *= 2;
    int e = ensure_batch(g, b);
    if (!e) e = reserve_update(g, b, 0, 2);
    if (!e) e = lock_state(g, cmax, s);
    if (e) {
        release_pool(g);
        return e;
    }
    e = lock_rounds(g, keys, b, s, st, rounds_out);
    release_pool(g);
    return e;
}

// The rounds of gpma_lock_insert_batch once its memory is reserved.
static int lock_rounds(gpma *g, const uint64_t *keys, uint64_t b, hipStream_t s, gpma_stats *st,
                       uint32_t *rounds_out) {
    int e = GPMA_OK;
    hipMemsetAsync(g->ctl, 0, sizeof(Ctl), s);
    const uint32_t sb = bit_width(g->V - 1);
    const uint64_t *sorted =
        radix_sort_keys(keys, b, sb, sb, g->V, g->kA, g->kB, g->tmp, s, nullptr, g->ctl, g->sort_chunks);
    uint64_t *ukeys = (sorted == g->kA) ? g->kB : g->kA;
    unique_sorted(sorted, b, ukeys, &g->ctl->n_in, g->flags, g->tmp, s);
    launch_locate(ukeys, &g->ctl->n_in, b, g->piv, g->L, g->ctl, g->leafA, g->stA, s);
    launch_lock_probe(ukeys, g->leafA, g->stA, &g->ctl->n_in, b, g->slots, g->cnt, g->lf_log2, g->ctl, s);
    LevelArrays cur{g->kC, g->leafB, g->stB, &g->ctl->lvl[0]};
    LevelArrays nxt{g->kD, g->leafA, g->stA, &g->ctl->lvl[1]};
    compact_pending(ukeys, g->leafA, g->stA, &g->ctl->n_in, b, cur.k, cur.l, cur.st, cur.n, g->flags, g->tmp, false,
                    0, g->ctl, s);
    read_ctl(g, s);
    if (g->ctl_h->err) return GPMA_EINVAL;
    uint64_t rem = g->ctl_h->lvl[0];
    uint32_t rounds = 0;
    bool resized = false;
    while (rem > 0) {
        // every round merges at least one insertion or doubles the root
        if (rounds > rem + b + 64) return GPMA_EDEVICE;
        e = lock_state(g, 0, s);
        if (e) return e;
        const uint32_t epoch = ++g->lk_epoch;
        launch_locate(cur.k, cur.n, rem, g->piv, g->L, g->ctl, cur.l, cur.st, s);
        for (uint32_t h = 0; h <= g->H; h++) {
            uint64_t lo, hi;
            bounds(g, g->H, h, &lo, &hi);
            launch_lock_try(h, g->H, cur.k, cur.l, cur.st, rem, g->slots, g->piv, g->cnt, g->dead, g->row_ptr, g->deg,
                            g->lk_scratch, g->lk_locks, epoch, g->L, g->lf_log2, hi, g->ctl, s);
        }
        compact_pending(cur.k, cur.l, cur.st, cur.n, rem, nxt.k, nxt.l, nxt.st, nxt.n, g->flags, g->tmp, false, 0,
                        g->ctl, s);
        read_ctl(g, s);
        rounds++;
        rem = (nxt.n == &g->ctl->lvl[0]) ? g->ctl_h->lvl[0] : g->ctl_h->lvl[1];
        std::swap(cur, nxt);
        if (g->ctl_h->root_full) {
            // "double the space of the root segment": re-dispatch everything over 2*cap
            const uint64_t n_now = (uint64_t)((int64_t)g->n + g->ctl_h->dn);
            if (2 * g->cap > kMaxCap) {
                g->n = n_now;
                return GPMA_ENOMEM;
            }
            e = rebuild_root(g, false, nullptr, nullptr, 0, n_now, 2 * g->cap, s);
            if (e) {
                g->n = n_now;
                return e;
            }
            hipMemsetAsync(&g->ctl->root_full, 0, sizeof(uint32_t), s);
            resized = true;
        }
    }
    read_ctl(g, s);
    g->n = (uint64_t)((int64_t)g->n + g->ctl_h->dn);
    if (st) {
        st->applied = g->ctl_h->applied;
        st->noops = b - st->applied;
        st->resized = resized ? 1 : 0;
    }
    if (rounds_out) *rounds_out = rounds;
    return GPMA_OK;
}

int gpma_locate(gpma_t *g, const uint64_t *keys, uint64_t n, uint32_t *leaf_out, hipStream_t s) {
    if (!g || g->readonly || (n && (!keys || !leaf_out)) || n >= (1ull << 31)) return GPMA_EINVAL;
    if (!n) return GPMA_OK;
    set_stream(g, s);
    int e = ensure_batch(g, n);
    if (e) return e;
    hipMemsetAsync(g->ctl, 0, sizeof(Ctl), s);
    launch_validate(keys, n, g->V, g->ctl, s);
    g->small_h[0] = (uint32_t)n;
    hipMemcpyAsync(&g->ctl->n_in, g->small_h, sizeof(uint32_t), hipMemcpyHostToDevice, s);
    do_locate(g, keys, &g->ctl->n_in, n, leaf_out, g->stA, s);
    read_ctl(g, s);
    if (g->ctl_h->err) return GPMA_EINVAL;
    if (g->learned) {
        g->loc_lookups += n;
        g->loc_misses += g->ctl_h->misses;
    }
    return GPMA_OK;
}

int gpma_locator_refit(gpma_t *g, hipStream_t s) {
    if (!g || !g->learned) return GPMA_EINVAL;
    set_stream(g, s);
    return locator_fit(g, s);
}

int gpma_locator_info(const gpma_t *g, uint32_t *eps, uint64_t *lookups, uint64_t *misses, uint64_t *fits) {
    if (!g || !g->learned) return GPMA_EINVAL;
    if (eps) *eps = g->loc_h.valid ? g->loc_h.eps : 0xFFFFFFFFu;
    if (lookups) *lookups = g->loc_lookups;
    if (misses) *misses = g->loc_misses;
    if (fits) *fits = g->loc_fits;
    return GPMA_OK;
}

int gpma_apply_batches(gpma_t *g, uint32_t count, const uint8_t *ops, const uint64_t *const *keys,
                       const uint64_t *sizes, hipStream_t s, gpma_stats *total, uint32_t *completed) {
    if (completed) *completed = 0;
    if (total) {
        memset(total, 0, sizeof(*total));
        total->top_level = -1;
    }
    if (!g || g->readonly || (count && (!ops || !keys || !sizes))) return GPMA_EINVAL;
    uint64_t cmax = 0, sum = 0, sum_ins = 0, sum_del = 0;
    for (uint32_t i = 0; i < count; i++) {
        if (ops[i] > 1 || sizes[i] >= (1ull << 31) || (sizes[i] && !keys[i])) return GPMA_EINVAL;
        cmax = std::max(cmax, batch_class(sizes[i]));
        sum += sizes[i];
        (ops[i] ? sum_del : sum_ins) += sizes[i];
        if (total) total->requested += sizes[i];
    }
    if (count == 0) return GPMA_OK;
    set_stream(g, s);
    // staging for windows of batches sorted together: up to 2^20 keys; then
    // everything the whole sequence may allocate, on both arrays, before any
    // batch runs
    cmax = std::max(cmax, std::min<uint64_t>(1ull << 20, batch_class(sum)));
    int e = GPMA_OK;
    for (gpma *h : {g, g->mir}) {
        if (!h || e) continue;
        e = ensure_batch(h, cmax);
        if (!e) e = ensure_fused(h);
        if (!e) e = reserve_update(h, sum_ins, sum_del, 2);
    }
    uint32_t done = 0;
    for (uint32_t c0 = 0; !e && c0 < count; c0 += kFusedChunk) {
        const uint32_t n = std::min(kFusedChunk, count - c0);
        uint32_t d = 0;
        e = apply_chunk(g, n, ops + c0, keys + c0, sizes + c0, s, total, &d);
        done += d;
    }
    release_pool(g);
    if (g->mir) release_pool(g->mir);
    if (completed) *completed = done;
    return e;
}

int gpma_reserve(gpma_t *g, uint64_t b, hipStream_t s) {
    if (!g || g->readonly || b >= (1ull << 31)) return GPMA_EINVAL;
    set_stream(g, s);
    int e = GPMA_OK;
    for (gpma *h : {g, g->mir}) {
        if (!h || e) continue;
        e = ensure_batch(h, std::max<uint64_t>(b, 1));
        if (!e) e = ensure_fused(h);
        if (!e) e = ensure_dt(h, h->n + b, h->L);
    }
    if (!e && g->mir && b > g->tkeys_cap) {
        dev_free(g, g->tkeys);
        g->tkeys_cap = 0;
        e = dev_alloc(g, &g->tkeys, next_pow2(b));
        if (!e) g->tkeys_cap = next_pow2(b);
    }
    return e;
}

int gpma_fused_pairing(gpma_t *g, hipStream_t s) {
    if (!g || !g->mir) return GPMA_EINVAL;
    if (g->lib_streams) return 0;
    for (auto &p : g->probes)
        if (p.first == s) return p.second ? 1 : 0;
    return GPMA_EINVAL;
}

uint64_t gpma_allocated_bytes(const gpma_t *g) {
    if (!g) return 0;
    return g->held_bytes + (g->mir ? g->mir->held_bytes : 0);
}

uint64_t gpma_num_edges(const gpma_t *g) { return g ? g->n - g->V : 0; }
uint64_t gpma_capacity(const gpma_t *g) { return g ? g->cap : 0; }
uint32_t gpma_leaf_size(const gpma_t *g) { return g ? g->lf : 0; }
uint32_t gpma_num_vertices(const gpma_t *g) { return g ? g->V : 0; }

int gpma_export_slots(gpma_t *g, uint64_t *out, uint64_t max, uint64_t *cap_out, hipStream_t s) {
    if (!g) return GPMA_EINVAL;
    if (cap_out) *cap_out = g->cap;
    if (!out || max < g->cap) return GPMA_EINVAL;
    hipMemcpyAsync(out, g->slots, g->cap * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
    return GPMA_OK;
}

int gpma_export_keys(gpma_t *g, uint64_t *out, uint64_t max, uint64_t *n_out, hipStream_t s) {
    if (!g) return GPMA_EINVAL;
    const uint64_t m = g->n - g->V;
    if (n_out) *n_out = m;
    if (!out || max < m) return GPMA_EINVAL;
    set_stream(g, s);
    uint32_t *fl = nullptr, *tmp = nullptr;
    if (dev_alloc(g, &fl, g->cap + 1) || dev_alloc(g, &tmp, scan_tmp_words(g->cap))) {
        dev_free(g, fl);
        dev_free(g, tmp);
        return GPMA_ENOMEM;
    }
    compact_edges(g->slots, g->cap, out, g->small, fl, tmp, s);
    hipStreamSynchronize(s);
    dev_free(g, fl);
    dev_free(g, tmp);
    return GPMA_OK;
}

int gpma_export_leaf_counts(gpma_t *g, uint16_t *out, uint64_t max, hipStream_t s) {
    if (!g || !out || max < g->L) return GPMA_EINVAL;
    hipMemcpyAsync(out, g->cnt, g->L * sizeof(uint16_t), hipMemcpyDeviceToDevice, s);
    return GPMA_OK;
}

int gpma_export_pivots(gpma_t *g, uint64_t *out, uint64_t max, hipStream_t s) {
    if (!g || !out || !g->piv || max < g->L) return GPMA_EINVAL;
    hipMemcpyAsync(out, g->piv, g->L * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
    return GPMA_OK;
}

int gpma_export_row_offsets(gpma_t *g, uint32_t *out, uint64_t max, hipStream_t s) {
    if (!g || !out || max < (uint64_t)g->V + 1) return GPMA_EINVAL;
    hipMemcpyAsync(out, g->row_ptr, ((uint64_t)g->V + 1) * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
    return GPMA_OK;
}

int gpma_export_degrees(gpma_t *g, uint32_t *out, uint64_t max, hipStream_t s) {
    if (!g || !out || max < g->V) return GPMA_EINVAL;
    hipMemcpyAsync(out, g->deg, (uint64_t)g->V * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
    return GPMA_OK;
}

int gpma_sync(gpma_t *g) {
    (void)g;
    hipDeviceSynchronize();
    return GPMA_OK;
}

namespace {

enum { kSpmvBinned = 0, kSpmvPull = 1, kSpmvPush = 2, kSpmvGather = 3 };

// Destination bins (edges binned once per call, contributions fetched by
// source) when V allows them, else pull over the dst-major mirror if there
// is one, else push; gpma_params.spmv_form picks one (tests compare them;
// validated at create).
int spmv_mode(const gpma *g) {
    switch (g->spmv_form) {
        case GPMA_SPMV_BINNED:
        case GPMA_SPMV_BINNED_COARSE: return kSpmvBinned;
        case GPMA_SPMV_PULL: return kSpmvPull;
        case GPMA_SPMV_PUSH: return kSpmvPush;
        case GPMA_SPMV_BINNED_GATHER: return kSpmvGather;
        default: return pb_supported(g->V) ? kSpmvGather : (g->mir ? kSpmvPull : kSpmvPush);
    }
}

// records for every stored edge, the count matrix and its scan scratch, the
// piece table; grown with 25% headroom so a slowly growing graph does not
// reallocate on every call
int ensure_pb(gpma *g, const PbLayout &L) {
    const uint64_t edges = g->n;   // >= stored edges (guards included)
    if (!g->pb_small && dev_alloc(g, &g->pb_small, 4)) return GPMA_ENOMEM;
    if (g->pb_rec_cap < edges) {
        dev_free(g, g->pb_rec);
        g->pb_rec_cap = 0;
        const uint64_t want = edges + edges / 4 + 1024;
        if (dev_alloc(g, &g->pb_rec, want)) return GPMA_ENOMEM;
        g->pb_rec_cap = want;
    }
    if (L.nc && g->pb_rec2_cap < edges) {
        dev_free(g, g->pb_rec2);
        g->pb_rec2_cap = 0;
        const uint64_t want = edges + edges / 4 + 1024;
        if (dev_alloc(g, &g->pb_rec2, want)) return GPMA_ENOMEM;
        g->pb_rec2_cap = want;
    }
    if (L.nc && g->pb_coffs_words < L.coarse_words) {
        dev_free(g, g->pb_coffs);
        g->pb_coffs_words = 0;
        if (dev_alloc(g, &g->pb_coffs, L.coarse_words)) return GPMA_ENOMEM;
        g->pb_coffs_words = L.coarse_words;
    }
    if (g->pb_offs_words < L.count_words) {
        dev_free(g, g->pb_offs);
        g->pb_offs_words = 0;
        if (dev_alloc(g, &g->pb_offs, L.count_words)) return GPMA_ENOMEM;
        g->pb_offs_words = L.count_words;
    }
    const uint64_t tw = scan_tmp_words(std::max(L.count_words, L.coarse_words));
    if (g->pb_tmp_words < tw) {
        dev_free(g, g->pb_tmp);
        g->pb_tmp_words = 0;
        if (dev_alloc(g, &g->pb_tmp, tw)) return GPMA_ENOMEM;
        g->pb_tmp_words = tw;
    }
    if (g->pb_keys_cap < g->cap) {
        dev_free(g, g->pb_keys);
        g->pb_keys_cap = 0;
        if (dev_alloc(g, &g->pb_keys, g->cap)) return GPMA_ENOMEM;
        g->pb_keys_cap = g->cap;
    }
    if (g->pb_ne_cap < L.W) {
        dev_free(g, g->pb_ne);
        g->pb_ne_cap = 0;
        if (dev_alloc(g, &g->pb_ne, L.W)) return GPMA_ENOMEM;
        g->pb_ne_cap = L.W;
    }
    if (g->pb_pieces_cap < L.max_pieces) {
        dev_free(g, g->pb_pieces);
        g->pb_pieces_cap = 0;
        const uint64_t want = L.max_pieces + L.max_pieces / 4;
        if (dev_alloc(g, &g->pb_pieces, want)) return GPMA_ENOMEM;
        g->pb_pieces_cap = want;
    }
    return GPMA_OK;
}

}  // namespace

int gpma_pagerank(gpma_t *g, const float *init, float *out, uint32_t iters, float damping,
                  hipStream_t s) {
    if (!g || !out || iters == 0 || !(damping > 0.f && damping < 1.f)) return GPMA_EINVAL;
    set_stream(g, s);
    if (!g->pr_contrib) {
        int e = GPMA_OK;
        e |= dev_alloc(g, &g->pr_contrib, g->V);
        e |= dev_alloc(g, &g->pr_y, g->V);
        e |= dev_alloc(g, &g->pr_dang, 1);
        if (e) {
            dev_free(g, g->pr_contrib); dev_free(g, g->pr_y); dev_free(g, g->pr_dang);
            return GPMA_ENOMEM;
        }
    }
    // algorithmic bytes of one SpMV: every stored entry once (8 B), the leaf
    // counts (2 B a leaf), and per vertex the fp32 input and its degree, the
    // fp64 accumulator written and read, and the fp32 output (28 B)
    const double spmv_bytes = 8.0 * (double)g->n + 2.0 * (double)(g->cap >> g->lf_log2) + 28.0 * (double)g->V;
    const int mode = spmv_mode(g);
    PbLayout L;
    if (mode == kSpmvBinned || mode == kSpmvGather) {
        L = pb_layout(g->V, g->cap, g->lf_log2, g->n, g->spmv_form == GPMA_SPMV_BINNED_COARSE);
        if (int e = ensure_pb(g, L)) return e;
        launch_pb_structure(g->slots, L, g->pb_keys, g->pb_ne, g->pb_offs, g->pb_small, g->pb_tmp, g->pb_pieces,
                            g->pb_small + 1, g->pb_coffs, s);
        // the gather form bins the edges once per call (records name their
        // source); every iteration then reads each record once
        if (mode == kSpmvGather)
            launch_pb_bin(g->pb_keys, g->pb_ne, L, g->pb_offs, g->pb_small, nullptr, g->pb_rec, true, s);
    }
    for (uint32_t it = 0; it < iters; it++) {
        const float *x = it == 0 ? init : out;
        launch_pr_prep(x, g->deg, g->V, x == nullptr, g->pr_contrib, g->pr_y, g->pr_dang, s);
        {
            ProfScope ps(g, GPMA_K_SPMV, s);
            if (mode == kSpmvBinned)
                launch_pb_spmv(g->pb_keys, g->pb_ne, L, g->pb_offs, g->pb_small, g->pb_pieces,
                               g->pb_small + 1, g->pb_coffs, g->pr_contrib, g->pb_rec, g->pb_rec2, g->V, g->pr_y, s);
            else if (mode == kSpmvGather)
                launch_pb_gather(L, g->pb_pieces, g->pb_small + 1, g->pr_contrib, g->pb_rec, g->V, g->pr_y, s);
            else if (mode == kSpmvPull)
                launch_pr_pull(g->mir->slots, g->mir->cnt, g->mir->cap, g->mir->lf_log2, g->pr_contrib,
                               g->pr_y, s);
            else
                launch_pr_push(g->slots, g->cnt, g->cap, g->lf_log2, g->pr_contrib, g->pr_y, s);
            ps.done(spmv_bytes);
        }
        launch_pr_combine(g->pr_y, g->pr_dang, g->V, (double)damping, out, s);
    }
    return GPMA_OK;
}

}  // extern "C"

namespace {

// BFS levels (Section 4.2, Algorithm "Breadth-First Search") with the
// caller's scratch: two frontier queues and the row-length scan (V words
// each), the scan's tmp (scan_tmp_words(V)) and 4 counter words (0: the
// frontier count, 1: the next frontier's count, 3: the scan total).
int bfs_run(gpma *g, uint32_t source, int32_t *dist, hipStream_t s, uint32_t *q0, uint32_t *q1, uint32_t *off,
            uint32_t *tmp, uint32_t *counters) {
    uint32_t *cur = q0, *nxt = q1;
    launch_bfs_init(dist, g->V, source, cur, counters, s);
    uint32_t nfront = 1;
    // Direction choice (with a mirror): expand top-down while the frontier's
    // rows are a small part of the rows not yet expanded; go bottom-up over
    // the in-edges when they exceed 1/14 of them or the frontier holds 1/64
    // of the vertices (the usual direction-optimising rule).
    uint64_t unexplored = g->n;
    for (int32_t level = 0; nfront > 0; level++) {
        if (hipMemsetAsync(counters + 1, 0, sizeof(uint32_t), s) != hipSuccess) return GPMA_EDEVICE;
        bool bottom_up = g->mir && (uint64_t)nfront * 64 >= g->V;
        if (!bottom_up) {
            // rows of the frontier end to end: lengths and their scan
            launch_bfs_row_len(g->row_ptr, cur, nfront, off, s);
            scan_u32(off, off, nfront, counters + 3, tmp, s);
            if (g->mir) {
                hipMemcpyAsync(g->small_h + 1, counters + 3, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
                if (hipStreamSynchronize(s) != hipSuccess) return GPMA_EDEVICE;
                const uint64_t mf = g->small_h[1];
                bottom_up = mf * 14 > unexplored;
                if (!bottom_up) unexplored = unexplored > mf ? unexplored - mf : 0;
            }
        }
        {
            ProfScope ps(g, GPMA_K_BFS, s);
            if (bottom_up) {
                launch_bfs_bottom_up(g->mir->slots, g->mir->row_ptr, g->V, level, dist, nxt, counters + 1, s);
            } else {
                launch_bfs_expand(g->slots, g->row_ptr, cur, off, nfront, counters + 3, g->cap, level, dist, nxt,
                                  counters + 1, s);
            }
        }
        hipMemcpyAsync(g->small_h, counters + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
        if (hipStreamSynchronize(s) != hipSuccess) return GPMA_EDEVICE;
        nfront = g->small_h[0];
        std::swap(cur, nxt);
    }
    return GPMA_OK;
}

// ---------------------------------------------------------------------------
// Scratch of gpma_bfs_noalloc: one file-scope device array per GPU (each GPU
// the library runs on holds its own copy until the process ends).  Host code
// never passes `scratch` itself to a kernel (on the host it only names the
// symbol): the device address comes from hipGetSymbolAddress, taken once per
// device with that device current, and every use goes through it.
constexpr uint32_t kNoallocMaxV = 1u << 22;
constexpr uint64_t kScrCounters = 64;       // counter words (256 B)
constexpr uint64_t kScrScanTmp = 4096;      // >= scan_tmp_words(kNoallocMaxV)
constexpr uint64_t kScrWords = kScrCounters + 3ull * kNoallocMaxV + kScrScanTmp;
constexpr int kScrMaxDevices = 64;

static __device__ __align__(256) uint32_t scratch[kScrWords];

std::mutex g_scr_mu;
uint32_t *g_scr_ptr[kScrMaxDevices] = {};

// The current device's address of `scratch` (nullptr if it cannot be had).
uint32_t *noalloc_scratch() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScrMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scr_mu);
    if (!g_scr_ptr[dev]) {
        if (scan_tmp_words(kNoallocMaxV) > kScrScanTmp) return nullptr;
        void *p = nullptr;
        const hipError_t r = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (r != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scr_ptr[dev] = (uint32_t *)p;
    }
    return g_scr_ptr[dev];
}

}  // namespace

extern "C" {

int gpma_bfs(gpma_t *g, uint32_t source, int32_t *dist, hipStream_t s) {
    if (!g || !dist || source >= g->V) return GPMA_EINVAL;
    set_stream(g, s);
    if (!g->bfs_q0) {
        int e = GPMA_OK;
        e |= dev_alloc(g, &g->bfs_q0, g->V);
        e |= dev_alloc(g, &g->bfs_q1, g->V);
        e |= dev_alloc(g, &g->bfs_off, g->V);
        e |= dev_alloc(g, &g->bfs_tmp, scan_tmp_words(g->V));
        if (e) {
            dev_free(g, g->bfs_q0); dev_free(g, g->bfs_q1); dev_free(g, g->bfs_off); dev_free(g, g->bfs_tmp);
            return GPMA_ENOMEM;
        }
    }
    return bfs_run(g, source, dist, s, g->bfs_q0, g->bfs_q1, g->bfs_off, g->bfs_tmp, g->small);
}

int gpma_bfs_noalloc(gpma_t *g, uint32_t source, int32_t *dist, hipStream_t s) {
    if (!g || !dist || source >= g->V) return GPMA_EINVAL;
    if (g->V > kNoallocMaxV) return GPMA_EINVAL;
    uint32_t *scr = noalloc_scratch();
    if (!scr) return GPMA_EDEVICE;
    uint32_t *q0 = scr + kScrCounters, *q1 = q0 + kNoallocMaxV, *off = q1 + kNoallocMaxV;
    uint32_t *tmp = off + kNoallocMaxV;
    return bfs_run(g, source, dist, s, q0, q1, off, tmp, scr);
}

int gpma_cc(gpma_t *g, uint32_t *label, hipStream_t s) {
    if (!g || !label) return GPMA_EINVAL;
    set_stream(g, s);
    launch_cc_init(label, g->V, s);
    if (g->mir && g->V >= 4096) {
        // sample one out- and one in-neighbour per vertex, find the largest
        // component from 1024 sampled labels, then sweep both arrays once,
        // skipping the rows of that component (an edge is skipped on both
        // sides only when both its ends are already in it)
        launch_cc_sample(g->slots, g->row_ptr, g->V, g->lf, label, s);
        launch_cc_sample(g->mir->slots, g->mir->row_ptr, g->V, g->lf, label, s);
        launch_cc_compress(label, g->V, s);
        if (!g->cc_pick && dev_alloc(g, &g->cc_pick, 1024)) return GPMA_ENOMEM;
        std::vector<uint32_t> smp(1024);
        launch_cc_pick(label, g->V / 1024, 1024, g->cc_pick, s);
        hipMemcpyAsync(smp.data(), g->cc_pick, 1024 * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
        hipStreamSynchronize(s);
        std::sort(smp.begin(), smp.end());
        uint32_t c = smp[0], best = 0;
        for (size_t i = 0; i < smp.size();) {
            size_t j = i;
            while (j < smp.size() && smp[j] == smp[i]) j++;
            if (j - i > best) { best = (uint32_t)(j - i); c = smp[i]; }
            i = j;
        }
        {
            // one sweep of each array: every union is applied (cc_union)
            ProfScope ps(g, GPMA_K_CC, s);
            launch_cc_hook_skip(g->slots, g->cap, label, c, s);
            launch_cc_hook_skip(g->mir->slots, g->mir->cap, label, c, s);
            ps.done(16.0 * (double)g->n + 8.0 * (double)g->V);
        }
        launch_cc_compress(label, g->V, s);
        return GPMA_OK;
    }
    {
        ProfScope ps(g, GPMA_K_CC, s);
        launch_cc_hook(g->slots, g->cap, label, s);
        ps.done(8.0 * (double)g->n + 8.0 * (double)g->V);
    }
    launch_cc_compress(label, g->V, s);
    return GPMA_OK;
}

int gpma_profile_enable(gpma_t *g, int enable) {
    if (!g) return GPMA_EINVAL;
    g->prof_on = enable ? 1 : 0;
    if (g->mir) g->mir->prof_on = g->prof_on;
    return GPMA_OK;
}

int gpma_profile_reset(gpma_t *g) {
    if (!g) return GPMA_EINVAL;
    if (g->mir) gpma_profile_reset(g->mir);
    prof_collect(g);
    for (int k = 0; k < GPMA_K_COUNT; k++) {
        g->prof_ms[k] = 0;
        g->prof_bytes[k] = 0;
        g->prof_n[k] = 0;
    }
    return GPMA_OK;
}

int gpma_profile_read(gpma_t *g, int kernel, double *ms, uint64_t *launches, double *bytes) {
    if (!g || kernel < 0 || kernel >= GPMA_K_COUNT) return GPMA_EINVAL;
    prof_collect(g);
    double m = g->prof_ms[kernel], by = g->prof_bytes[kernel];
    uint64_t n = g->prof_n[kernel];
    if (g->mir) {   // the mirror's update kernels count with the handle's
        prof_collect(g->mir);
        m += g->mir->prof_ms[kernel];
        by += g->mir->prof_bytes[kernel];
        n += g->mir->prof_n[kernel];
    }
    if (ms) *ms = m;
    if (launches) *launches = n;
    if (bytes) *bytes = by;
    return GPMA_OK;
}

}  // extern "C"
