/*
 * gpma_oracle.c -- CPU oracle for the GPMA+ dynamic-graph hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * entry point and the CPU-baseline leg of the benchmark can check the GPU
 * library against a plain, sequential, obviously correct implementation.
 * The product path never loads or calls it, and it shares no code with the
 * GPU library (not even the threshold tables).
 *
 * Source: Sha, Li, He, Tan, "Accelerating Dynamic Graph Analytics on GPUs"
 * (PVLDB 11(1), 2017; arXiv 1709.05061).  Citations below name the section,
 * algorithm, figure or table of that paper.
 *
 * What is computed:
 *   - a packed memory array (PMA, Section 4.1 "Background of PMA"): a sorted
 *     array of 64-bit keys with gaps, cut into leaf segments of `lf` slots,
 *     with an implicit binary tree of segments over the leaves;
 *   - the batched, level-by-level GPMA+ update (Section 5.2, Algorithm
 *     "GPMA+ Segment-Oriented Insertion") and its dual for deletions, run
 *     sequentially, one segment after the other, in ascending segment order
 *     inside a level (segments of one level are disjoint, so the order does
 *     not change the result);
 *   - CSR on the PMA (Section 4.2, "CSR as a case study"): one guard entry per
 *     vertex u, key u<<32 | 0xFFFFFFFF, sorting after every edge of row u;
 *   - the three analytics of Section 6.1 ("Applications") on the plain edge
 *     set: PageRank in fp64, BFS hop distances, connected components.
 *
 * Readings where the paper is silent (the same readings the GPU library
 * implements, each written out independently there):
 *   - empty slot = all-ones key (key 0 is the real edge (0,0));
 *   - density bounds interpolate linearly in the height between the leaf and
 *     root values of the figure "PMA insertion example"; an insert into a
 *     segment passes iff (n_s+|U_s|)/cap < tau, a delete iff
 *     (n_s-|D_s|)/cap > rho;
 *   - "re-dispatch entries evenly": leaf j of a segment of P leaves holding N
 *     entries receives floor((j+1)N/P) - floor(jN/P) of them, packed at the
 *     front of the leaf in key order;
 *   - an update's leaf is the leaf holding the greatest stored key <= it
 *     (leaf 0 when there is none);
 *   - set semantics: duplicates inside a batch collapse, inserting a stored
 *     key and deleting an absent key are no-ops, removed before the levels;
 *   - the root is tried like any other segment; when it fails, an insert
 *     doubles the capacity until the bound holds and a delete halves it while
 *     the lower bound fails (never below one leaf, never above the upper
 *     bound of the halved array); every entry is then re-dispatched;
 *   - edge mode takes 1 <= V <= 2^31 (the V guards must fit the GPU
 *     library's 2^31-slot array); raw-key mode (V = 0) stores any key but
 *     the empty one, and lazy deletion, which takes bit 63 of a key for its
 *     mark, is refused there.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EMPTY UINT64_MAX
#define ORC_GUARD_DST 0xFFFFFFFFull
/* lazy deletion (Section 6, the GPMA/GPMA+ setup of the experiments): a
 * deleted entry stays in its slot, marked; lazy mode needs src < 2^31 for
 * every key, so bit 63 is free for the mark and the masked key keeps the
 * array order.  Outside lazy mode bit 63 is an ordinary key bit. */
#define ORC_TOMB (1ull << 63)
#define ORC_MAX_V (1u << 31)

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2 };

typedef struct {
    uint32_t V;    /* vertices; 0 selects raw-key mode (no guards, no key checks) */
    uint32_t lf;   /* leaf segment length in slots */
    uint32_t tau_leaf, tau_root, rho_leaf, rho_root; /* per mille */
    uint64_t cap;  /* slots */
    uint64_t n;    /* stored entries, guards included */
    uint64_t *slots;
    /* merge log of the last batch: (level, segment, live entries of the
       segment before the merge, updates merged into it); a root rebuild is
       logged as level -1 with the new capacity in place of the segment */
    uint64_t log_len, log_cap;
    int32_t *log_level;
    uint64_t *log_seg, *log_ns, *log_k;
    uint64_t applied, noops;
    int lazy;      /* deletions mark entries instead of merging */
} orc_pma;

/* ------------------------------------------------------------------------ */
/* small helpers                                                            */

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* sort and drop repeats; returns the new length */
static uint64_t sort_unique(uint64_t *a, uint64_t n)
{
    if (n == 0) return 0;
    qsort(a, n, sizeof(uint64_t), cmp_u64);
    uint64_t m = 1;
    for (uint64_t i = 1; i < n; i++)
        if (a[i] != a[m - 1]) a[m++] = a[i];
    return m;
}

/* number of elements of sorted a[0..n) that are < k */
static uint64_t count_below(const uint64_t *a, uint64_t n, uint64_t k)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < k) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static int contains(const uint64_t *a, uint64_t n, uint64_t k)
{
    uint64_t i = count_below(a, n, k);
    return i < n && a[i] == k;
}

static uint32_t log2_u64(uint64_t x)
{
    uint32_t r = 0;
    while (x > 1) { x >>= 1; r++; }
    return r;
}

static int is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

/* an occupied slot that holds a live key (in lazy mode a marked entry is
 * free space); mark_free() is the key with the mark cleared */
static int is_live(const orc_pma *p, uint64_t k)
{
    return k != ORC_EMPTY && !(p->lazy && (k & ORC_TOMB));
}
static uint64_t mark_free(const orc_pma *p, uint64_t k)
{
    return p->lazy ? (k & ~ORC_TOMB) : k;
}

/* ------------------------------------------------------------------------ */
/* density bounds (Section 4.1, figure "PMA insertion example")             */

/* Bounds of a segment at height h in a tree of height H.  cap_h = lf*2^h.
 * rho_h, tau_h run linearly from the leaf values (h=0) to the root values
 * (h=H); a tree of height 0 is a single leaf that is also the root, and takes
 * the root values.  Integer forms:
 *   max_h = the largest m with m < tau_h*cap_h   (insert bound)
 *   min_h = the smallest m with m > rho_h*cap_h  (delete bound)          */
static void orc_bounds(const orc_pma *p, uint32_t H, uint32_t h,
                       uint64_t *mn, uint64_t *mx)
{
    uint64_t cap_h = (uint64_t)p->lf << h;
    uint64_t den, rnum, tnum;
    if (H == 0) {
        den = 1000;
        rnum = (uint64_t)p->rho_root * cap_h;
        tnum = (uint64_t)p->tau_root * cap_h;
    } else {
        den = 1000ull * H;
        rnum = ((uint64_t)p->rho_leaf * (H - h) + (uint64_t)p->rho_root * h) * cap_h;
        tnum = ((uint64_t)p->tau_leaf * (H - h) + (uint64_t)p->tau_root * h) * cap_h;
    }
    *mn = rnum / den + 1;
    *mx = (tnum + den - 1) / den - 1;
}

static uint64_t root_max(const orc_pma *p, uint64_t cap)
{
    uint64_t mn, mx;
    uint32_t H = log2_u64(cap / p->lf);
    orc_bounds(p, H, H, &mn, &mx);
    return mx;
}

static uint64_t root_min(const orc_pma *p, uint64_t cap)
{
    uint64_t mn, mx;
    uint32_t H = log2_u64(cap / p->lf);
    orc_bounds(p, H, H, &mn, &mx);
    return mn;
}

/* exported for the threshold tests: fills mn[0..H], mx[0..H] */
int orc_level_bounds(uint32_t lf, uint32_t tau_leaf, uint32_t tau_root,
                     uint32_t rho_leaf, uint32_t rho_root, uint32_t H,
                     uint64_t *mn, uint64_t *mx)
{
    orc_pma p;
    memset(&p, 0, sizeof p);
    p.lf = lf; p.tau_leaf = tau_leaf; p.tau_root = tau_root;
    p.rho_leaf = rho_leaf; p.rho_root = rho_root;
    for (uint32_t h = 0; h <= H; h++) orc_bounds(&p, H, h, &mn[h], &mx[h]);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* even re-dispatch of a segment's entries (Section 4.1, Example 1; the step
 * after Merge in Algorithm GPMA+)                                           */

static void dispatch(uint64_t *slots, uint64_t base, uint32_t lf, uint64_t P,
                     const uint64_t *M, uint64_t N)
{
    for (uint64_t j = 0; j < P; j++) {
        uint64_t a = (uint64_t)(((unsigned __int128)j * N) / P);
        uint64_t b = (uint64_t)(((unsigned __int128)(j + 1) * N) / P);
        for (uint64_t o = 0; o < lf; o++)
            slots[base + j * lf + o] = (o < b - a) ? M[a + o] : ORC_EMPTY;
    }
}

/* the live entries of slots [base, base+len) in array order (a merge drops
 * the marks of lazily deleted entries: their slots are recycled) */
static uint64_t gather(const orc_pma *p, uint64_t base, uint64_t len, uint64_t *out)
{
    uint64_t m = 0;
    for (uint64_t i = 0; i < len; i++)
        if (is_live(p, p->slots[base + i])) out[m++] = p->slots[base + i];
    return m;
}

/* Merge(s, U_s): sorted union of two disjoint sorted lists */
static uint64_t merge_union(const uint64_t *a, uint64_t na, const uint64_t *b,
                            uint64_t nb, uint64_t *out)
{
    uint64_t i = 0, j = 0, m = 0;
    while (i < na || j < nb) {
        if (j >= nb || (i < na && a[i] < b[j])) out[m++] = a[i++];
        else out[m++] = b[j++];
    }
    return m;
}

/* the dual: a with every element of b removed */
static uint64_t merge_minus(const uint64_t *a, uint64_t na, const uint64_t *b,
                            uint64_t nb, uint64_t *out)
{
    uint64_t m = 0;
    for (uint64_t i = 0; i < na; i++)
        if (!contains(b, nb, a[i])) out[m++] = a[i];
    return m;
}

static void log_push(orc_pma *p, int32_t level, uint64_t seg, uint64_t ns, uint64_t k)
{
    if (p->log_len == p->log_cap) {
        uint64_t nc = p->log_cap ? 2 * p->log_cap : 64;
        p->log_level = (int32_t *)realloc(p->log_level, nc * sizeof(int32_t));
        p->log_seg = (uint64_t *)realloc(p->log_seg, nc * sizeof(uint64_t));
        p->log_ns = (uint64_t *)realloc(p->log_ns, nc * sizeof(uint64_t));
        p->log_k = (uint64_t *)realloc(p->log_k, nc * sizeof(uint64_t));
        p->log_cap = nc;
    }
    p->log_level[p->log_len] = level;
    p->log_seg[p->log_len] = seg;
    p->log_ns[p->log_len] = ns;
    p->log_k[p->log_len] = k;
    p->log_len++;
}

/* ------------------------------------------------------------------------ */
/* creation                                                                 */

static int params_ok(uint32_t lf, uint32_t tau_leaf, uint32_t tau_root,
                     uint32_t rho_leaf, uint32_t rho_root)
{
    if (!is_pow2(lf) || lf < 4) return 0;
    if (!(rho_leaf > 0 && rho_leaf <= rho_root && rho_root < tau_root &&
          tau_root <= tau_leaf && tau_leaf < 1000))
        return 0;
    if (2 * rho_root > tau_root) return 0;
    return 1;
}

static int key_ok(uint32_t V, uint64_t k)
{
    return (k >> 32) < V && (k & 0xFFFFFFFFull) < V;
}

/* Build a PMA holding the set of `keys` (and, in edge mode, one guard per
 * vertex).  The capacity is the smallest lf*2^k whose root upper bound
 * admits every entry; the entries are dispatched evenly over all leaves. */
orc_pma *orc_create(uint32_t V, const uint64_t *keys, uint64_t n,
                    uint32_t lf, uint32_t tau_leaf, uint32_t tau_root,
                    uint32_t rho_leaf, uint32_t rho_root, int *err)
{
    *err = ORC_EINVAL;
    if (!params_ok(lf, tau_leaf, tau_root, rho_leaf, rho_root)) return NULL;
    if (V) {
        /* the GPU library's domain: V guards must fit a 2^31-slot array */
        if (V > ORC_MAX_V) return NULL;
        for (uint64_t i = 0; i < n; i++)
            if (!key_ok(V, keys[i])) return NULL;
    }
    *err = ORC_ENOMEM;
    orc_pma *p = (orc_pma *)calloc(1, sizeof(orc_pma));
    if (!p) return NULL;
    p->V = V; p->lf = lf;
    p->tau_leaf = tau_leaf; p->tau_root = tau_root;
    p->rho_leaf = rho_leaf; p->rho_root = rho_root;

    uint64_t tot = n + V;
    uint64_t *all = (uint64_t *)malloc((tot ? tot : 1) * sizeof(uint64_t));
    if (!all) { free(p); return NULL; }
    memcpy(all, keys, n * sizeof(uint64_t));
    for (uint32_t u = 0; u < V; u++) all[n + u] = ((uint64_t)u << 32) | ORC_GUARD_DST;
    tot = sort_unique(all, tot);

    uint64_t cap = lf;
    while (tot > root_max(p, cap)) cap *= 2;
    p->cap = cap;
    p->n = tot;
    p->slots = (uint64_t *)malloc(cap * sizeof(uint64_t));
    if (!p->slots) { free(all); free(p); return NULL; }
    dispatch(p->slots, 0, lf, cap / lf, all, tot);
    free(all);
    *err = ORC_OK;
    return p;
}

/* Adopt an explicit slot image (raw-key mode), e.g. a worked example. */
orc_pma *orc_from_slots(const uint64_t *slots, uint64_t cap, uint32_t lf,
                        uint32_t tau_leaf, uint32_t tau_root,
                        uint32_t rho_leaf, uint32_t rho_root, int *err)
{
    *err = ORC_EINVAL;
    if (!params_ok(lf, tau_leaf, tau_root, rho_leaf, rho_root)) return NULL;
    if (!is_pow2(cap) || cap < lf) return NULL;
    uint64_t prev = 0, n = 0;
    for (uint64_t i = 0; i < cap; i++) {
        if (slots[i] == ORC_EMPTY) continue;
        if (n && slots[i] <= prev) return NULL;   /* keys must ascend */
        prev = slots[i]; n++;
    }
    *err = ORC_ENOMEM;
    orc_pma *p = (orc_pma *)calloc(1, sizeof(orc_pma));
    if (!p) return NULL;
    p->lf = lf; p->tau_leaf = tau_leaf; p->tau_root = tau_root;
    p->rho_leaf = rho_leaf; p->rho_root = rho_root;
    p->cap = cap; p->n = n;
    p->slots = (uint64_t *)malloc(cap * sizeof(uint64_t));
    if (!p->slots) { free(p); return NULL; }
    memcpy(p->slots, slots, cap * sizeof(uint64_t));
    *err = ORC_OK;
    return p;
}

void orc_free(orc_pma *p)
{
    if (!p) return;
    free(p->slots); free(p->log_level); free(p->log_seg);
    free(p->log_ns); free(p->log_k); free(p);
}

uint64_t orc_capacity(const orc_pma *p) { return p->cap; }
uint64_t orc_size(const orc_pma *p) { return p->n; }
uint32_t orc_leaf_size(const orc_pma *p) { return p->lf; }
const uint64_t *orc_slots(const orc_pma *p) { return p->slots; }
uint64_t orc_log_len(const orc_pma *p) { return p->log_len; }
const int32_t *orc_log_levels(const orc_pma *p) { return p->log_level; }
const uint64_t *orc_log_segs(const orc_pma *p) { return p->log_seg; }
const uint64_t *orc_log_counts(const orc_pma *p) { return p->log_ns; }
const uint64_t *orc_log_updates(const orc_pma *p) { return p->log_k; }
uint64_t orc_last_applied(const orc_pma *p) { return p->applied; }
uint64_t orc_last_noops(const orc_pma *p) { return p->noops; }
/* Lazy mode takes bit 63 of a key for the mark, so it refuses an array
 * that may hold keys with that bit set: raw-key mode (V = 0) or V > 2^31. */
int orc_set_lazy(orc_pma *p, int lazy)
{
    if (lazy && (p->V == 0 || p->V > ORC_MAX_V)) return ORC_EINVAL;
    p->lazy = lazy ? 1 : 0;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* the batched update (Section 5.2, Algorithm GPMA+ Segment-Oriented
 * Insertion; deletions are its dual, Section 4.1)                          */

/* TryInsert+ / TryDelete+ on segment s at height h with the updates u[0..k).
 * Returns 1 when the segment passed its bound and now holds the merge. */
static int try_segment(orc_pma *p, uint32_t H, uint32_t h, uint64_t s,
                       const uint64_t *u, uint64_t k, int del,
                       uint64_t *bufE, uint64_t *bufM)
{
    uint64_t cap_h = (uint64_t)p->lf << h;
    uint64_t base = s * cap_h;
    uint64_t mn, mx;
    orc_bounds(p, H, h, &mn, &mx);

    /* CountSegment: live entries (marked ones are free space) */
    uint64_t ns = 0;
    for (uint64_t i = 0; i < cap_h; i++)
        if (is_live(p, p->slots[base + i])) ns++;

    if (!del) {
        if (ns + k > mx) return 0;
    } else {
        if (ns < k + mn) return 0;   /* ns - k < mn */
    }
    uint64_t ne = gather(p, base, cap_h, bufE);
    uint64_t N = del ? merge_minus(bufE, ne, u, k, bufM)
                     : merge_union(bufE, ne, u, k, bufM);
    dispatch(p->slots, base, p->lf, (uint64_t)1 << h, bufM, N);
    log_push(p, (int32_t)h, s, ns, k);
    p->n = p->n - ne + N;
    return 1;
}

static int apply_batch(orc_pma *p, const uint64_t *keys, uint64_t b, int del)
{
    p->log_len = 0;
    p->applied = 0;
    p->noops = 0;
    if (p->V)
        for (uint64_t i = 0; i < b; i++)
            if (!key_ok(p->V, keys[i])) return ORC_EINVAL;
    if (b == 0) return ORC_OK;

    /* Sort(U), duplicates collapse */
    uint64_t *U = (uint64_t *)malloc(b * sizeof(uint64_t));
    memcpy(U, keys, b * sizeof(uint64_t));
    uint64_t nu = sort_unique(U, b);

    /* the current content, in order: every occupied slot (masked key, leaf,
       position) and the live keys */
    uint64_t occ = 0;
    for (uint64_t i = 0; i < p->cap; i++)
        if (p->slots[i] != ORC_EMPTY) occ++;
    uint64_t *ok = (uint64_t *)malloc((occ ? occ : 1) * sizeof(uint64_t));
    uint64_t *el = (uint64_t *)malloc((occ ? occ : 1) * sizeof(uint64_t));
    uint64_t *ep = (uint64_t *)malloc((occ ? occ : 1) * sizeof(uint64_t));
    uint64_t *ek = (uint64_t *)malloc((p->n ? p->n : 1) * sizeof(uint64_t));
    uint64_t no = 0, ne = 0;
    for (uint64_t i = 0; i < p->cap; i++) {
        const uint64_t k = p->slots[i];
        if (k == ORC_EMPTY) continue;
        ok[no] = mark_free(p, k); el[no] = i / p->lf; ep[no] = i; no++;
        if (is_live(p, k)) ek[ne++] = k;
    }

    /* drop no-ops: inserting a live key, deleting a key that is not live */
    uint64_t r = 0;
    for (uint64_t i = 0; i < nu; i++) {
        int present = contains(ek, ne, U[i]);
        if (present == !del) p->noops++;
        else U[r++] = U[i];
    }
    p->noops += b - nu;   /* in-batch repeats are no-ops too */

    if (del && p->lazy) {
        /* lazy deletion: mark each entry in place, no density maintenance */
        for (uint64_t i = 0; i < r; i++) {
            uint64_t c = count_below(ok, no, U[i]);
            p->slots[ep[c]] |= ORC_TOMB;
        }
        p->n -= r;
        p->applied = r;
        free(ok); free(el); free(ep); free(ek); free(U);
        return ORC_OK;
    }

    /* BinarySearchLeafSegments: leaf of the greatest occupied key <= u (a
       marked entry still orders the array) */
    uint64_t *leaf = (uint64_t *)malloc((r ? r : 1) * sizeof(uint64_t));
    for (uint64_t i = 0; i < r; i++) {
        uint64_t c = count_below(ok, no, U[i]);           /* occupied keys < u */
        if (c < no && ok[c] == U[i]) leaf[i] = el[c];      /* u itself */
        else leaf[i] = c ? el[c - 1] : 0;
    }
    free(el); free(ok); free(ep);

    uint64_t *bufE = (uint64_t *)malloc((p->cap + r + 1) * sizeof(uint64_t));
    uint64_t *bufM = (uint64_t *)malloc((p->cap + r + 1) * sizeof(uint64_t));
    uint8_t *done = (uint8_t *)calloc(r ? r : 1, 1);
    uint32_t H = log2_u64(p->cap / p->lf);
    uint64_t total = r;

    /* levels, bottom-up: group the remaining updates by segment, try every
       segment, keep the updates of the failed ones for the parent level */
    for (uint32_t h = 0; h <= H && r > 0; h++) {
        uint64_t i = 0;
        while (i < r) {
            uint64_t s = leaf[i] >> h, j = i;
            while (j < r && (leaf[j] >> h) == s) j++;
            if (try_segment(p, H, h, s, U + i, j - i, del, bufE, bufM))
                memset(done + i, 1, j - i);
            i = j;
        }
        uint64_t w = 0;
        for (uint64_t t = 0; t < r; t++)
            if (!done[t]) { U[w] = U[t]; leaf[w] = leaf[t]; w++; }
        memset(done, 0, r);
        r = w;
    }
    free(done);

    if (r > 0) {
        /* the root failed: resize, then re-dispatch everything */
        /* p->n already counts the merges made at lower levels of this batch */
        uint64_t ncap = p->cap;
        if (!del) {
            while (p->n + r > root_max(p, ncap)) ncap *= 2;
        } else {
            uint64_t left = p->n - r;
            while (ncap > p->lf && left < root_min(p, ncap) &&
                   left <= root_max(p, ncap / 2))
                ncap /= 2;
        }
        uint64_t nall = gather(p, 0, p->cap, bufE);
        uint64_t *M = (uint64_t *)malloc((nall + r + 1) * sizeof(uint64_t));
        uint64_t N = del ? merge_minus(bufE, nall, U, r, M)
                         : merge_union(bufE, nall, U, r, M);
        uint64_t *ns = (uint64_t *)malloc(ncap * sizeof(uint64_t));
        dispatch(ns, 0, p->lf, ncap / p->lf, M, N);
        free(p->slots);
        p->slots = ns;
        p->cap = ncap;
        p->n = N;
        log_push(p, -1, ncap, nall, r);
        free(M);
    }
    p->applied = total;
    free(bufE); free(bufM); free(leaf); free(U); free(ek);
    return ORC_OK;
}

int orc_insert(orc_pma *p, const uint64_t *keys, uint64_t b)
{
    return apply_batch(p, keys, b, 0);
}

int orc_delete(orc_pma *p, const uint64_t *keys, uint64_t b)
{
    return apply_batch(p, keys, b, 1);
}

/* ------------------------------------------------------------------------ */
/* analytics on the plain edge set (Section 6.1, "Applications")            */

/* PageRank by power iteration with damping d (Section 6.1).  Orientation and
 * dangling vertices are not fixed by the paper; this is the usual in-link
 * form over all V vertices:
 *   x'[v] = (1-d)/V + d * ( sum_{u->v} x[u]/outdeg(u) + D/V ),
 *   D = sum of x[u] over vertices with no out-edge.
 * `edges` are sorted unique keys src<<32|dst; `x0` may be NULL (uniform). */
void orc_pagerank(uint32_t V, const uint64_t *edges, uint64_t m,
                  const double *x0, uint32_t iters, double d, double *out)
{
    uint64_t *deg = (uint64_t *)calloc(V, sizeof(uint64_t));
    double *x = (double *)malloc(V * sizeof(double));
    double *y = (double *)malloc(V * sizeof(double));
    for (uint64_t e = 0; e < m; e++) deg[edges[e] >> 32]++;
    for (uint32_t v = 0; v < V; v++) x[v] = x0 ? x0[v] : 1.0 / V;
    for (uint32_t it = 0; it < iters; it++) {
        double D = 0.0;
        for (uint32_t v = 0; v < V; v++) {
            y[v] = 0.0;
            if (deg[v] == 0) D += x[v];
        }
        for (uint64_t e = 0; e < m; e++) {
            uint32_t u = (uint32_t)(edges[e] >> 32), v = (uint32_t)edges[e];
            y[v] += x[u] / (double)deg[u];
        }
        for (uint32_t v = 0; v < V; v++)
            x[v] = (1.0 - d) / V + d * (y[v] + D / V);
    }
    memcpy(out, x, V * sizeof(double));
    free(deg); free(x); free(y);
}

/* Breadth-first search, Algorithm "Breadth-First Search" (Section 4.2):
 * minimum hop distance from the root along out-edges, -1 when unreached. */
void orc_bfs(uint32_t V, const uint64_t *edges, uint64_t m, uint32_t src, int32_t *dist)
{
    uint64_t *off = (uint64_t *)calloc((uint64_t)V + 1, sizeof(uint64_t));
    for (uint64_t e = 0; e < m; e++) off[(edges[e] >> 32) + 1]++;
    for (uint32_t v = 0; v < V; v++) off[v + 1] += off[v];
    uint32_t *queue = (uint32_t *)malloc((V ? V : 1) * sizeof(uint32_t));
    for (uint32_t v = 0; v < V; v++) dist[v] = -1;
    uint64_t head = 0, tail = 0;
    dist[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        uint32_t u = queue[head++];
        for (uint64_t e = off[u]; e < off[u + 1]; e++) {
            uint32_t v = (uint32_t)edges[e];
            if (dist[v] < 0) { dist[v] = dist[u] + 1; queue[tail++] = v; }
        }
    }
    free(off); free(queue);
}

static uint32_t uf_find(uint32_t *par, uint32_t x)
{
    while (par[x] != x) { par[x] = par[par[x]]; x = par[x]; }
    return x;
}

/* Connected components (Section 6.1): vertices joined by a path when edge
 * direction is ignored share a label, the smallest vertex id among them. */
void orc_cc(uint32_t V, const uint64_t *edges, uint64_t m, uint32_t *label)
{
    uint32_t *par = (uint32_t *)malloc((V ? V : 1) * sizeof(uint32_t));
    for (uint32_t v = 0; v < V; v++) par[v] = v;
    for (uint64_t e = 0; e < m; e++) {
        uint32_t a = uf_find(par, (uint32_t)(edges[e] >> 32));
        uint32_t b = uf_find(par, (uint32_t)edges[e]);
        if (a != b) { if (a < b) par[b] = a; else par[a] = b; }
    }
    for (uint32_t v = 0; v < V; v++) label[v] = uf_find(par, v);
    free(par);
}

/* ------------------------------------------------------------------------ */
/* the semantic layer: the graph's edge set as one sorted vector of unique
 * keys, each batch merged in (set union) or out (set difference).  It fixes
 * what the PMA must hold after any batch sequence, without any layout, and
 * plays the role of the rebuild-based baselines of Section 6 (CSR updated
 * by rebuilding; the single-threaded CPU structures) as a timing baseline. */

typedef struct {
    uint64_t *k;
    uint64_t n, cap;
} orc_set;

orc_set *orc_set_create(const uint64_t *keys, uint64_t n)
{
    orc_set *s = (orc_set *)calloc(1, sizeof(orc_set));
    if (!s) return NULL;
    s->cap = n ? n : 1;
    s->k = (uint64_t *)malloc(s->cap * sizeof(uint64_t));
    if (!s->k) { free(s); return NULL; }
    memcpy(s->k, keys, n * sizeof(uint64_t));
    s->n = sort_unique(s->k, n);
    return s;
}

void orc_set_free(orc_set *s)
{
    if (!s) return;
    free(s->k);
    free(s);
}

uint64_t orc_set_size(const orc_set *s) { return s->n; }
const uint64_t *orc_set_keys(const orc_set *s) { return s->k; }

/* Apply one batch: del = 0 union, 1 difference.  Returns the number of keys
 * that changed the set, or -1 when memory runs out (set unchanged). */
int64_t orc_set_apply(orc_set *s, const uint64_t *keys, uint64_t b, int del)
{
    uint64_t *U = (uint64_t *)malloc((b ? b : 1) * sizeof(uint64_t));
    if (!U) return -1;
    memcpy(U, keys, b * sizeof(uint64_t));
    uint64_t nu = sort_unique(U, b);
    uint64_t *out = (uint64_t *)malloc((s->n + nu + 1) * sizeof(uint64_t));
    if (!out) { free(U); return -1; }
    uint64_t i = 0, j = 0, m = 0, changed = 0;
    while (i < s->n || j < nu) {
        if (j >= nu || (i < s->n && s->k[i] < U[j])) {
            out[m++] = s->k[i++];
        } else if (i >= s->n || U[j] < s->k[i]) {
            if (!del) { out[m++] = U[j]; changed++; }
            j++;
        } else {                     /* present in both */
            if (!del) out[m++] = s->k[i];
            else changed++;
            i++; j++;
        }
    }
    free(U);
    free(s->k);
    s->k = out;
    s->n = m;
    s->cap = s->n + nu + 1;
    return (int64_t)changed;
}
