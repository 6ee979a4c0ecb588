// Learned segment locator: the leaf an update goes to is found from a model
// of where keys sit, and an exact bounded search corrects it, so the result
// is always the leaf BinarySearchLeafSegments would return (Algorithm "GPMA+
// Segment-Oriented Insertion"; the model is a design addition, not the
// paper's).
//
// The key CDF has two parts.  The source part is known exactly: row u runs
// from just after guard u-1 to guard u, and the CSR offsets kept with the
// array (Section 4.2) give both positions, so the key's leaf lies in the
// row's leaf span [first, last].  The destination part -- how far through
// its row's span a key with destination v sits -- is learned: x = u/V,
// y = v/(V+1), 32 hidden units h = relu(W1 [x y]^T + b1), t = y + w2 . h + b2,
// predicted leaf = first + floor(t * span).  Rows spanning at most kMinSpan
// leaves are searched directly.  Layer 1 (a K=2 product that needs full
// input precision) runs on the vector ALU in fp32; layer 2 runs on MFMA
// (v_mfma_f32_16x16x16_bf16, fp32 accumulate) with bf16 weights, the
// activations split into a bf16 high part and a bf16 low part (two MFMAs),
// which keeps about 16 bits of each activation.
//
// Error bounds are kept per row: row_eps[u] is the largest leaf error over
// row u's pivots, measured at the fit with this same code.  A lookup
// searches the window of e + e/4 + 2 leaves (e = row_eps[u]) on either side
// of the prediction, the slack absorbing merges since the fit.  The search
// runs over the window and the leaf past it, so it also tells whether the
// window brackets the key (pivot[lo] <= k < pivot[hi+1]); when it does not,
// a binary search over the whole span takes over.  One bound per row rather
// than one for the array keeps the windows of the long rows, where the model
// fits well, from taking the width the worst row needs.
#include "common.h"
#include "locator.h"
#include "pair.h"

using namespace gpma_dev;

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    // round to nearest even (inputs here are finite)
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ void key_features(uint64_t k, float inv_v, float inv_v1, uint32_t V, float &x,
                                             float &y) {
    const uint32_t src = (uint32_t)(k >> 32), dst = (uint32_t)k;
    x = (float)src * inv_v;
    y = (float)(dst == kGuardDst ? V : dst) * inv_v1;
}

// The model, copied into LDS by the whole block (lanes index its weights by
// their quad, which a register copy could only serve from scratch memory).
__device__ __forceinline__ void stage_model(const LocModel *__restrict__ model, LocModel *s_m) {
    const uint32_t *src = reinterpret_cast<const uint32_t *>(model);
    uint32_t *dst = reinterpret_cast<uint32_t *>(s_m);
    for (uint32_t t = threadIdx.x; t < sizeof(LocModel) / 4; t += blockDim.x) dst[t] = src[t];
    __syncthreads();
}

// Positions of the 64 keys kq[lane] of a wave (every lane active).  Lane l
// supplies row l%16 of the A operand (its key within a 16-key row block) and
// hidden units 4*(l/16) .. +3 of each 16-unit K block; B holds w2 in every
// column; the result for key 16*rb + 4*(l/16) + i comes back in lane l's
// value i.  s_out: 64 floats of LDS for the wave.
__device__ __forceinline__ float model_position(const LocModel &m, uint64_t kq, float *s_out) {
    const uint32_t lane = __lane_id();
    const uint32_t quad = lane >> 4;     // which 4 hidden units / which 4 output rows
    const uint32_t row = lane & 15;
    float xq, yq;
    key_features(kq, m.inv_v, m.inv_v1, m.V, xq, yq);
    // B operand: w2 for k = 4*quad + i of each K block, the same in every column
    bf16x4 b[2];
#pragma unroll
    for (int kb = 0; kb < 2; kb++)
#pragma unroll
        for (int i = 0; i < 4; i++) b[kb][i] = (short)m.w2[kb * 16 + 4 * quad + i];
#pragma unroll
    for (int rb = 0; rb < 4; rb++) {
        // features of key 16*rb + row, fetched from its owner lane
        const float x = __shfl(xq, 16 * rb + row, kWave);
        const float y = __shfl(yq, 16 * rb + row, kWave);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; kb++) {
            bf16x4 ahi, alo;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int u = kb * 16 + 4 * quad + i;
                const float h = fmaxf(m.w1x[u] * x + m.w1y[u] * y + m.b1[u], 0.f);
                const uint16_t hi = f32_to_bf16(h);
                ahi[i] = (short)hi;
                alo[i] = (short)f32_to_bf16(h - bf16_to_f32(hi));
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, b[kb], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, b[kb], acc, 0, 0, 0);
        }
        if (row == 0) {
#pragma unroll
            for (int i = 0; i < 4; i++) s_out[16 * rb + 4 * quad + i] = acc[i];
        }
    }
    wave_lds_sync();
    const float r = s_out[lane];
    wave_lds_sync();
    return yq + r + m.b2;
}

// leaf span of row u: from the leaf of guard u-1 (leaf 0 for u = 0) to the
// leaf of guard u; row_ptr[u] is one past guard u-1
struct Span {
    uint64_t first, last;
};
__device__ __forceinline__ Span row_span(const uint32_t *row_ptr, uint32_t u, uint32_t lf_log2) {
    const uint64_t rs = u ? row_ptr[u] : 0;
    const uint64_t re = row_ptr[u + 1];
    return Span{rs ? (rs - 1) >> lf_log2 : 0, (re - 1) >> lf_log2};
}

__device__ __forceinline__ uint64_t predict_in_span(float t, const Span &sp) {
    const uint64_t n = sp.last - sp.first + 1;
    float f = floorf(t * (float)n);
    if (!(f >= 0.f)) f = 0.f;
    if (f > (float)(n - 1)) f = (float)(n - 1);
    return sp.first + (uint64_t)f;
}

// leaf j's pivot: its first entry, a marked one ordering by its masked key
// (the dense pivot array the update kernels keep)
__device__ __forceinline__ uint64_t pivot(const uint64_t *piv, uint64_t j) { return piv[j]; }

// the largest leaf j in [lo, hi] with pivot(j) <= k (lo if none).  (An
// 8-way search, seven pivots loaded per step, measured slower: 71 against
// 43 us for a paired locate of 2^16 keys at scale 24.)
__device__ __forceinline__ uint64_t search_range(const uint64_t *piv, uint64_t lo, uint64_t hi, uint64_t k) {
    uint64_t a = lo, b = hi + 1;   // pivots in [a, b) : count of those <= k
    while (a < b) {
        const uint64_t mid = (a + b) >> 1;
        if (pivot(piv, mid) <= k) a = mid + 1; else b = mid;
    }
    return a > lo ? a - 1 : lo;
}

// Locate with the model.  The whole wave runs the MFMA inference (lanes past
// the end use key 0), then each lane corrects its own prediction.
struct LocateLearnedOp {
    struct Args {
        const uint64_t *keys;
        const uint32_t *n_dev;
        uint64_t n_max;
        const uint64_t *piv;
        const uint32_t *row_ptr;
        const uint32_t *row_eps;
        uint64_t L;
        uint32_t lf_log2;
        const LocModel *model;
        const Ctl *ctl;
        uint32_t *leaf;
        uint8_t *status;
        uint32_t *misses;
        WinSrc ws;
    };
    static __device__ __forceinline__ void run(const Args &args) {
        const uint64_t *__restrict__ keys = args.keys;
        const uint32_t *__restrict__ n_dev = args.n_dev;
        uint64_t n_max = args.n_max;
        const uint64_t *__restrict__ piv = args.piv;
        const uint32_t *__restrict__ row_ptr = args.row_ptr;
        const uint32_t *__restrict__ row_eps = args.row_eps;
        uint64_t L = args.L;
        uint32_t lf_log2 = args.lf_log2;
        const LocModel *__restrict__ model = args.model;
        const Ctl * ctl = args.ctl;
        uint32_t *__restrict__ leaf = args.leaf;
        uint8_t *__restrict__ status = args.status;
        uint32_t * misses = args.misses;
        WinSrc ws = args.ws;
        __shared__ float s_out[256];
        __shared__ LocModel s_m;
        const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
        const BatchView bv = batch_view(ws, keys, n_dev, n_max, ctl);
        const uint64_t n = bv.n;
        if ((uint64_t)blockIdx.x * blockDim.x >= n || bv.err) return;   // block-uniform
        stage_model(model, &s_m);
        const LocModel &m = s_m;
        const bool active = i < n;
        const uint64_t k = active ? (bv.keys[i] & bv.mask) : 0;
        if (active && ws.ukeys) ws.dense[i] = k;
        const uint32_t re = row_eps[key_src(k)];   // issued beside the row offsets
        const Span sp = row_span(row_ptr, key_src(k), lf_log2);
        const uint64_t span = sp.last - sp.first + 1;
        // the model runs (wave-wide, on MFMA) only for waves with a key in a
        // long row; the batch is sorted, so most waves hold short rows only or
        // long rows only
        float t = 0.f;
        if (__ballot(active && span > kMinSpan)) t = model_position(m, k, s_out + (threadIdx.x & ~63u));
        if (!active) return;
        uint64_t j;
        if (span <= kMinSpan) {
            j = search_range(piv, sp.first, sp.last, k);
        } else {
            const uint64_t p = predict_in_span(t, sp);
            const uint64_t e = (uint64_t)re + (re >> 2) + 2;
            const uint64_t lo = p > sp.first + e ? p - e : sp.first;
            const uint64_t hi = p + e < sp.last ? p + e : sp.last;
            // count the pivots <= k over leaves lo .. top (the window and the
            // leaf past it, inside the span)
            const uint64_t top = hi < sp.last ? hi + 1 : hi;
            uint64_t a = lo, b = top + 1;
            while (a < b) {
                const uint64_t mid = (a + b) >> 1;
                if (pivot(piv, mid) <= k) a = mid + 1; else b = mid;
            }
            const bool below = a == lo && lo > sp.first;   // pivot[lo] > k
            const bool above = a == top + 1 && top > hi;    // pivot[hi+1] <= k
            if (m.valid && m.L == L && !below && !above) {
                j = a > lo ? a - 1 : lo;
            } else {
                j = search_range(piv, sp.first, sp.last, k);
                atomicAdd(misses, 1u);
            }
        }
        leaf[i] = (uint32_t)j;
        status[i] = kPending;
    }
};

__global__ void __launch_bounds__(256)
k_locate_learned(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ n_dev, uint64_t n_max,
                 const uint64_t *__restrict__ piv, const uint32_t *__restrict__ row_ptr,
                 const uint32_t *__restrict__ row_eps, uint64_t L, uint32_t lf_log2,
                 const LocModel *__restrict__ model, const Ctl *ctl, uint32_t *__restrict__ leaf,
                 uint8_t *__restrict__ status, uint32_t *misses, WinSrc ws) {
    LocateLearnedOp::run(LocateLearnedOp::Args{keys, n_dev, n_max, piv, row_ptr, row_eps, L, lf_log2, model, ctl,
        leaf, status, misses, ws});
}

// Fit: sampled pivots, their features and the fp64 normal equations.  Each
// thread owns some entries of the symmetric 33x33 Gram matrix (plus the
// right-hand side) and walks the block's samples staged in LDS.
constexpr int kFeat = 33;                    // 32 hidden + bias
constexpr int kGram = kFeat * kFeat + kFeat; // G and r
constexpr int kFitChunk = 128;

__global__ void __launch_bounds__(256)
k_loc_gram(const uint64_t *__restrict__ piv, const uint32_t *__restrict__ row_ptr, uint64_t L, uint32_t lf_log2,
           uint64_t stride, uint64_t S, const LocModel *__restrict__ model, double *__restrict__ gram) {
    __shared__ double phi[kFitChunk][kFeat + 1];   // features and target (all 0: not a sample)
    const LocModel m = *model;
    double acc[5] = {0, 0, 0, 0, 0};
    for (uint64_t c0 = (uint64_t)blockIdx.x * kFitChunk; c0 < S; c0 += (uint64_t)gridDim.x * kFitChunk) {
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < kFitChunk; t += blockDim.x) {
            const uint64_t s = c0 + t;
            bool use = false;
            if (s < S) {
                const uint64_t j = s * stride;
                const uint64_t k = pivot(piv, j);
                const Span sp = row_span(row_ptr, key_src(k), lf_log2);
                const uint64_t span = sp.last - sp.first + 1;
                if (!is_guard(k) && span > kMinSpan) {
                    float x, y;
                    key_features(k, m.inv_v, m.inv_v1, m.V, x, y);
                    for (int u = 0; u < 32; u++)
                        phi[t][u] = fmax((double)m.w1x[u] * x + (double)m.w1y[u] * y + (double)m.b1[u], 0.0);
                    phi[t][32] = 1.0;
                    // target: the middle of leaf j's share of the span, less the skip term
                    phi[t][33] = ((double)(j - sp.first) + 0.5) / (double)span - (double)y;
                    use = true;
                }
            }
            if (!use)
                for (int u = 0; u <= kFeat; u++) phi[t][u] = 0.0;
        }
        __syncthreads();
        for (int q = 0; q < 5; q++) {
            const int e = threadIdx.x + q * 256;
            if (e >= kGram) break;
            const int a = e < kFeat * kFeat ? e / kFeat : e - kFeat * kFeat;
            const int bcol = e < kFeat * kFeat ? e % kFeat : kFeat;   // kFeat: the target column
            double s = 0.0;
            for (int t = 0; t < kFitChunk; t++) s += phi[t][a] * phi[t][bcol];
            acc[q] += s;
        }
    }
    for (int q = 0; q < 5; q++) {
        const int e = threadIdx.x + q * 256;
        if (e < kGram && acc[q] != 0.0) unsafeAtomicAdd(&gram[e], acc[q]);
    }
}

// Error bounds over every long-row leaf pivot: the largest leaf error of
// each row (row_eps) and of the array (*err).  A wave's pivots are
// consecutive leaves, so lanes of one row are adjacent: a segmented max
// leaves each row's largest at its first lane, which alone takes the atomic.
__global__ void __launch_bounds__(256)
k_loc_eval(const uint64_t *__restrict__ piv, const uint32_t *__restrict__ row_ptr, uint64_t L, uint32_t lf_log2,
           const LocModel *__restrict__ model, uint32_t *__restrict__ err, uint32_t *__restrict__ row_eps) {
    __shared__ float s_out[256];
    __shared__ LocModel s_m;
    stage_model(model, &s_m);
    const LocModel &m = s_m;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint32_t lane = __lane_id();
    uint32_t worst = 0;
    // the loop bound is wave-uniform (L is a multiple of 64 or the wave is the last)
    for (uint64_t j0 = (uint64_t)blockIdx.x * blockDim.x; j0 < L; j0 += stride) {
        const uint64_t j = j0 + threadIdx.x;
        const uint64_t k = j < L ? pivot(piv, j) : 0;
        const float t = model_position(m, k, s_out + (threadIdx.x & ~63u));
        uint32_t d = 0;
        bool use = false;
        if (j < L && !is_guard(k)) {
            const Span sp = row_span(row_ptr, key_src(k), lf_log2);
            if (sp.last - sp.first + 1 > kMinSpan) {
                const uint64_t p = predict_in_span(t, sp);
                const uint64_t dd = p > j ? p - j : j - p;
                d = dd > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)dd;
                use = true;
            }
        }
        worst = d > worst ? d : worst;
        // rows of the lanes that measured one (others take a row no lane has)
        const uint32_t u = use ? key_src(k) : 0xFFFFFFFFu;
#pragma unroll
        for (int w = 1; w < kWave; w <<= 1) {
            const uint32_t od = __shfl_down(d, w, kWave);
            const uint32_t ou = __shfl_down(u, w, kWave);
            if (lane + w < (uint32_t)kWave && ou == u && od > d) d = od;
        }
        const uint32_t pu = __shfl_up(u, 1, kWave);
        if (use && (lane == 0 || pu != u)) atomicMax(&row_eps[u], d);
    }
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        const uint32_t o = __shfl_xor(worst, d, kWave);
        worst = o > worst ? o : worst;
    }
    if (lane == 0) atomicMax(err, worst);
}

}  // namespace

namespace gpma_host {

void launch_locate_learned(const uint64_t *keys, const uint32_t *n_dev, uint64_t n_max, const uint64_t *piv,
                           const uint32_t *row_ptr, const uint32_t *row_eps, uint64_t L, uint32_t lf_log2,
                           const LocModel *model,
                           const Ctl *ctl, uint32_t *leaf, uint8_t *status, uint32_t *misses, hipStream_t s,
                           const WinSrc *ws) {
    if (!n_max) return;
    const WinSrc w = ws ? *ws : WinSrc{};
    hipLaunchKernelGGL(k_locate_learned, dim3((uint32_t)((n_max + 255) / 256)), dim3(256), 0, s, keys, n_dev,
                       n_max, piv, row_ptr, row_eps, L, lf_log2, model, ctl, leaf, status, misses, w);
}

size_t loc_gram_words() { return kGram; }

void launch_loc_gram(const uint64_t *piv, const uint32_t *row_ptr, uint64_t L, uint32_t lf_log2, uint64_t stride,
                     uint64_t S, const LocModel *model, double *gram, hipStream_t s) {
    uint64_t blocks = (S + kFitChunk - 1) / kFitChunk;
    if (blocks > 128) blocks = 128;
    hipLaunchKernelGGL(k_loc_gram, dim3((uint32_t)blocks), dim3(256), 0, s, piv, row_ptr, L, lf_log2, stride, S,
                       model, gram);
}

void launch_loc_eval(const uint64_t *piv, const uint32_t *row_ptr, uint64_t L, uint32_t lf_log2,
                     const LocModel *model, uint32_t *err, uint32_t *row_eps, hipStream_t s) {
    uint64_t blocks = (L + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_loc_eval, dim3((uint32_t)blocks), dim3(256), 0, s, piv, row_ptr, L, lf_log2, model, err,
                       row_eps);
}

void launch_locate_learned2(uint64_t n_max, const uint64_t *const piv[2], const uint32_t *const row_ptr[2],
                            const uint32_t *const row_eps[2],
                            const uint64_t L[2], uint32_t lf_log2, const LocModel *const model[2],
                            const Ctl *const ctl[2], uint32_t *const leaf[2], uint8_t *const status[2],
                            uint32_t *const misses[2], const WinSrc ws[2], hipStream_t s) {
    if (!n_max) return;
    LocateLearnedOp::Args a[2];
    for (int k = 0; k < 2; k++)
        a[k] = {nullptr, nullptr, n_max, piv[k], row_ptr[k], row_eps[k], L[k], lf_log2, model[k], ctl[k], leaf[k], status[k],
                misses[k], ws[k]};
    launch_pair<LocateLearnedOp, 256>((uint32_t)((n_max + 255) / 256), a[0], a[1], s);
}

}  // namespace gpma_host

