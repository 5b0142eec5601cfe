// Matrix-core sampling product S = K(X, X; h) R (each row's own leaf block
// removed): the dominant kernel of the randomized HSS construction.
//
// Per workgroup: 256 rows (8 waves x 32 rows) and up to 256 sample columns
// (RB blocks of 32), loop over all points j in tiles of 32.  Per tile each
// lane evaluates the 16 kernel entries it feeds to the matrix cores -- its
// row i = lane % 32 and points j = 8 g + q, 16 + 8 g + q (g = lane / 32,
// q = 0..7), exactly the A-operand layout of v_mfma_f32_32x32x16_{f16,bf16}
// -- so the entries never leave registers:
//     t = -c |x'_i|^2 - c |y'_j|^2 + sum_k (2 c x'_ik) y'_jk,  e = exp2(t),
// with c = log2(e) / (2 h^2) and x' = x - a, y' = y - a re-centred on the
// workgroup's first point a (the kernel is translation invariant; this keeps
// the FP32 norm expansion free of large cancellations for the pairs that
// matter).  e is split into FP16 / BF16 hi (+ lo = e - hi) terms (FP16
// entries carry a 2^14 scale so small values keep full precision) and
// multiplied into the FP32 accumulators with the random block, which is
// pre-swizzled into the B-operand layout and staged through LDS.  The FP32
// mode uses v_mfma_f32_32x32x2_f32 on the FP32 entries instead.
//
// Far from the diagonal most Gaussian kernel entries are negligibly small
// (Section 4.1); in tree order they come in whole tiles.  A wave skips a
// 32 x 32 (row, point) tile -- its exp2, split and products with R -- when
// every exponent of the tile is below kSkipLog2 (all entries < 2^-32): the
// decision is one ballot per tile and wave-uniform.  Each skipped entry
// changes a sample by at most 2^-32 |R_jk|, so a row changes by at most
// n 2^-32 max|R| (2^-12 at n = 2^20), below the FP32 accumulation error of
// the sample itself and far below the compression tolerance.
#include <algorithm>

#include "internal.hpp"
#include "wide.hpp"

namespace krr {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));

enum Mode : int { M_F32 = 0, M_F16 = 1, M_BF16 = 2 };

constexpr int WAVES = 8;
constexpr float kSkipLog2 = -32.0f;  // tiles with every entry below 2^-32 are skipped
constexpr int THREADS = 64 * WAVES;
constexpr int ROWS = 32 * WAVES;  // rows per workgroup
constexpr int JT = 32;            // points per tile
// points per staged Y super-tile (a multiple of JT, smaller for wide points)
template <int D> struct YTile { static constexpr int N = D <= 16 ? 256 : (D <= 32 ? 128 : 64); };

// ---------------------------------------------------------------- swizzle

// Rsw layout for FP16 / BF16: [tile][cb][kb][lane][q] with column
// 32 cb + lane % 32 and point j = 32 tile + 16 kb + p(q, g), g = lane / 32,
// p = 4 g + q for q < 4 and 8 + 4 g + (q - 4) above: the order in which the
// distance product leaves the kernel entries in each lane's registers.
template <class H>
__global__ void k_swizzle_h(const float *__restrict__ R, int64_t n, int r, int64_t tiles, H *__restrict__ Rsw) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int RBt = r / 32;
    if (t >= tiles * RBt * 2 * 64) return;
    int lane = (int)(t % 64);
    int64_t u = t / 64;
    int kb = (int)(u % 2);
    u /= 2;
    int cb = (int)(u % RBt);
    int64_t tile = u / RBt;
    int col = 32 * cb + lane % 32;
    for (int q = 0; q < 8; ++q) {
        const int gg = lane / 32;
        int64_t j = 32 * tile + 16 * kb + (q < 4 ? 4 * gg + q : 8 + 4 * gg + (q - 4));
        float v = j < n ? R[j * r + col] : 0.0f;
        Rsw[t * 8 + q] = (H)v;
    }
}

// Rsw layout for FP32: [tile][cb][s][lane] with point j = 32 tile + 2 s + lane / 32.
__global__ void k_swizzle_f(const float *__restrict__ R, int64_t n, int r, int64_t tiles, float *__restrict__ Rsw) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int RBt = r / 32;
    if (t >= tiles * RBt * 16 * 64) return;
    int lane = (int)(t % 64);
    int64_t u = t / 64;
    int s = (int)(u % 16);
    u /= 16;
    int cb = (int)(u % RBt);
    int64_t tile = u / RBt;
    int64_t j = 32 * tile + 2 * s + lane / 32;
    Rsw[t] = j < n ? R[j * r + 32 * cb + lane % 32] : 0.0f;
}

__global__ void k_to_float(const double *__restrict__ x, int64_t len, float *__restrict__ y) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < len) y[t] = (float)x[t];
}

// ----------------------------------------------------------------- kernel

template <int MODE> struct Op;
template <> struct Op<M_F16> {
    typedef _Float16 H;
    typedef half8 V;
    static __device__ __forceinline__ f16v mfma(V a, V b, f16v c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct Op<M_BF16> {
    typedef __bf16 H;
    typedef bf8 V;
    static __device__ __forceinline__ f16v mfma(V a, V b, f16v c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

template <class T, int D, int YS = YTile<D>::N>
__device__ __forceinline__ void stage_y(const T *__restrict__ X, int64_t jlo, int64_t jhi, int d, int64_t j0,
                                        const float *anchor, float cs, float (*ys)[D + 1]) {
    // ys[p][0..D) = y' = y - a, ys[p][D] = -c |y'|^2 (or -inf outside the columns [jlo, jhi))
    for (int p = threadIdx.x; p < YS; p += THREADS) {
        int64_t j = j0 + p;
        const bool ok = j >= jlo && j < jhi;
        float nrm = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            float v = (ok && k < d) ? (float)X[j * d + k] - anchor[k] : 0.0f;
            ys[p][k] = v;
            nrm = fmaf(v, v, nrm);
        }
        ys[p][D] = ok ? -cs * nrm : -INFINITY;
    }
}

// Augmented points for the distance product: row p of ya holds
// (y'_1 .. y'_D, 1, -c |y'_p|^2) (zero outside the columns [jlo, jhi), where
// the last entry is -inf so that the kernel value is exactly 0).
template <class T, int D, int YS>
__device__ __forceinline__ void stage_ya(const T *__restrict__ X, int64_t jlo, int64_t jhi, int d, int64_t j0,
                                         const float *anchor, float cs, float (*ya)[D + 3]) {
    for (int p = threadIdx.x; p < YS; p += THREADS) {
        int64_t j = j0 + p;
        const bool ok = j >= jlo && j < jhi;
        float nrm = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            float v = (ok && k < d) ? (float)X[j * d + k] - anchor[k] : 0.0f;
            ya[p][k] = v;
            nrm = fmaf(v, v, nrm);
        }
        ya[p][D] = 1.0f;
        ya[p][D + 1] = ok ? -cs * nrm : -INFINITY;
    }
}

// Exponents of one 32 x 32 (point j, row i) block on the matrix cores:
// t[r] = x~_i . y~_j for j = 8 (r / 4) + 4 g + r % 4 (the C layout of
// v_mfma_f32_32x32x2_f32 with points as rows and the wave's rows as columns).
// xa[s] holds the lane's own x~ entry 2 s + g.
template <int D>
__device__ __forceinline__ f16v dist_mfma(const float *xa, const float (*ya)[D + 3], int pbase, int lane) {
    constexpr int KS = (D + 2 + 1) / 2;
    const int g = lane >> 5;
    f16v t = {};
#pragma unroll
    for (int sidx = 0; sidx < KS; ++sidx) {
        const int k = 2 * sidx + g;
        const float a = (k < D + 2) ? ya[pbase + (lane & 31)][k] : 0.0f;
        t = __builtin_amdgcn_mfma_f32_32x32x2f32(a, xa[sidx], t, 0, 0, 0);
    }
    return t;
}

// BF16 form of the exponent product (split modes, D <= 16): both augmented
// vectors are split into three BF16 terms (hi + mid + lo: 24 bits, FP32's
// range) and the six cross products down to 2^-16 (hh, hm, mh, hl, lh, mm)
// are packed along K, 6 (D + 2) slots rounded up to 16: KB / 16
// v_mfma_f32_32x32x16_bf16 per 32 x 32 block instead of (D + 3) / 2
// v_mfma_f32_32x32x2_f32, with the same C layout.  Products of BF16 terms are
// exact in FP32, so the exponents keep the FP32 form's accuracy.
template <int D> struct BExp {
    static constexpr bool on = D <= 16;
    static constexpr int KB = 16 * ((6 * (D + 2) + 15) / 16);  // packed K
    static constexpr int LDB = KB + 8;                         // staged row (16 bytes of padding)
};

__device__ __forceinline__ void split3b(float v, __bf16 &h, __bf16 &m, __bf16 &l) {
    h = (__bf16)v;
    const float r1 = v - (float)h;
    m = (__bf16)r1;
    l = (__bf16)(r1 - (float)m);
}

// the term of each packed pair on the A side (points) and on the B side (rows)
__device__ __forceinline__ int pair_a(int t) { return t == 2 || t == 5 ? 1 : (t == 4 ? 2 : 0); }
__device__ __forceinline__ int pair_b(int t) { return t == 1 || t == 5 ? 1 : (t == 3 ? 2 : 0); }

// Packed A rows of the augmented points y~ = (y', 1, -c |y'|^2) (outside the
// columns [jlo, jhi) the last entry is -1e30, so the kernel value is 0).
template <class T, int D, int YS>
__device__ __forceinline__ void stage_yb(const T *__restrict__ X, int64_t jlo, int64_t jhi, int d, int64_t j0,
                                         const float *anchor, float cs, __bf16 *yb) {
    constexpr int KB = BExp<D>::KB, LDB = BExp<D>::LDB, DA = D + 2;
    for (int p = threadIdx.x; p < YS; p += THREADS) {
        const int64_t j = j0 + p;
        const bool ok = j >= jlo && j < jhi;
        float v[DA];
        float nrm = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            v[k] = (ok && k < d) ? (float)X[j * d + k] - anchor[k] : 0.0f;
            nrm = fmaf(v[k], v[k], nrm);
        }
        v[D] = 1.0f;
        v[D + 1] = ok ? -cs * nrm : -1e30f;
        __bf16 *row = yb + (int64_t)p * LDB;
#pragma unroll
        for (int k = 0; k < DA; ++k) {
            __bf16 hml[3];
            split3b(v[k], hml[0], hml[1], hml[2]);
#pragma unroll
            for (int t = 0; t < 6; ++t) row[t * DA + k] = hml[pair_a(t)];
        }
        for (int k = 6 * DA; k < KB; ++k) row[k] = (__bf16)0.0f;
    }
}

// Exponents of one 32 x 32 (point j, row i) block from the packed operands
// (C layout as dist_mfma); xb[s] holds the lane's row slots 16 s + 8 g + e.
template <int D>
__device__ __forceinline__ f16v dist_bf16(const bf8 *xb, const __bf16 *yb, int pbase, int lane) {
    constexpr int KS = BExp<D>::KB / 16, LDB = BExp<D>::LDB;
    const int g = lane >> 5;
    const __bf16 *row = yb + (int64_t)(pbase + (lane & 31)) * LDB + 8 * g;
    f16v t = {};
#pragma unroll
    for (int sidx = 0; sidx < KS; ++sidx)
        t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const bf8 *>(row + 16 * sidx), xb[sidx], t, 0, 0,
                                                   0);
    return t;
}

// Kernel entries from the exponents (masking entries of the row's own leaf),
// split into the A operands of the two 16-point blocks: block kb takes
// registers 8 kb .. 8 kb + 7, i.e. points 16 kb + (4 g + q, 8 + 4 g + q).
template <int MODE, int TERMS, bool MASK>
__device__ __forceinline__ void exp_split(typename Op<MODE>::V (&ahi)[2], typename Op<MODE>::V (&alo)[2],
                                          const f16v &t, int g, int64_t jt, int32_t my_lb, int32_t my_le) {
    typedef typename Op<MODE>::H H;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        float e = __builtin_amdgcn_exp2f(t[r]);
        if (MASK) {
            const int64_t j = jt + 8 * (r >> 2) + 4 * g + (r & 3);
            e = (j >= my_lb && j < my_le) ? 0.0f : e;
        }
        const H hi = (H)e;
        ahi[r >> 3][r & 7] = hi;
        if (TERMS == 2) alo[r >> 3][r & 7] = (H)(e - (float)hi);
    }
}

// Wave-uniform test: no entry of the wave's tile reaches the skip threshold
// (thr in the exponents' log2 units, which include the FP16 scale).
__device__ __forceinline__ bool tile_negligible(const float *t, int cnt, float thr) {
    float m = t[0];
    for (int r = 1; r < cnt; ++r) m = fmaxf(m, t[r]);
    return __ballot(m >= thr) == 0;
}

// FP32 mode: the exponents of the lane's 16 entries of one tile (its row and
// points j = 2 s + g), on the vector ALUs.
template <int D>
__device__ __forceinline__ void expo_f(float (&t)[16], const float *xs, float nx, const float (*ys)[D + 1], int pbase,
                                       int g) {
#pragma unroll
    for (int sidx = 0; sidx < 16; ++sidx) {
        const int p = pbase + 2 * sidx + g;
        float v = nx + ys[p][D];
#pragma unroll
        for (int k = 0; k < D; ++k) v = fmaf(xs[k], ys[p][k], v);
        t[sidx] = v;
    }
}

// FP32 mode: entries from the exponents (masking the row's own leaf).
template <bool MASK>
__device__ __forceinline__ void exp_f(float (&a)[16], const float (&t)[16], int g, int64_t jt, int32_t my_lb,
                                      int32_t my_le) {
#pragma unroll
    for (int sidx = 0; sidx < 16; ++sidx) {
        float e = __builtin_amdgcn_exp2f(t[sidx]);
        if (MASK) {
            const int64_t j = jt + 2 * sidx + g;
            e = (j >= my_lb && j < my_le) ? 0.0f : e;
        }
        a[sidx] = e;
    }
}

// FP32 mode: 16 v_mfma_f32_32x32x2_f32 steps per column block.
template <int RB>
__device__ __forceinline__ void mfma_f(f16v (&acc)[RB], const float (&cur)[16], const char *rtile, int lane) {
    const float *rt = reinterpret_cast<const float *>(rtile);
#pragma unroll
    for (int sidx = 0; sidx < 16; ++sidx) {
#pragma unroll
        for (int c = 0; c < RB; ++c) {
            const float b = rt[(c * 16 + sidx) * 64 + lane];
            acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(cur[sidx], b, acc[c], 0, 0, 0);
        }
    }
}

template <class T, int D, int RB, int MODE, int TERMS>
__global__ __launch_bounds__(THREADS) void k_sample_mfma(const T *__restrict__ X, int64_t n, int d, float cs,
                                                         const void *__restrict__ Rsw_, int RBt, int cb0,
                                                         const int32_t *__restrict__ lb, const int32_t *__restrict__ le,
                                                         float *__restrict__ S, int ldS,
                                                         const SampBlock *__restrict__ bt, float skip_log2) {
    constexpr int OPM = MODE == M_F32 ? M_F16 : MODE;
    typedef typename Op<OPM>::V V;
    constexpr int RTILE_H = RB * 2 * 64 * 8;
    constexpr int RTILE_F = RB * 16 * 64;
    constexpr int RTILE_B = MODE == M_F32 ? RTILE_F * 4 : RTILE_H * 2;
    constexpr int YS = YTile<D>::N;
    constexpr int SUPER = YS / JT;  // tiles per Y super-tile
    __shared__ __attribute__((aligned(16))) char rbuf[2][RTILE_B];
    // plain Y tiles (FP32 mode), augmented ones (split modes) or packed BF16
    // terms of the augmented ones (split modes, D <= 32)
    constexpr bool BX = MODE != M_F32 && BExp<D>::on;
    constexpr int YBYTES = MODE == M_F32 ? 2 * YS * (D + 1) * 4
                                         : (BX ? 2 * YS * BExp<D>::LDB * 2 : 2 * YS * (D + 3) * 4);
    __shared__ __attribute__((aligned(16))) char yraw[YBYTES];
    __shared__ float anchor[D];
    float(*ysh0)[D + 1] = reinterpret_cast<float(*)[D + 1]>(yraw);
    float(*ysh1)[D + 1] = reinterpret_cast<float(*)[D + 1]>(yraw) + YS;
    float(*const ysh[2])[D + 1] = {ysh0, ysh1};

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 5;
    // rows [i0, iend) against columns [jlo, jhi): the whole matrix, or one
    // problem's diagonal block in a batch
    int64_t i0, iend, jlo, jhi;
    if (bt) {
        const SampBlock sb = bt[blockIdx.x];
        i0 = sb.i0;
        iend = sb.iend;
        jlo = sb.jlo;
        jhi = sb.jhi;
        cs = sb.cs;
    } else {
        i0 = (int64_t)blockIdx.x * ROWS;
        iend = n;
        jlo = 0;
        jhi = n;
    }
    const int64_t i = i0 + 32 * w + (lane & 31);
    const bool row_ok = i < iend;
    if (tid < D) anchor[tid] = (tid < d) ? (float)X[i0 * d + tid] : 0.0f;
    __syncthreads();
    float xs[D];
    float nx = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        float v = (row_ok && k < d) ? (float)X[i * d + k] - anchor[k] : 0.0f;
        nx = fmaf(v, v, nx);
        xs[k] = 2.0f * cs * v;
    }
    // FP16 entries are evaluated as e * 2^14 (the exponent gains 14) so that
    // small kernel values stay in FP16's normal range; the accumulators are
    // scaled back by 2^-14 on write-out (both exact power-of-two scalings).
    constexpr float kE2 = MODE == M_F16 ? 14.0f : 0.0f;
    constexpr float kInvScale = MODE == M_F16 ? 1.0f / 16384.0f : 1.0f;
    nx = -cs * nx + kE2;
    const int32_t my_lb = (row_ok && lb) ? lb[i] : 0;
    const int32_t my_le = (row_ok && lb) ? le[i] : 0;
    // the wave's masked column range (tiles outside it take the unmasked path)
    int32_t wlb = (row_ok && lb) ? my_lb : INT32_MAX, wle = (row_ok && lb) ? my_le : INT32_MIN;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        wlb = min(wlb, __shfl_xor(wlb, o, 64));
        wle = max(wle, __shfl_xor(wle, o, 64));
    }

    const int64_t t_lo = jlo / JT, t_hi = (jhi + JT - 1) / JT, s0 = t_lo / SUPER;
    const int t_lo_off = (int)((t_lo * JT) % YS);
    const char *Rg = static_cast<const char *>(Rsw_);
    const int64_t tile_stride_b = (int64_t)RBt * (RTILE_B / RB);
    const int64_t cb_off_b = (int64_t)cb0 * (RTILE_B / RB);
    constexpr int PIECES = RTILE_B / 16;
    constexpr int PER_T = (PIECES + THREADS - 1) / THREADS;
    static_assert(PER_T <= 4, "R tile too large for the prefetch registers");
    uint4 pre0, pre1, pre2, pre3;
#define KRR_PIECE_OK(u) ((u) < PER_T && (PIECES % THREADS == 0 || tid + (u) * THREADS < PIECES))
#define KRR_LOAD_R(tile)                                                                          \
    do {                                                                                          \
        const uint4 *src_ = reinterpret_cast<const uint4 *>(Rg + (tile) * tile_stride_b + cb_off_b); \
        if (KRR_PIECE_OK(0)) pre0 = src_[tid];                                                    \
        if (KRR_PIECE_OK(1)) pre1 = src_[tid + THREADS];                                          \
        if (KRR_PIECE_OK(2)) pre2 = src_[tid + 2 * THREADS];                                      \
        if (KRR_PIECE_OK(3)) pre3 = src_[tid + 3 * THREADS];                                      \
    } while (0)
#define KRR_STORE_R(buf)                                                                          \
    do {                                                                                          \
        uint4 *dst_ = reinterpret_cast<uint4 *>(rbuf[buf]);                                       \
        if (KRR_PIECE_OK(0)) dst_[tid] = pre0;                                                    \
        if (KRR_PIECE_OK(1)) dst_[tid + THREADS] = pre1;                                          \
        if (KRR_PIECE_OK(2)) dst_[tid + 2 * THREADS] = pre2;                                      \
        if (KRR_PIECE_OK(3)) dst_[tid + 3 * THREADS] = pre3;                                      \
    } while (0)

    f16v acc[RB];
#pragma unroll
    for (int c = 0; c < RB; ++c)
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[c][q] = 0.0f;

    // prologue: R tile t_lo in LDS, R tile t_lo + 1 in flight; Y super-tiles
    // s0 and s0 + 1 staged (the loop stages each later one a super-tile ahead)
    if constexpr (MODE == M_F32) {
        stage_y<T, D>(X, jlo, jhi, d, s0 * YS, anchor, cs, ysh[s0 & 1]);
        stage_y<T, D>(X, jlo, jhi, d, (s0 + 1) * YS, anchor, cs, ysh[(s0 + 1) & 1]);
    }
    KRR_LOAD_R(t_lo);
    KRR_STORE_R(t_lo & 1);
    KRR_LOAD_R(t_lo + 1);
    __syncthreads();

    // the padded random block has two zero tiles past the end, so every
    // prefetch below is in bounds; tiles past n evaluate to exp2(-inf) = 0
    // Tile t's masking (wave-uniform decision): its columns meet the wave's leaf range.
#define KRR_TILE_MASKED(tt) ((int64_t)(tt) * JT < (int64_t)wle && (int64_t)(tt) * JT + JT > (int64_t)wlb)
    if constexpr (MODE == M_F32) {
        float a0[16], a1[16], tv[16];
        bool sk0, sk1 = false;
        expo_f<D>(tv, xs, nx, ysh[s0 & 1], t_lo_off, g);
        sk0 = tile_negligible(tv, 16, skip_log2);
        if (!sk0) exp_f<true>(a0, tv, g, t_lo * JT, my_lb, my_le);
        for (int64_t t = t_lo; t < t_hi; t += 2) {
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const int64_t tc = t + half;
                if (half == 1 && tc >= t_hi) break;
                if (tc % SUPER == 0 && tc != t_lo) {
                    const int64_t sup = tc / SUPER + 1;
                    stage_y<T, D>(X, jlo, jhi, d, sup * YS, anchor, cs, ysh[sup & 1]);
                }
                const int64_t tn = tc + 1;
                const float(*ysn)[D + 1] = ysh[(tn / SUPER) & 1];
                const int pbn = (int)((tn * JT) % YS);
                float(&cur)[16] = half == 0 ? a0 : a1;
                float(&nxt)[16] = half == 0 ? a1 : a0;
                bool &skc = half == 0 ? sk0 : sk1;
                bool &skn = half == 0 ? sk1 : sk0;
                expo_f<D>(tv, xs, nx, ysn, pbn, g);
                skn = tile_negligible(tv, 16, skip_log2);
                if (!skc) mfma_f<RB>(acc, cur, rbuf[tc & 1], lane);
                if (!skn) {
                    if (KRR_TILE_MASKED(tn))
                        exp_f<true>(nxt, tv, g, tn * JT, my_lb, my_le);
                    else
                        exp_f<false>(nxt, tv, g, tn * JT, my_lb, my_le);
                }
                KRR_STORE_R((tc + 1) & 1);
                KRR_LOAD_R(tc + 2);
                __syncthreads();
            }
        }
    } else {
        // x~ = (2 c x', -c |x'|^2 (+ 14 for FP16), 1): entries 2 s + g of the lane's own row
        constexpr int KS = (D + 2 + 1) / 2;
        float xa[KS];
        auto xt = [&](int k) { return k < D ? xs[k] : (k == D ? nx : (k == D + 1 ? 1.0f : 0.0f)); };
#pragma unroll
        for (int sidx = 0; sidx < KS; ++sidx) xa[sidx] = g ? xt(2 * sidx + 1) : xt(2 * sidx);
        // BF16 form: the lane's packed row slots 16 s + 8 g + e
        constexpr int KS16 = BX ? BExp<D>::KB / 16 : 1;
        bf8 xb[KS16];
        if constexpr (BX) {
#pragma unroll
            for (int sidx = 0; sidx < KS16; ++sidx)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int slot = 16 * sidx + 8 * g + e, DA = D + 2;
                    __bf16 v = (__bf16)0.0f;
                    if (slot < 6 * DA) {
                        __bf16 hml[3];
                        split3b(xt(slot % DA), hml[0], hml[1], hml[2]);
                        v = hml[pair_b(slot / DA)];
                    }
                    xb[sidx][e] = v;
                }
        }
        // augmented Y tiles replace the plain ones in this mode
        float(*ya0)[D + 3] = reinterpret_cast<float(*)[D + 3]>(yraw);
        float(*ya1)[D + 3] = reinterpret_cast<float(*)[D + 3]>(yraw) + YS;
        __bf16 *yb0 = reinterpret_cast<__bf16 *>(yraw);
        __bf16 *yb1 = yb0 + (BX ? YS * BExp<D>::LDB : 0);
        auto stage = [&](int64_t sup) {
            if constexpr (BX)
                stage_yb<T, D, YS>(X, jlo, jhi, d, sup * YS, anchor, cs, (sup & 1) ? yb1 : yb0);
            else
                stage_ya<T, D, YS>(X, jlo, jhi, d, sup * YS, anchor, cs, (sup & 1) ? ya1 : ya0);
        };
        auto dist = [&](int64_t tt) -> f16v {
            const bool odd = ((tt / SUPER) & 1) != 0;
            const int pb = (int)((tt * JT) % YS);
            if constexpr (BX)
                return dist_bf16<D>(xb, odd ? yb1 : yb0, pb, lane);
            else
                return dist_mfma<D>(xa, odd ? ya1 : ya0, pb, lane);
        };
        stage(s0);
        stage(s0 + 1);
        __syncthreads();
        V h0[2], l0[2], h1[2], l1[2];
        // the threshold in the exponents' units (FP16 entries carry 2^14)
        const float thr = skip_log2 + kE2;
        bool sk0, sk1 = false;
        {
            f16v t0 = dist(t_lo);
            float tt[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) tt[r] = t0[r];
            sk0 = tile_negligible(tt, 16, thr);
            if (!sk0) {
                if (KRR_TILE_MASKED(t_lo))
                    exp_split<MODE, TERMS, true>(h0, l0, t0, g, t_lo * JT, my_lb, my_le);
                else
                    exp_split<MODE, TERMS, false>(h0, l0, t0, g, t_lo * JT, my_lb, my_le);
            }
        }
        for (int64_t t = t_lo; t < t_hi; t += 2) {
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const int64_t tc = t + half;
                if (half == 1 && tc >= t_hi) break;
                if (tc % SUPER == 0 && tc != t_lo) stage(tc / SUPER + 1);
                const int64_t tn = tc + 1;
                V(&ch)[2] = half == 0 ? h0 : h1;
                V(&cl)[2] = half == 0 ? l0 : l1;
                V(&nh)[2] = half == 0 ? h1 : h0;
                V(&nl)[2] = half == 0 ? l1 : l0;
                // exponents of the next tile first (matrix pipe), then this
                // tile's products, then the next tile's entries (vector ALUs)
                bool &skc = half == 0 ? sk0 : sk1;
                bool &skn = half == 0 ? sk1 : sk0;
                const f16v tnext = dist(tn);
                {
                    float tt[16];
#pragma unroll
                    for (int r = 0; r < 16; ++r) tt[r] = tnext[r];
                    skn = tile_negligible(tt, 16, thr);
                }
                if (!skc) {
                    const V *rt = reinterpret_cast<const V *>(rbuf[tc & 1]);
#pragma unroll
                    for (int c = 0; c < RB; ++c)
#pragma unroll
                        for (int kb = 0; kb < 2; ++kb) {
                            const V b = rt[(c * 2 + kb) * 64 + lane];
                            acc[c] = Op<MODE>::mfma(ch[kb], b, acc[c]);
                            if (TERMS == 2) acc[c] = Op<MODE>::mfma(cl[kb], b, acc[c]);
                        }
                }
                if (!skn) {
                    if (KRR_TILE_MASKED(tn))
                        exp_split<MODE, TERMS, true>(nh, nl, tnext, g, tn * JT, my_lb, my_le);
                    else
                        exp_split<MODE, TERMS, false>(nh, nl, tnext, g, tn * JT, my_lb, my_le);
                }
                KRR_STORE_R((tc + 1) & 1);
                KRR_LOAD_R(tc + 2);
                __syncthreads();
            }
        }
    }
    // write out: lane holds column 32 c + lane % 32 of rows 8 (q / 4) + 4 g + q % 4
#pragma unroll
    for (int c = 0; c < RB; ++c)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int m = 8 * (q >> 2) + 4 * g + (q & 3);
            const int64_t row = i0 + 32 * w + m;
            if (row < iend) S[row * ldS + 32 * (cb0 + c) + (lane & 31)] = acc[c][q] * kInvScale;
        }
#undef KRR_TILE_MASKED
#undef KRR_LOAD_R
#undef KRR_STORE_R
#undef KRR_PIECE_OK
}

// Column blocks per pass: 8 (256 columns) where the accumulators fit in
// registers next to the operands, fewer for wide points and the FP32 mode.
template <int D, int MODE> struct RbMax {
    static constexpr int V = MODE == M_F32 ? (D <= 8 ? 8 : (D <= 32 ? 4 : 2)) : (D <= 32 ? 8 : 4);
};

template <class T, int D, int MODE, int TERMS>
void launch_passes(const T *X, int64_t n, int d, float cs, const void *Rsw, int r, const int32_t *lb,
                   const int32_t *le, float *S, hipStream_t s, const SampBlock *bt, int64_t nblk) {
    constexpr int RBM = RbMax<D, MODE>::V;
    const int cap = std::min(RBM, tune_get(KRR_TUNE_SAMPLE_RB));  // column blocks per pass
    // no tile's exponents are below -inf: the knob off evaluates every tile
    const float skip = tune_get(KRR_TUNE_SAMPLE_SKIP) ? kSkipLog2 : -INFINITY;
    const int RBt = r / 32;
    int cb0 = 0;
    while (cb0 < RBt) {
        const int left = RBt - cb0;
        dim3 grid((unsigned)(bt ? nblk : ceil_div(n, ROWS)));
        if (RBM >= 8 && cap >= 8 && left >= 8) {
            k_sample_mfma<T, D, (RBM >= 8 ? 8 : RBM), MODE, TERMS><<<grid, THREADS, 0, s>>>(X, n, d, cs, Rsw, RBt, cb0,
                                                                                        lb, le, S, r, bt, skip);
            cb0 += 8;
        } else if (RBM >= 4 && cap >= 4 && left >= 4) {
            k_sample_mfma<T, D, (RBM >= 4 ? 4 : RBM), MODE, TERMS><<<grid, THREADS, 0, s>>>(X, n, d, cs, Rsw, RBt, cb0,
                                                                                        lb, le, S, r, bt, skip);
            cb0 += 4;
        } else if (cap >= 2 && left >= 2) {
            k_sample_mfma<T, D, 2, MODE, TERMS><<<grid, THREADS, 0, s>>>(X, n, d, cs, Rsw, RBt, cb0, lb, le, S, r, bt, skip);
            cb0 += 2;
        } else {
            k_sample_mfma<T, D, 1, MODE, TERMS><<<grid, THREADS, 0, s>>>(X, n, d, cs, Rsw, RBt, cb0, lb, le, S, r, bt, skip);
            cb0 += 1;
        }
        check_launch("k_sample_mfma");
    }
}

template <class T, int D>
void dispatch_mode(const T *X, int64_t n, int d, float cs, const void *Rsw, int r, const int32_t *lb, const int32_t *le,
                   float *S, int prec, int split, hipStream_t s, const SampBlock *bt, int64_t nb) {
    if (prec == KRR_F32)
        launch_passes<T, D, M_F32, 1>(X, n, d, cs, Rsw, r, lb, le, S, s, bt, nb);
    else if (prec == KRR_F16_SPLIT)
        split == 2 ? launch_passes<T, D, M_F16, 2>(X, n, d, cs, Rsw, r, lb, le, S, s, bt, nb)
                   : launch_passes<T, D, M_F16, 1>(X, n, d, cs, Rsw, r, lb, le, S, s, bt, nb);
    else
        split == 2 ? launch_passes<T, D, M_BF16, 2>(X, n, d, cs, Rsw, r, lb, le, S, s, bt, nb)
                   : launch_passes<T, D, M_BF16, 1>(X, n, d, cs, Rsw, r, lb, le, S, s, bt, nb);
}

template <class T>
void dispatch_d(const T *X, int64_t n, int d, float cs, const void *Rsw, int r, const int32_t *lb, const int32_t *le,
                float *S, int prec, int split, hipStream_t s, const SampBlock *bt, int64_t nb) {
    if (d <= 8)
        dispatch_mode<T, 8>(X, n, d, cs, Rsw, r, lb, le, S, prec, split, s, bt, nb);
    else if (d <= 16)
        dispatch_mode<T, 16>(X, n, d, cs, Rsw, r, lb, le, S, prec, split, s, bt, nb);
    else if (d <= 32)
        dispatch_mode<T, 32>(X, n, d, cs, Rsw, r, lb, le, S, prec, split, s, bt, nb);
    else
        dispatch_mode<T, 64>(X, n, d, cs, Rsw, r, lb, le, S, prec, split, s, bt, nb);
}


// ------------------------------------------------------ wide points (d > 64)
//
// For wide points the augmented coordinates no longer fit in registers, so
// the exponents are an ordinary GEMM on the matrix cores: a workgroup owns
// 128 rows (4 waves x 32) and walks the points in panels of 128 (4 tiles of
// 32); per panel it accumulates t = x~_i . y~_j over the K = d + 2 augmented
// coordinates in chunks of 64 staged through LDS (v_mfma_f32_32x32x2_f32,
// points as A rows, the wave's rows as B columns: the C layout is the one
// exp_split turns into the FP16 / BF16 A operands), then applies exp2, the
// split and the products with the panel's random block as in k_sample_mfma.
// The coordinates are centred on the mean point (x' = x - mean) and prepared
// once per call: XA_i = (2 c x'_i, -c |x'_i|^2 (+14 in FP16 mode), 1, 0..),
// YA_j = (x'_j, 1, -c |x'_j|^2, 0..), rows of KP floats, c per problem.
constexpr int WW = 4;            // waves per workgroup (wide kernel)
constexpr int WROWS = 32 * WW;   // rows per workgroup
constexpr int WPT = 4;           // point tiles per panel
constexpr int WKC = 64;          // augmented coordinates per LDS chunk
constexpr int WRB = 4;           // 32-column blocks per pass

// Kernel entries of one 32-point tile from its exponents, masking the row's
// own leaf and points outside the row's problem [jlo, jhi).
template <int MODE, int TERMS>
__device__ __forceinline__ void exp_split_range(typename Op<MODE>::V (&ahi)[2], typename Op<MODE>::V (&alo)[2],
                                                const f16v &t, int g, int64_t jt, int32_t my_lb, int32_t my_le,
                                                int64_t jlo, int64_t jhi) {
    typedef typename Op<MODE>::H H;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        float e = __builtin_amdgcn_exp2f(t[r]);
        const int64_t j = jt + 8 * (r >> 2) + 4 * g + (r & 3);
        e = (j < jlo || j >= jhi || (j >= my_lb && j < my_le)) ? 0.0f : e;
        const H hi = (H)e;
        ahi[r >> 3][r & 7] = hi;
        if (TERMS == 2) alo[r >> 3][r & 7] = (H)(e - (float)hi);
    }
}

template <int MODE, int TERMS>
__global__ __launch_bounds__(64 * WW) void k_sample_wide(const float *__restrict__ XA, const float *__restrict__ YA,
                                                         int KP, int64_t n, const void *__restrict__ Rsw_, int RBt,
                                                         const int32_t *__restrict__ lb,
                                                         const int32_t *__restrict__ le, float *__restrict__ S,
                                                         int ldS, const SampBlock *__restrict__ bt) {
    typedef typename Op<MODE>::V V;
    constexpr int TH = 64 * WW;
    constexpr int LDK = WKC + 1;
    // x~ / y~ chunks during the exponent GEMM, then the panel's random block
    __shared__ __attribute__((aligned(16))) float lds[2 * WROWS * LDK];
    float(*xs)[LDK] = reinterpret_cast<float(*)[LDK]>(lds);
    float(*ys)[LDK] = reinterpret_cast<float(*)[LDK]>(lds + WROWS * LDK);
    const V *rl = reinterpret_cast<const V *>(lds);

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 5;
    const int cb0 = blockIdx.y * WRB;
    int64_t i0, iend, jlo, jhi;
    if (bt) {
        const SampBlock sb = bt[blockIdx.x];
        i0 = sb.i0;
        iend = sb.iend;
        jlo = sb.jlo;
        jhi = sb.jhi;
    } else {
        i0 = (int64_t)blockIdx.x * WROWS;
        iend = n;
        jlo = 0;
        jhi = n;
    }
    const int64_t i = i0 + 32 * w + (lane & 31);
    const bool row_ok = i < iend;
    const int32_t my_lb = (row_ok && lb) ? lb[i] : 0;
    const int32_t my_le = (row_ok && lb) ? le[i] : 0;
    constexpr float kInvScale = MODE == M_F16 ? 1.0f / 16384.0f : 1.0f;
    const char *Rg = static_cast<const char *>(Rsw_);
    constexpr int TILE_B = 2 * 64 * 16;  // bytes of one (tile, column block) of the FP16 / BF16 layout
    f16v acc[WRB];
#pragma unroll
    for (int c = 0; c < WRB; ++c)
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[c][q] = 0.0f;

    for (int64_t p0 = (jlo / 32) * 32; p0 < jhi; p0 += 32 * WPT) {
        f16v t[WPT];
#pragma unroll
        for (int pt = 0; pt < WPT; ++pt)
#pragma unroll
            for (int q = 0; q < 16; ++q) t[pt][q] = 0.0f;
        for (int kc = 0; kc < KP; kc += WKC) {
            for (int u = tid; u < WROWS * WKC; u += TH) {
                const int rr = u / WKC, kk = u % WKC;
                const int64_t gi = i0 + rr, gj = p0 + rr;
                xs[rr][kk] = gi < iend ? XA[gi * KP + kc + kk] : 0.0f;
                ys[rr][kk] = gj < jhi ? YA[gj * KP + kc + kk] : 0.0f;
            }
            __syncthreads();
#pragma unroll 4
            for (int s2 = 0; s2 < WKC / 2; ++s2) {
                const int kk = 2 * s2 + g;
                const float b = xs[32 * w + (lane & 31)][kk];
#pragma unroll
                for (int pt = 0; pt < WPT; ++pt)
                    t[pt] = __builtin_amdgcn_mfma_f32_32x32x2f32(ys[32 * pt + (lane & 31)][kk], b, t[pt], 0, 0, 0);
            }
            __syncthreads();
        }
        // the panel's random block (WPT tiles x WRB column blocks) into LDS
        {
            const int pieces = WPT * WRB * TILE_B / 16;
            uint4 *dst = reinterpret_cast<uint4 *>(lds);
            for (int u = tid; u < pieces; u += TH) {
                const int per = WRB * TILE_B / 16, pt = u / per, rem = u % per, c = rem / (TILE_B / 16);
                const uint4 *src = reinterpret_cast<const uint4 *>(
                    Rg + ((p0 / 32 + pt) * (int64_t)RBt + cb0) * TILE_B);
                // column blocks past the last one (a ragged final pass) read as zeros
                dst[u] = cb0 + c < RBt ? src[rem] : make_uint4(0u, 0u, 0u, 0u);
            }
            __syncthreads();
        }
#pragma unroll
        for (int pt = 0; pt < WPT; ++pt) {
            V hi[2], lo[2];
            exp_split_range<MODE, TERMS>(hi, lo, t[pt], g, p0 + 32 * pt, my_lb, my_le, jlo, jhi);
#pragma unroll
            for (int c = 0; c < WRB; ++c)
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    const V b = rl[((pt * WRB + c) * 2 + kb) * 64 + lane];
                    acc[c] = Op<MODE>::mfma(hi[kb], b, acc[c]);
                    if (TERMS == 2) acc[c] = Op<MODE>::mfma(lo[kb], b, acc[c]);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < WRB; ++c)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int m = 8 * (q >> 2) + 4 * g + (q & 3);
            const int64_t row = i0 + 32 * w + m;
            if (row < iend && cb0 + c < RBt) S[row * ldS + 32 * (cb0 + c) + (lane & 31)] = acc[c][q] * kInvScale;
        }
}

}  // namespace

constexpr int kSampleMfmaMaxD = 64;

namespace {

template <int MODE, int TERMS>
void launch_wide(dim3 grid, const float *XA, const float *YA, int KP, int64_t n, const void *Rsw, int RBt,
                 const int32_t *lb, const int32_t *le, float *S, int ldS, const SampBlock *bt, hipStream_t s) {
    k_sample_wide<MODE, TERMS><<<grid, 64 * WW, 0, s>>>(XA, YA, KP, n, Rsw, RBt, lb, le, S, ldS, bt);
    check_launch("k_sample_wide");
}

// Split-mode sampling of points wider than the register-resident kernel.
void sample_wide(const float *X, int64_t n, int d, double h, const void *Rsw, int r, const int32_t *lb,
                 const int32_t *le, float *S, int prec, int split, hipStream_t s, const Batch *batch) {
    const int KP = (d + 2 + WKC - 1) / WKC * WKC;
    const double c2 = 1.4426950408889634 / (2.0 * h * h);
    DBuf mean = dalloc<double>(d), XA = dalloc<float>((size_t)n * KP), YA = dalloc<float>((size_t)n * KP);
    DBuf pb, cp, bt;
    int64_t nb = 0;
    std::vector<SampBlock> blocks;
    if (batch) {
        std::vector<double> cpr(batch->np());
        for (int k = 0; k < batch->np(); ++k) cpr[k] = 1.4426950408889634 / (2.0 * batch->h[k] * batch->h[k]);
        pb = upload(batch->pbeg, s);
        cp = upload(cpr, s);
        blocks = row_blocks(*batch, WROWS);
        nb = (int64_t)blocks.size();
        bt = upload(blocks, s);
        sync(s);
    }
    k_col_mean<float><<<d, 256, 0, s>>>(X, n, d, mean.as<double>());
    check_launch("k_col_mean");
    const float off = prec == KRR_F16_SPLIT ? 14.0f : 0.0f;  // FP16 entries carry a 2^14 scale
    k_wide_aug<<<(unsigned)n, 256, 0, s>>>(X, n, d, KP, mean.as<double>(), c2, pb.as<int64_t>(), cp.as<double>(),
                                          batch ? batch->np() : 0, off, 0, XA.as<float>());
    check_launch("k_wide_aug");
    k_wide_aug<<<(unsigned)n, 256, 0, s>>>(X, n, d, KP, mean.as<double>(), c2, pb.as<int64_t>(), cp.as<double>(),
                                          batch ? batch->np() : 0, off, 1, YA.as<float>());
    check_launch("k_wide_aug");
    const int RBt = r / 32;
    dim3 grid((unsigned)(batch ? nb : ceil_div(n, WROWS)), ceil_div(RBt, WRB));
    const SampBlock *b = bt.as<SampBlock>();
    if (prec == KRR_F16_SPLIT)
        split == 2 ? launch_wide<M_F16, 2>(grid, XA.as<float>(), YA.as<float>(), KP, n, Rsw, RBt, lb, le, S, r, b, s)
                   : launch_wide<M_F16, 1>(grid, XA.as<float>(), YA.as<float>(), KP, n, Rsw, RBt, lb, le, S, r, b, s);
    else
        split == 2 ? launch_wide<M_BF16, 2>(grid, XA.as<float>(), YA.as<float>(), KP, n, Rsw, RBt, lb, le, S, r, b, s)
                   : launch_wide<M_BF16, 1>(grid, XA.as<float>(), YA.as<float>(), KP, n, Rsw, RBt, lb, le, S, r, b, s);
    sync(s);  // the prepared coordinates are released on return
}

}  // namespace

bool sample_mfma_supported(int d, int prec) {
    // FP32 entries of wide points stay on the vector ALUs; the split modes of
    // any width run on the matrix cores
    return prec != KRR_F64 && (d <= kSampleMfmaMaxD || prec != KRR_F32);
}

// R: n x r FP32 (exact in the operand precision); S: n x r FP32.
void sample_mfma(const void *X, int64_t n, int d, int xprec, double h, const float *R, int r, const int32_t *lb,
                 const int32_t *le, float *S, int prec, int split, hipStream_t s, const Batch *batch) {
    // zero tiles past the end keep every prefetch in bounds: two for the
    // narrow kernel, a whole panel for the wide one
    const int64_t tiles = (n + JT - 1) / JT + WPT;
    const float cs = (float)(1.4426950408889634 / (2.0 * h * h));
    DBuf Rsw;
    if (prec == KRR_F32) {
        Rsw.alloc(sizeof(float) * tiles * 32 * r);
        int64_t tot = tiles * (r / 32) * 16 * 64;
        k_swizzle_f<<<ceil_div(tot, 256), 256, 0, s>>>(R, n, r, tiles, Rsw.as<float>());
    } else {
        Rsw.alloc(2 * tiles * 32 * r);
        int64_t tot = tiles * (r / 32) * 2 * 64;
        if (prec == KRR_F16_SPLIT)
            k_swizzle_h<_Float16><<<ceil_div(tot, 256), 256, 0, s>>>(R, n, r, tiles, Rsw.as<_Float16>());
        else
            k_swizzle_h<__bf16><<<ceil_div(tot, 256), 256, 0, s>>>(R, n, r, tiles, Rsw.as<__bf16>());
    }
    check_launch("k_swizzle");
    DBuf Xf;
    const float *Xs = static_cast<const float *>(X);
    if (xprec == KRR_F64) {
        Xf.alloc(sizeof(float) * n * d);
        k_to_float<<<ceil_div(n * d, 256), 256, 0, s>>>(static_cast<const double *>(X), n * d, Xf.as<float>());
        check_launch("k_to_float");
        Xs = Xf.as<float>();
    }
    DBuf bt;
    int64_t nb = 0;
    if (batch) {
        std::vector<SampBlock> blocks = row_blocks(*batch, ROWS);
        nb = (int64_t)blocks.size();
        bt = upload(blocks, s);
        sync(s);  // `blocks` is released on return from this scope
    }
    if (d > kSampleMfmaMaxD) {
        sample_wide(Xs, n, d, h, Rsw.get(), r, lb, le, S, prec, split, s, batch);
        sync(s);  // Rsw is released on return
        return;
    }
    dispatch_d<float>(Xs, n, d, cs, Rsw.get(), r, lb, le, S, prec, split, s, bt.as<SampBlock>(), nb);
    sync(s);  // Rsw and the block table are released on return
}

}  // namespace krr
