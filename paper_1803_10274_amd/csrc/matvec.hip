// Gaussian-kernel products without storing K (eq. (1.1)):
//   * kernel_matvec: Out = K(X, Y; h) W for a few right-hand sides; FP64
//     entries from exact coordinate differences, FP32 entries from an FP64
//     norm expansion of the exponent; FP32 sums over a 64-column tile and
//     FP64 across tiles;
//   * the tiled VALU sampling product S = K R with each row's own leaf block
//     removed (Section 3.1 randomized construction), used for FP64 samples
//     and as the portable reference of the matrix-core sampler;
//   * small helpers: the +-1 random block, row gather / scatter, column dots.
#include "internal.hpp"

namespace krr {

// ------------------------------------------------------------------ exp

__device__ __forceinline__ float kexp(float q, float s2) {
    // exp(-q / (2 h^2)) = exp2(-q * log2(e) / (2 h^2)); v_exp_f32
    return __builtin_amdgcn_exp2f(-q * s2);
}
__device__ __forceinline__ double kexp(double q, double s) { return exp(-q * s); }

template <class C> C kernel_scale(double h);
template <> float kernel_scale<float>(double h) { return (float)(1.4426950408889634 / (2.0 * h * h)); }
// the FP64 exponent of the FP32-entry expansion kernel keeps c in FP64
inline double kernel_scale_log2(double h) { return 1.4426950408889634 / (2.0 * h * h); }
template <> double kernel_scale<double>(double h) { return 1.0 / (2.0 * h * h); }

// ---------------------------------------------------------- kernel_matvec

namespace {
constexpr int MV_ROWS = 256;
constexpr int MV_TN = 64;

// part[(split * m + i) * nrhs + rhs0 + r] = sum over the split's columns.
template <class T, class C, int D, int NR>
__global__ __launch_bounds__(MV_ROWS) void k_kmv(const T *__restrict__ X, int64_t m,
                                                 const T *__restrict__ Y, int64_t n, int d, C scale,
                                                 const double *__restrict__ W, int nrhs, int rhs0,
                                                 int64_t cols_per_split, double *__restrict__ part,
                                                 const SampBlock *__restrict__ bt) {
    __shared__ C ys[MV_TN][D];
    __shared__ C ws[MV_TN][NR];
    const int tid = threadIdx.x;
    const int split = blockIdx.y;
    int64_t i, iend, j0, j1;
    if (bt) {
        const SampBlock sb = bt[blockIdx.x];
        i = sb.i0 + tid;
        iend = sb.iend;
        j0 = sb.jlo + split * sb.cps;
        j1 = min(sb.jhi, j0 + sb.cps);
        if constexpr (sizeof(C) == 8) scale = sb.inv; else scale = sb.cs;
    } else {
        i = (int64_t)blockIdx.x * MV_ROWS + tid;
        iend = m;
        j0 = split * cols_per_split;
        j1 = min(n, j0 + cols_per_split);
    }
    C x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = (i < iend && k < d) ? (C)X[i * d + k] : (C)0;
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = 0.0;
    const int nr = min(NR, nrhs - rhs0);
    for (int64_t jt = j0; jt < j1; jt += MV_TN) {
        for (int t = tid; t < MV_TN * D; t += MV_ROWS) {
            int jj = t / D, k = t % D;
            int64_t j = jt + jj;
            ys[jj][k] = (j < j1 && k < d) ? (C)Y[j * d + k] : (C)0;
        }
        for (int t = tid; t < MV_TN * NR; t += MV_ROWS) {
            int jj = t / NR, r = t % NR;
            int64_t j = jt + jj;
            ws[jj][r] = (j < j1 && r < nr) ? (C)W[j * nrhs + rhs0 + r] : (C)0;
        }
        __syncthreads();
        C pacc[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) pacc[r] = (C)0;
        for (int jj = 0; jj < MV_TN; ++jj) {
            C q = (C)0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                C t = x[k] - ys[jj][k];
                q = fma(t, t, q);
            }
            C kv = kexp(q, scale);
#pragma unroll
            for (int r = 0; r < NR; ++r) pacc[r] = fma(kv, ws[jj][r], pacc[r]);
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] += (double)pacc[r];
        __syncthreads();
    }
    if (i < iend) {
        for (int r = 0; r < nr; ++r) part[((int64_t)split * m + i) * nrhs + rhs0 + r] = acc[r];
    }
}

// FP32-entry mode for d <= 64.  The exponent is the FP64 norm expansion
// t = -c |x_i|^2 + (-c |y_j|^2 + sum_k x_ik (2 c y_jk)) (c in log2 units), with
// the column terms prepared once per product (ya, LDP doubles per column) and
// staged per 64-column tile in LDS; FP64 FMAs cost the same as FP32 ones here
// and keep the expansion free of cancellation trouble.  The entry is exp2 of
// t rounded to FP32 (t = -inf past the end of the tile: entry 0); products and
// the tile sum are FP32, sums across tiles FP64.  Each thread owns RPT rows,
// so that every broadcast LDS read of a column serves RPT entries (a wave's
// LDS reads return one copy per lane and would otherwise bound the loop).
template <int D> struct ColLd { static constexpr int V = (D + 2) & ~1; };

// QM: the entry is exp2(t) t instead of exp2(t) (K o T in log2 units: the
// h-derivative of the kernel up to a constant, for the fused backward's dh).
template <class T, int D, int NR, int RPT, bool QM = false>
__global__ __launch_bounds__(MV_ROWS) void k_kmv_sc(const T *__restrict__ X, int64_t m, int d, double c2,
                                                    const double *__restrict__ ya, const float *__restrict__ wf,
                                                    int nrhs, int rhs0, int64_t n, int64_t cols_per_split,
                                                    double *__restrict__ part, const SampBlock *__restrict__ bt) {
    constexpr int LD = ColLd<D>::V;
    __shared__ __attribute__((aligned(16))) double ys[MV_TN][LD];
    __shared__ float ws[MV_TN][NR];
    const int tid = threadIdx.x;
    const int split = blockIdx.y;
    int64_t i0, iend, j0, j1;
    if (bt) {
        const SampBlock sb = bt[blockIdx.x];
        i0 = sb.i0;
        iend = sb.iend;
        j0 = sb.jlo + split * sb.cps;
        j1 = min(sb.jhi, j0 + sb.cps);
        c2 = sb.c2;
    } else {
        i0 = (int64_t)blockIdx.x * (MV_ROWS * RPT);
        iend = m;
        j0 = split * cols_per_split;
        j1 = min(n, j0 + cols_per_split);
    }
    double xs[RPT][D];
    double nx[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t i = i0 + tid + (int64_t)MV_ROWS * q;
        double a = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double v = (i < iend && k < d) ? (double)X[i * d + k] : 0.0;
            a = fma(v, v, a);
            xs[q][k] = v;
        }
        nx[q] = -c2 * a;
    }
    double acc[RPT][NR];
#pragma unroll
    for (int q = 0; q < RPT; ++q)
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[q][r] = 0.0;
    for (int64_t jt = j0; jt < j1; jt += MV_TN) {
        const int64_t cnt = min((int64_t)MV_TN, j1 - jt);
        const double *src = ya + jt * LD;
        for (int t = tid; t < MV_TN * LD; t += MV_ROWS) {
            const int jj = t / LD, k = t % LD;
            ys[jj][k] = jj < cnt ? src[t] : (k == D ? -INFINITY : 0.0);
        }
        for (int t = tid; t < MV_TN * NR; t += MV_ROWS) {
            const int jj = t / NR, r = t % NR;
            ws[jj][r] = jj < cnt ? wf[(jt + jj) * nrhs + rhs0 + r] : 0.0f;
        }
        __syncthreads();
        float pacc[RPT][NR];
#pragma unroll
        for (int q = 0; q < RPT; ++q)
#pragma unroll
            for (int r = 0; r < NR; ++r) pacc[q][r] = 0.0f;
        for (int jj = 0; jj < MV_TN; ++jj) {
            double yv[D + 1];
#pragma unroll
            for (int k = 0; k <= D; ++k) yv[k] = ys[jj][k];
            float wv[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) wv[r] = ws[jj][r];
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                double t = nx[q] + yv[D];
#pragma unroll
                for (int k = 0; k < D; ++k) t = fma(xs[q][k], yv[k], t);
                const float tf = (float)t;
                float kv = __builtin_amdgcn_exp2f(tf);
                if (QM) kv = kv == 0.0f ? 0.0f : kv * tf;  // t = -inf past the tile: entry 0
#pragma unroll
                for (int r = 0; r < NR; ++r) pacc[q][r] = fmaf(kv, wv[r], pacc[q][r]);
            }
        }
#pragma unroll
        for (int q = 0; q < RPT; ++q)
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[q][r] += (double)pacc[q][r];
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t i = i0 + tid + (int64_t)MV_ROWS * q;
        if (i < iend)
            for (int r = 0; r < NR; ++r) part[((int64_t)split * m + i) * nrhs + rhs0 + r] = acc[q][r];
    }
}

// Rows per thread of k_kmv_sc by width (register budget).
constexpr int sc_rpt(int D) { return D <= 16 ? 4 : (D <= 24 ? 3 : (D <= 32 ? 2 : 1)); }

// ------------------------------------------------ symmetric kernel product
//
// y = K(X, X) w uses K's symmetry: the entries right of each row block's
// diagonal block are evaluated once and used twice, for the block's rows
// (row sums, as in k_kmv_sc) and for the columns (column sums reduced across
// the workgroup's rows).  An item is one row block (RPT * 256 rows) against
// one chunk of columns right of its diagonal block, inside its problem.
// Row partials go to rowpart[chunk][row] (FP64), column partials to
// colpart[block][column] (FP32: a 256-term tree sum per block and column), and
// k_sym_reduce adds them in a fixed order with the diagonal blocks' products.
struct SymItem {
    int64_t i0, iend, j0, j1;
    int64_t blk, chunk;
    double c2;
    int64_t mid;  // index of the item's words in a negligible-tile map (stable across a batch's skips)
};

template <class T, int D, int NR, int RPT>
__global__ __launch_bounds__(MV_ROWS) void k_kmv_sym(const T *__restrict__ X, int d, const double *__restrict__ ya,
                                                     const float *__restrict__ wf, int nrhs, int64_t n,
                                                     const SymItem *__restrict__ items, double *__restrict__ rowpart,
                                                     float *__restrict__ colpart) {
    constexpr int LD = ColLd<D>::V;
    constexpr int NW = MV_ROWS / 64;
    __shared__ __attribute__((aligned(16))) double ys[MV_TN][LD];
    __shared__ float ws[MV_TN][NR];
    __shared__ float csum[NW][NR][64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const SymItem it = items[blockIdx.x];
    const double c2 = it.c2;
    double xs[RPT][D];
    double nx[RPT];
    float wi[RPT][NR];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t i = it.i0 + tid + (int64_t)MV_ROWS * q;
        const bool ok = i < it.iend;
        double a = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double v = (ok && k < d) ? (double)X[i * d + k] : 0.0;
            a = fma(v, v, a);
            xs[q][k] = v;
        }
        nx[q] = -c2 * a;
#pragma unroll
        for (int r = 0; r < NR; ++r) wi[q][r] = ok ? wf[i * nrhs + r] : 0.0f;
    }
    double acc[RPT][NR];
#pragma unroll
    for (int q = 0; q < RPT; ++q)
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[q][r] = 0.0;
    for (int64_t jt = it.j0; jt < it.j1; jt += MV_TN) {
        const int64_t cnt = min((int64_t)MV_TN, it.j1 - jt);
        const double *src = ya + jt * LD;
        for (int t = tid; t < MV_TN * LD; t += MV_ROWS) {
            const int jj = t / LD, k = t % LD;
            ys[jj][k] = jj < cnt ? src[t] : (k == D ? -INFINITY : 0.0);
        }
        for (int t = tid; t < MV_TN * NR; t += MV_ROWS) {
            const int jj = t / NR, r = t % NR;
            ws[jj][r] = jj < cnt ? wf[(jt + jj) * nrhs + r] : 0.0f;
        }
        __syncthreads();
        float pacc[RPT][NR];
#pragma unroll
        for (int q = 0; q < RPT; ++q)
#pragma unroll
            for (int r = 0; r < NR; ++r) pacc[q][r] = 0.0f;
        // columns in groups of 8: this lane's rows' contributions to each column
        // of the group are summed across the wave (reduce-scatter inside each
        // 8-lane group, then across the groups), leaving column jg + (l & 7) in
        // lane l; the four waves' sums meet in LDS
#pragma unroll 1
        for (int jg = 0; jg < MV_TN; jg += 8) {
            float cacc[8][NR];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int jj = jg + u;
                double yv[D + 1];
#pragma unroll
                for (int k = 0; k <= D; ++k) yv[k] = ys[jj][k];
                float wv[NR];
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    wv[r] = ws[jj][r];
                    cacc[u][r] = 0.0f;
                }
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    double t = nx[q] + yv[D];
#pragma unroll
                    for (int k = 0; k < D; ++k) t = fma(xs[q][k], yv[k], t);
                    const float kv = __builtin_amdgcn_exp2f((float)t);
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        pacc[q][r] = fmaf(kv, wv[r], pacc[q][r]);
                        cacc[u][r] = fmaf(kv, wi[q][r], cacc[u][r]);
                    }
                }
            }
#pragma unroll
            for (int o = 4; o >= 1; o >>= 1) {
                const bool up = (lane & o) != 0;
#pragma unroll
                for (int kk = 0; kk < o; ++kk)
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        const float a = cacc[kk][r], b = cacc[kk + o][r];
                        const float send = up ? a : b;
                        cacc[kk][r] = (up ? b : a) + __shfl_xor(send, o, 64);
                    }
            }
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                float v = cacc[0][r];
                v += __shfl_xor(v, 8, 64);
                v += __shfl_xor(v, 16, 64);
                v += __shfl_xor(v, 32, 64);
                if (lane < 8) csum[wv][r][jg + lane] = v;
            }
        }
#pragma unroll
        for (int q = 0; q < RPT; ++q)
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[q][r] += (double)pacc[q][r];
        __syncthreads();
        if (wv == 0 && lane < cnt) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                float c = csum[0][r][lane];
#pragma unroll
                for (int w = 1; w < NW; ++w) c += csum[w][r][lane];
                colpart[((int64_t)it.blk * n + jt + lane) * NR + r] = c;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t i = it.i0 + tid + (int64_t)MV_ROWS * q;
        if (i < it.iend)
            for (int r = 0; r < NR; ++r) rowpart[((int64_t)it.chunk * n + i) * NR + r] = acc[q][r];
    }
}

// The same items with the FP64 exponents on the matrix cores.  Per 16 x 16
// tile, v_mfma_f64_16x16x4_f64 multiplies 16 points (A: 2 c y_p, D / 4
// k-steps) into 16 rows (B: x_r) on top of the rows' constant -c |x_r|^2
// (the C operand); the points' constant -c |y_p|^2 enters through a spare k
// slot when d < D (A holds it, B a one), else as one FP64 add per entry.  The
// vector ALUs are left with the FP32 entry (convert, exp2) and its two uses.
// (On gfx950 the matrix-core and vector work of a SIMD do not overlap, and
// FP64 matrix throughput equals FP64 vector throughput, so the gain is the
// removed per-entry adds and LDS traffic: measured 3% at d = 8, 30% at
// d = 18 for one right-hand side, none for two.)  A wave owns RT row tiles of 16;
// in the FP64 C layout register q of lane l holds row l % 16 of the row tile
// against point l / 16 + 4 q of the point tile, so row sums stay in the lane
// (the four quarters are added at the end) and column sums are reduced
// across the 16 lanes of a quarter, then across the waves in LDS.  Entries
// and their tile sums are FP32 over a panel of SM_PN points (SM_PN / 4 terms
// per lane and row), FP64 across panels.
constexpr int SM_WAVES = 8;
constexpr int SM_PN = 256;  // points per staged panel
constexpr int symm_rt(int D) { return D <= 8 ? 8 : 4; }  // row tiles per wave (registers)
constexpr int symm_rows(int D) { return 16 * SM_WAVES * symm_rt(D); }

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <int D, bool PCK>
__global__ __launch_bounds__(64 * SM_WAVES) void k_kmv_symm(const float *__restrict__ X, int d,
                                                            const double *__restrict__ ya,
                                                            const float *__restrict__ wf, int64_t n,
                                                            const SymItem *__restrict__ items,
                                                            double *__restrict__ rowpart, float *__restrict__ colpart) {
    constexpr int NR = 1;  // one right-hand side (two take the vector form)
    constexpr int RT = symm_rt(D);
    constexpr int KS = D / 4;  // k-steps of 4
    constexpr int LDG = ColLd<D>::V;  // the column data's stride (k_col_aug)
    constexpr int LD = D + 1;         // staged point: 2 c y (D slots), -c |y|^2
    constexpr int TH = 64 * SM_WAVES;
    __shared__ double ys[SM_PN * LD];
    __shared__ float ws[SM_PN][NR];
    __shared__ float csum[SM_WAVES][SM_PN][NR];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = lane >> 4, lr = lane & 15;
    const SymItem it = items[blockIdx.x];
    const double c2 = it.c2;
    double xb[RT][KS];
    d4v rc[RT];
    float wi[RT][NR];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t i = it.i0 + (int64_t)(wv * RT + rt) * 16 + lr;
        const bool ok = i < it.iend;
        double nrm = 0.0;
        if (ok)
            for (int k = 0; k < d; ++k) {
                const double v = (double)X[i * d + k];
                nrm = fma(v, v, nrm);
            }
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int k = g + 4 * s;
            xb[rt][s] = !ok ? 0.0 : (k < d ? (double)X[i * d + k] : ((PCK && k == d) ? 1.0 : 0.0));
        }
        const double r0 = ok ? -c2 * nrm : 0.0;
        rc[rt] = d4v{r0, r0, r0, r0};
#pragma unroll
        for (int r = 0; r < NR; ++r) wi[rt][r] = ok ? wf[i * NR + r] : 0.0f;
    }
    double acc[RT][NR];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[rt][r] = 0.0;
    for (int64_t p0 = it.j0; p0 < it.j1; p0 += SM_PN) {
        const int cnt = (int)min((int64_t)SM_PN, it.j1 - p0);
        // stage the panel; points past the item get zero coordinates and a
        // constant of -1e300 (entry 0 for every row, no infinities in the GEMM)
        for (int u = tid; u < SM_PN * LD; u += TH) {
            const int pp = u / LD, k = u % LD;
            const bool cst = k == D || (PCK && k == d);
            double v;
            if (pp < cnt) {
                const double *row = ya + (p0 + pp) * LDG;
                v = cst ? row[D] : row[k];
            } else {
                v = cst ? -1e300 : 0.0;
            }
            ys[u] = v;
        }
        for (int u = tid; u < SM_PN * NR; u += TH) {
            const int pp = u / NR, r = u % NR;
            ws[pp][r] = pp < cnt ? wf[(p0 + pp) * NR + r] : 0.0f;
        }
        __syncthreads();
        float pacc[RT][NR];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < NR; ++r) pacc[rt][r] = 0.0f;
#pragma unroll 1
        for (int tl = 0; tl < SM_PN / 16; ++tl) {
            const int pb = tl * 16 + g;  // this quarter's points: pb + 4 q
            double a[KS];
#pragma unroll
            for (int s = 0; s < KS; ++s) a[s] = ys[(tl * 16 + lr) * LD + g + 4 * s];
            double pq[4];
            float wp[4][NR];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                pq[q] = PCK ? 0.0 : ys[(pb + 4 * q) * LD + D];
#pragma unroll
                for (int r = 0; r < NR; ++r) wp[q][r] = ws[pb + 4 * q][r];
            }
            float cacc[4][NR];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < NR; ++r) cacc[q][r] = 0.0f;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                d4v t = rc[rt];
#pragma unroll
                for (int s = 0; s < KS; ++s) t = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], xb[rt][s], t, 0, 0, 0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double tq = PCK ? t[q] : t[q] + pq[q];
                    const float e = __builtin_amdgcn_exp2f((float)tq);
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        pacc[rt][r] = fmaf(e, wp[q][r], pacc[rt][r]);
                        cacc[q][r] = fmaf(e, wi[rt][r], cacc[q][r]);
                    }
                }
            }
            // column sums over the quarter's 16 lanes: reduce-scatter over
            // lane bits 3 and 2 (leaving point q = 2 b3 + b2), then add over
            // bits 1 and 0
#pragma unroll
            for (int o = 8, h = 2; o >= 4; o >>= 1, h >>= 1) {
                const bool up = (lane & o) != 0;
#pragma unroll
                for (int kk = 0; kk < h; ++kk)
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        const float lo = cacc[kk][r], hi = cacc[kk + h][r];
                        const float send = up ? lo : hi;
                        cacc[kk][r] = (up ? hi : lo) + __shfl_xor(send, o, 64);
                    }
            }
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                float v = cacc[0][r];
                v += __shfl_xor(v, 2, 64);
                v += __shfl_xor(v, 1, 64);
                if ((lane & 3) == 0) csum[wv][pb + 4 * ((lane >> 2) & 3)][r] = v;
            }
        }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[rt][r] += (double)pacc[rt][r];
        __syncthreads();
        // the waves' column sums; the next panel's staging touches ys / ws only
        for (int u = tid; u < cnt * NR; u += TH) {
            const int pp = u / NR, r = u % NR;
            float c = csum[0][pp][r];
#pragma unroll
            for (int w = 1; w < SM_WAVES; ++w) c += csum[w][pp][r];
            colpart[((int64_t)it.blk * n + p0 + pp) * NR + r] = c;
        }
    }
    // row sums: the four quarters hold the same rows
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t i = it.i0 + (int64_t)(wv * RT + rt) * 16 + lr;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            double v = acc[rt][r];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            if (g == 0 && i < it.iend) rowpart[((int64_t)it.chunk * n + i) * NR + r] = v;
        }
    }
}

// Per row block of the symmetric product (problem order).
struct SymBlock {
    int64_t i0, iend;
    int64_t first_blk;           // the problem's first block
    int64_t chunk_lo, chunk_hi;  // chunks holding this block's row partials
};

// Out[i] = diag[i] + sum of the row partials of i's block + the column
// partials of i from the earlier blocks of its problem (+ beta Out[i]).
template <int NR>
__global__ void k_sym_reduce(const SymBlock *__restrict__ blocks, int rows_pb, const double *__restrict__ diag,
                             const double *__restrict__ rowpart, const float *__restrict__ colpart, int64_t n,
                             double beta, double *__restrict__ out) {
    const SymBlock b = blocks[blockIdx.y];
    const int64_t i = b.i0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b.iend) return;
    const int64_t blk = blockIdx.y;
    double s[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) s[r] = diag[i * NR + r];
    for (int64_t c = b.chunk_lo; c < b.chunk_hi; ++c)
#pragma unroll
        for (int r = 0; r < NR; ++r) s[r] += rowpart[(c * n + i) * NR + r];
    for (int64_t bb = b.first_blk; bb < blk; ++bb)
#pragma unroll
        for (int r = 0; r < NR; ++r) s[r] += (double)colpart[(bb * n + i) * NR + r];
#pragma unroll
    for (int r = 0; r < NR; ++r) out[i * NR + r] = beta != 0.0 ? s[r] + beta * out[i * NR + r] : s[r];
}

// The same items with FP32 exponents on the matrix cores.  The kernel is
// translation invariant, so each item re-centres its rows and columns on its
// row block's mean point a (x' = x - a, y' = y - a, all FP32): for the pairs
// that carry weight both vectors are short and the FP32 norm expansion
// t = -c |x'|^2 + 2 c x'.y' - c |y'|^2 loses little to cancellation.
// v_mfma_f32_16x16x4_f32 forms t on top of the row constant (C operand), the
// column constant enters through a spare k slot when d < D, else as one FP32
// add.  Register q of lane l holds row l % 16 of the row tile against point
// 4 (l / 16) + q of the point tile; sums as in k_kmv_symm.
constexpr __device__ __forceinline__ int symf_point(int g, int q) { return 4 * g + q; }

template <int D, bool PCK>
__global__ __launch_bounds__(64 * SM_WAVES) void k_kmv_symf(const float *__restrict__ X, int d,
                                                            const float *__restrict__ anchors,
                                                            const float *__restrict__ wf, int64_t n,
                                                            const SymItem *__restrict__ items,
                                                            double *__restrict__ rowpart, float *__restrict__ colpart) {
    constexpr int RT = symm_rt(D);
    constexpr int KS = D / 4;  // k-steps of 4
    constexpr int LD = D + 1;  // staged point: 2 c y' (D slots), -c |y'|^2
    constexpr int TH = 64 * SM_WAVES;
    __shared__ float ys[SM_PN * LD];
    __shared__ float ws[SM_PN];
    __shared__ float csum[SM_WAVES][SM_PN];
    __shared__ float anc[D];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = lane >> 4, lr = lane & 15;
    const SymItem it = items[blockIdx.x];
    const float c = (float)it.c2;
    if (tid < D) anc[tid] = tid < d ? anchors[it.blk * d + tid] : 0.0f;
    __syncthreads();
    float xb[RT][KS];
    f4v rc[RT];
    float wi[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t i = it.i0 + (int64_t)(wv * RT + rt) * 16 + lr;
        const bool ok = i < it.iend;
        float nrm = 0.0f;
        if (ok)
            for (int k = 0; k < d; ++k) {
                const float v = X[i * d + k] - anc[k];
                nrm = fmaf(v, v, nrm);
            }
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int k = g + 4 * s;
            xb[rt][s] = !ok ? 0.0f : (k < d ? X[i * d + k] - anc[k] : ((PCK && k == d) ? 1.0f : 0.0f));
        }
        const float r0 = ok ? -c * nrm : 0.0f;
        rc[rt] = f4v{r0, r0, r0, r0};
        wi[rt] = ok ? wf[i] : 0.0f;
    }
    double acc[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) acc[rt] = 0.0;
    for (int64_t p0 = it.j0; p0 < it.j1; p0 += SM_PN) {
        const int cnt = (int)min((int64_t)SM_PN, it.j1 - p0);
        // stage the panel re-centred on the anchor; points past the item get
        // zero coordinates and a constant of -1e30 (entry 0 for every row)
        if (tid < SM_PN) {
            float *dst = ys + tid * LD;
            if (tid < cnt) {
                const float *y = X + (p0 + tid) * d;
                float nrm = 0.0f;
                for (int k = 0; k < D; ++k) {
                    const float v = k < d ? y[k] - anc[k] : 0.0f;
                    nrm = fmaf(v, v, nrm);
                    dst[k] = (2.0f * c) * v;
                }
                dst[D] = -c * nrm;
                if (PCK) dst[d] = dst[D];
            } else {
                for (int k = 0; k < D; ++k) dst[k] = 0.0f;
                dst[D] = -1e30f;
                if (PCK) dst[d] = -1e30f;
            }
            ws[tid] = tid < cnt ? wf[p0 + tid] : 0.0f;
        }
        __syncthreads();
        float pacc[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) pacc[rt] = 0.0f;
#pragma unroll 1
        for (int tl = 0; tl < SM_PN / 16; ++tl) {
            float a[KS];
#pragma unroll
            for (int s = 0; s < KS; ++s) a[s] = ys[(tl * 16 + lr) * LD + g + 4 * s];
            float pq[4], wp[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int pp = tl * 16 + symf_point(g, q);
                pq[q] = PCK ? 0.0f : ys[pp * LD + D];
                wp[q] = ws[pp];
            }
            float cacc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                f4v t = rc[rt];
#pragma unroll
                for (int s = 0; s < KS; ++s) t = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], xb[rt][s], t, 0, 0, 0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float e = __builtin_amdgcn_exp2f(PCK ? t[q] : t[q] + pq[q]);
                    pacc[rt] = fmaf(e, wp[q], pacc[rt]);
                    cacc[q] = fmaf(e, wi[rt], cacc[q]);
                }
            }
            // column sums over the quarter's 16 lanes (reduce-scatter over lane
            // bits 3 and 2, leaving q = 2 b3 + b2, then add over bits 1 and 0)
#pragma unroll
            for (int o = 8, h = 2; o >= 4; o >>= 1, h >>= 1) {
                const bool up = (lane & o) != 0;
#pragma unroll
                for (int kk = 0; kk < h; ++kk) {
                    const float lo = cacc[kk], hi = cacc[kk + h];
                    const float send = up ? lo : hi;
                    cacc[kk] = (up ? hi : lo) + __shfl_xor(send, o, 64);
                }
            }
            float v = cacc[0];
            v += __shfl_xor(v, 2, 64);
            v += __shfl_xor(v, 1, 64);
            if ((lane & 3) == 0) csum[wv][tl * 16 + symf_point(g, (lane >> 2) & 3)] = v;
        }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt] += (double)pacc[rt];
        __syncthreads();
        // the waves' column sums; the next panel's staging touches ys / ws only
        if (tid < cnt) {
            float cs = csum[0][tid];
#pragma unroll
            for (int w = 1; w < SM_WAVES; ++w) cs += csum[w][tid];
            colpart[(int64_t)it.blk * n + p0 + tid] = cs;
        }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t i = it.i0 + (int64_t)(wv * RT + rt) * 16 + lr;
        double v = acc[rt];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (g == 0 && i < it.iend) rowpart[(int64_t)it.chunk * n + i] = v;
    }
}

// The same items with the exponent GEMM on the BF16 matrix cores: each FP32
// operand (2 c y', x' and the column constant -c |y'|^2) is split into three
// BF16 terms (hi + mid + lo, 24 bits, FP32's range), and the six cross
// products down to 2^-16 (hh, hm, mh, hl, lh, mm) plus the column and row
// constants' three terms against ones are packed along K (so the C operand
// is zero and holds no registers): KT = 32 ceil((6 d + 6) / 32) slots,
// KT / 32 v_mfma_f32_16x16x32_bf16 per 16 x 16 tile instead of d / 4
// FP32 ones at a sixteenth of the rate.  Products of BF16 terms are exact in
// FP32, so the exponent carries the FP32 form's accuracy.  QM: the entry is
// exp2(t) t (as in k_kmv_sc), for the fused backward's dh.  SYM false: the
// rows are X's and the columns Y's (no column sums; the row partials of item
// chunk c at rowpart[c * n + i], n being then the number of rows).
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split3(float v, __bf16 &h, __bf16 &m, __bf16 &l) {
    h = (__bf16)v;
    const float r1 = v - (float)h;
    m = (__bf16)r1;
    l = (__bf16)(r1 - (float)m);
}

constexpr int symb_pn(int KT) { return KT <= 96 ? SM_PN : SM_PN / 2; }  // points per panel (LDS)
constexpr int symb_rt(int KT) { return KT <= 64 ? 8 : (KT <= 128 ? 4 : 2); }  // row tiles per wave (registers)
constexpr int symb_kt(int d) { return (6 * d + 6 + 31) / 32 * 32; }
constexpr int symb_rows(int d) { return 16 * SM_WAVES * symb_rt(symb_kt(d)); }
constexpr int symb_max_d = 31;  // KT <= 192
// Waves per SIMD the registers are budgeted for.  The symmetric form runs
// half the rectangular form's row tiles per wave (a map bit covers 16 of its
// RT rows) at four waves per SIMD: two workgroups share a CU, and one's waves
// run while the other's wait at a panel barrier (for the wave with the most
// kept tiles, with a map).  The rectangular form of wide points also fits
// four waves per SIMD without spills.
constexpr int symb_wpe(int KT, bool SYM) { return SYM || KT >= 96 ? 4 : 2; }
constexpr int symb_rt_sym(int KT) { return symb_rt(KT) > 1 ? symb_rt(KT) / 2 : 1; }
constexpr int symb_rows_sym(int d) { return 16 * SM_WAVES * symb_rt_sym(symb_kt(d)); }

// MK: the negligible-tile map (SYM only).  0 none; 1 record: every tile is
// evaluated, and each wave writes per panel the word whose bit t says that
// its 16 x 16-point tile t (all RT row tiles) holds an exponent of at least
// kSymSkipLog2 (rows and points past the item do not count); 2 use: a wave
// evaluates only the tiles whose bit is set, and a panel with no bit set in
// any wave is not staged.  The word of (item, panel p, wave w) is
// mask[(mid * ppi + p) * SM_WAVES + w].
constexpr float kSymSkipLog2 = -32.0f;
constexpr int kMapPanels = 64;  // panels per item with a map in use (the item's words fit one load per thread)
constexpr int kStageK = 8;      // coordinates per staging thread (d <= 15 at 2 threads per point, <= 31 at 4)

template <int KT, int RT, bool QM, bool SYM, int MK = 0>
__global__ __launch_bounds__(64 * SM_WAVES) __attribute__((amdgpu_waves_per_eu(symb_wpe(KT, SYM))))
void k_kmv_symb(const float *__restrict__ X, const float *__restrict__ Ycols, int d, const float *__restrict__ anchors,
                const float *__restrict__ wf, int64_t n, const SymItem *__restrict__ items,
                double *__restrict__ rowpart, float *__restrict__ colpart, uint32_t *__restrict__ mask = nullptr,
                int ppi = 0) {
    static_assert(MK == 0 || (SYM && !QM), "the tile map is for the symmetric product");
    static_assert(symb_pn(KT) / 16 <= 32, "a panel's tiles fill at most one map word");
    constexpr int KS = KT / 32;  // MFMAs per tile
    constexpr int LDB = KT + 8;  // staged point stride (BF16 elements; 16 bytes of padding)
    constexpr int PN = symb_pn(KT);
    constexpr int TH = 64 * SM_WAVES;
    __shared__ __attribute__((aligned(16))) __bf16 ys[PN * LDB];
    __shared__ float ws[PN];
    __shared__ float csum[SM_WAVES][PN];
    __shared__ float anc[32];
    __shared__ uint32_t mwl[MK == 2 ? kMapPanels * SM_WAVES : 1];  // MK 2: the item's map words
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = lane >> 4, lr = lane & 15;
    const SymItem it = items[blockIdx.x];
    const float c = (float)it.c2;
    if (tid < 32) anc[tid] = tid < d ? anchors[it.blk * d + tid] : 0.0f;
    if (MK == 2 && tid < (int)((it.j1 - it.j0 + PN - 1) / PN) * SM_WAVES)
        mwl[tid] = mask[it.mid * ppi * SM_WAVES + tid];
    __syncthreads();
    // The packed row vectors, one row tile of every wave per round: a thread
    // packs one row into the panel buffer (B side of hh, hm, mh, hl, lh, mm:
    // terms hi, mid, hi, lo, hi, mid; ones against the column constant's
    // three terms; the row constant's three terms; zero padding), then each
    // lane loads its K slots 32 s + 8 g .. + 7.  Rows past the item are zero.
    bf8v xb[RT][KS];
    float wi[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        if (tid < 16 * SM_WAVES) {
            const int64_t i = it.i0 + (int64_t)((tid >> 4) * RT + rt) * 16 + (tid & 15);
            const bool ok = i < it.iend;
            __bf16 *dst = ys + tid * LDB;
            float nrm = 0.0f;
            for (int k = 0; k < d; ++k) {
                const float v = ok ? X[i * d + k] - anc[k] : 0.0f;
                nrm = fmaf(v, v, nrm);
                __bf16 h, m, l;
                split3(v, h, m, l);
                dst[k] = h;
                dst[d + k] = m;
                dst[2 * d + k] = h;
                dst[3 * d + k] = l;
                dst[4 * d + k] = h;
                dst[5 * d + k] = m;
            }
            const __bf16 one = (__bf16)(ok ? 1.0f : 0.0f);
            dst[6 * d] = one;
            dst[6 * d + 1] = one;
            dst[6 * d + 2] = one;
            __bf16 h, m, l;
            split3(ok ? -c * nrm : 0.0f, h, m, l);
            dst[6 * d + 3] = h;
            dst[6 * d + 4] = m;
            dst[6 * d + 5] = l;
            for (int k = 6 * d + 6; k < KT; ++k) dst[k] = (__bf16)0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < KS; ++s) xb[rt][s] = *reinterpret_cast<const bf8v *>(ys + (wv * 16 + lr) * LDB + 32 * s + 8 * g);
        const int64_t i = it.i0 + (int64_t)(wv * RT + rt) * 16 + lr;
        wi[rt] = (SYM && i < it.iend) ? wf[i] : 0.0f;  // row weights: the column sums only
        __syncthreads();
    }
    double acc[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) acc[rt] = 0.0;
    // Panels are staged from registers: each thread loads its share of the
    // next panel's points (TPP threads per point, a contiguous share of the
    // coordinates, at most kStageK of them) and its weight while the current
    // panel is computed.
    constexpr int TPP = TH / PN;
    constexpr int SK = ((KT - 6) / 6 + TPP - 1) / TPP;  // coordinates per staging thread at most
    static_assert(SK <= kStageK, "a staging thread's coordinates fit its registers");
    const int pt = tid / TPP, sub = tid % TPP;
    const int kb = (d * sub) / TPP, ke = (d * (sub + 1)) / TPP;
    float pre[SK];
    float prew = 0.0f;
    // MK 2: the first panel at or after p that some wave evaluates; the
    // column partials of the panels passed over are 0
    auto visit = [&](int64_t p) {
        if (MK == 2) {
            while (p < it.j1) {
                const int pi = (int)((p - it.j0) / PN);
                uint32_t any = 0;
#pragma unroll
                for (int w = 0; w < SM_WAVES; ++w) any |= mwl[pi * SM_WAVES + w];
                if (any != 0) break;
                if (tid < PN && tid < it.j1 - p) colpart[(int64_t)it.blk * n + p + tid] = 0.0f;
                p += PN;
            }
        }
        return p;
    };
    auto fetch = [&](int64_t p) {
        const bool ok = p + pt < it.j1;
        const float *y = (SYM ? X : Ycols) + (ok ? p + pt : 0) * d;
#pragma unroll
        for (int k = 0; k < SK; ++k) pre[k] = (ok && kb + k < ke) ? y[kb + k] : 0.0f;
        prew = (ok && sub == 0) ? wf[p + pt] : 0.0f;
    };
    // the rectangular form of wide points keeps its registers for 4 waves per
    // SIMD: it loads each panel just before staging it
    constexpr bool PREF = SYM;
    bool fresh = true;  // no panel staged yet: the constant slots are still to be written
    int64_t p0 = visit(it.j0);
    if (PREF && p0 < it.j1) fetch(p0);
    while (p0 < it.j1) {
        const int cnt = (int)min((int64_t)PN, it.j1 - p0);
        const int pi = (int)((p0 - it.j0) / PN);
        // stage the panel: packed BF16 terms of 2 c y' and of the column
        // constant; points past the item get a constant of -1e30.  The
        // norm's partial sums meet by shuffles.  The slots of ones and the
        // zero padding are the same in every panel and are written with the
        // first.
        {
            __bf16 *dst = ys + pt * LDB;
            const bool ok = pt < cnt;
            float nrm = 0.0f;
            // A side of (hh, hm, mh, hl, lh, mm)
            auto put = [&](int kk, float yk) {
                const float v = ok ? yk - anc[kk] : 0.0f;
                nrm = fmaf(v, v, nrm);
                __bf16 h, m, l;
                split3((2.0f * c) * v, h, m, l);
                dst[kk] = h;
                dst[d + kk] = h;
                dst[2 * d + kk] = m;
                dst[3 * d + kk] = h;
                dst[4 * d + kk] = l;
                dst[5 * d + kk] = m;
            };
            if constexpr (PREF && SK >= 4) {
                if (ke - kb == 4 && (d & 3) == 0) {
                    // four coordinates per thread, each term group's four
                    // values 8-byte aligned: one 8-byte store per group
                    bf4v th, tm, tl;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float v = ok ? pre[k] - anc[kb + k] : 0.0f;
                        nrm = fmaf(v, v, nrm);
                        __bf16 h, m, l;
                        split3((2.0f * c) * v, h, m, l);
                        th[k] = h;
                        tm[k] = m;
                        tl[k] = l;
                    }
                    *reinterpret_cast<bf4v *>(dst + kb) = th;
                    *reinterpret_cast<bf4v *>(dst + d + kb) = th;
                    *reinterpret_cast<bf4v *>(dst + 2 * d + kb) = tm;
                    *reinterpret_cast<bf4v *>(dst + 3 * d + kb) = th;
                    *reinterpret_cast<bf4v *>(dst + 4 * d + kb) = tl;
                    *reinterpret_cast<bf4v *>(dst + 5 * d + kb) = tm;
                } else {
#pragma unroll
                    for (int k = 0; k < SK; ++k) {
                        if (kb + k >= ke) break;
                        put(kb + k, pre[k]);
                    }
                }
            } else if constexpr (PREF) {
#pragma unroll
                for (int k = 0; k < SK; ++k) {
                    if (kb + k >= ke) break;
                    put(kb + k, pre[k]);
                }
            } else {
                const float *y = (SYM ? X : Ycols) + (ok ? p0 + pt : 0) * d;
                for (int k = kb; k < ke; ++k) put(k, ok ? y[k] : 0.0f);
            }
#pragma unroll
            for (int o = 1; o < TPP; o <<= 1) nrm += __shfl_xor(nrm, o, 64);
            if (sub == 0) {
                __bf16 h, m, l;
                split3(ok ? -c * nrm : -1e30f, h, m, l);
                dst[6 * d] = h;
                dst[6 * d + 1] = m;
                dst[6 * d + 2] = l;
                if (fresh) {
                    for (int k = 6 * d + 3; k < 6 * d + 6; ++k) dst[k] = (__bf16)1.0f;
                    for (int k = 6 * d + 6; k < KT; ++k) dst[k] = (__bf16)0.0f;
                }
                ws[pt] = PREF ? prew : (ok ? wf[p0 + pt] : 0.0f);
            }
        }
        fresh = false;
        __syncthreads();
        const int64_t pnext = visit(p0 + PN);
        if (PREF && pnext < it.j1) fetch(pnext);  // in flight during the panel's products
        uint32_t wbits = ~0u;  // the wave's tiles to evaluate in this panel
        if (MK == 2) wbits = __builtin_amdgcn_readfirstlane(mwl[pi * SM_WAVES + wv]);
        uint32_t rec = 0;  // MK 1: the tiles found to matter
        float pacc[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) pacc[rt] = 0.0f;
#pragma unroll 1
        for (int tl = 0; tl < PN / 16; ++tl) {
            if (MK == 2 && !((wbits >> tl) & 1u)) {  // every entry of the wave's tile is negligible
                if ((lane & 3) == 0) csum[wv][tl * 16 + symf_point(g, (lane >> 2) & 3)] = 0.0f;
                continue;
            }
            bf8v a[KS];
#pragma unroll
            for (int s = 0; s < KS; ++s) a[s] = *reinterpret_cast<const bf8v *>(ys + (tl * 16 + lr) * LDB + 32 * s + 8 * g);
            float wp[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) wp[q] = ws[tl * 16 + symf_point(g, q)];
            float cacc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            float tmax = -INFINITY;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                f4v t = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int s = 0; s < KS; ++s) t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[s], xb[rt][s], t, 0, 0, 0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float e = __builtin_amdgcn_exp2f(t[q]);
                    if (QM) e = e == 0.0f ? 0.0f : e * t[q];  // -1e30 past the item: entry 0
                    pacc[rt] = fmaf(e, wp[q], pacc[rt]);
                    if (SYM) cacc[q] = fmaf(e, wi[rt], cacc[q]);
                }
                if (MK == 1 && it.i0 + (int64_t)(wv * RT + rt) * 16 + lr < it.iend)
                    tmax = fmaxf(tmax, fmaxf(fmaxf(t[0], t[1]), fmaxf(t[2], t[3])));
            }
            if (MK == 1 && __ballot(tmax >= kSymSkipLog2) != 0) rec |= 1u << tl;
            if (!SYM) continue;
#pragma unroll
            for (int o = 8, h = 2; o >= 4; o >>= 1, h >>= 1) {
                const bool up = (lane & o) != 0;
#pragma unroll
                for (int kk = 0; kk < h; ++kk) {
                    const float lo = cacc[kk], hi = cacc[kk + h];
                    const float send = up ? lo : hi;
                    cacc[kk] = (up ? hi : lo) + __shfl_xor(send, o, 64);
                }
            }
            float v = cacc[0];
            v += __shfl_xor(v, 2, 64);
            v += __shfl_xor(v, 1, 64);
            if ((lane & 3) == 0) csum[wv][tl * 16 + symf_point(g, (lane >> 2) & 3)] = v;
        }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt] += (double)pacc[rt];
        if (MK == 1 && lane == 0) mask[(it.mid * ppi + pi) * SM_WAVES + wv] = rec;
        __syncthreads();
        if (SYM && tid < cnt) {
            float cs = csum[0][tid];
#pragma unroll
            for (int w = 1; w < SM_WAVES; ++w) cs += csum[w][tid];
            colpart[(int64_t)it.blk * n + p0 + tid] = cs;
        }
        p0 = pnext;
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t i = it.i0 + (int64_t)(wv * RT + rt) * 16 + lr;
        double v = acc[rt];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (g == 0 && i < it.iend) rowpart[(int64_t)it.chunk * n + i] = v;
    }
}

// anchors[b] = the mean point of row block b (FP64 sums, stored in FP32).
__global__ void k_block_mean(const float *__restrict__ X, int d, const SymBlock *__restrict__ blocks,
                             float *__restrict__ anchors) {
    const SymBlock b = blocks[blockIdx.x];
    __shared__ double part[256];
    for (int k = 0; k < d; ++k) {
        double sacc = 0.0;
        for (int64_t i = b.i0 + threadIdx.x; i < b.iend; i += blockDim.x) sacc += (double)X[i * d + k];
        part[threadIdx.x] = sacc;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) anchors[blockIdx.x * d + k] = (float)(part[0] / (double)(b.iend - b.i0));
        __syncthreads();
    }
}

// Column data of k_kmv_sc: ya[j] = (2 c y_j1 .. 2 c y_jd, 0 .., -c |y_j|^2 at
// index D, 0 ..) in rows of ld doubles, c the column's problem's scale
// (pbeg / cprob: a batch) or c2.
template <class T>
__global__ void k_col_aug(const T *__restrict__ Y, int64_t n, int d, int D, int ld, double c2,
                          const int64_t *__restrict__ pbeg, const double *__restrict__ cprob, int np,
                          double *__restrict__ ya) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double c = c2;
    if (pbeg) {
        int lo = 0, hi = np - 1;  // last problem starting at or before j
        while (lo < hi) {
            int mid = (lo + hi + 1) / 2;
            if (pbeg[mid] <= j)
                lo = mid;
            else
                hi = mid - 1;
        }
        c = cprob[lo];
    }
    double nrm = 0.0;
    double *row = ya + j * ld;
    for (int k = 0; k < ld; ++k) {
        double v = k < d ? (double)Y[j * d + k] : 0.0;
        nrm = fma(v, v, nrm);
        if (k != D) row[k] = 2.0 * c * v;
    }
    row[D] = -c * nrm;
}

__global__ void k_w_to_float(const double *__restrict__ W, int64_t len, float *__restrict__ wf) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < len) wf[t] = (float)W[t];
}

// Large d: coordinates streamed from memory instead of registers.
template <class T, class C, int NR>
__global__ __launch_bounds__(MV_ROWS) void k_kmv_wide(const T *__restrict__ X, int64_t m,
                                                      const T *__restrict__ Y, int64_t n, int d, C scale,
                                                      const double *__restrict__ W, int nrhs, int rhs0,
                                                      int64_t cols_per_split, double *__restrict__ part,
                                                      const SampBlock *__restrict__ bt) {
    constexpr int TK = 64;
    __shared__ C ys[16][TK + 1];
    __shared__ C ws[16][NR];
    const int tid = threadIdx.x;
    const int split = blockIdx.y;
    int64_t i, iend, j0, j1;
    if (bt) {
        const SampBlock sb = bt[blockIdx.x];
        i = sb.i0 + tid;
        iend = sb.iend;
        j0 = sb.jlo + split * sb.cps;
        j1 = min(sb.jhi, j0 + sb.cps);
        if constexpr (sizeof(C) == 8) scale = sb.inv; else scale = sb.cs;
    } else {
        i = (int64_t)blockIdx.x * MV_ROWS + tid;
        iend = m;
        j0 = split * cols_per_split;
        j1 = min(n, j0 + cols_per_split);
    }
    const int nr = min(NR, nrhs - rhs0);
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = 0.0;
    const T *xr = X + (i < iend ? i : 0) * (int64_t)d;
    for (int64_t jt = j0; jt < j1; jt += 16) {
        C q[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) q[jj] = (C)0;
        for (int k0 = 0; k0 < d; k0 += TK) {
            for (int t = tid; t < 16 * TK; t += MV_ROWS) {
                int jj = t / TK, k = t % TK;
                int64_t j = jt + jj;
                ys[jj][k] = (j < j1 && k0 + k < d) ? (C)Y[j * d + k0 + k] : (C)0;
            }
            __syncthreads();
            int kend = min(TK, d - k0);
            for (int k = 0; k < kend; ++k) {
                C xv = (C)xr[k0 + k];
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) {
                    C t = xv - ys[jj][k];
                    q[jj] = fma(t, t, q[jj]);
                }
            }
            __syncthreads();
        }
        for (int t = tid; t < 16 * NR; t += MV_ROWS) {
            int jj = t / NR, r = t % NR;
            int64_t j = jt + jj;
            ws[jj][r] = (j < j1 && r < nr) ? (C)W[j * nrhs + rhs0 + r] : (C)0;
        }
        __syncthreads();
        C pacc[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) pacc[r] = (C)0;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            C kv = kexp(q[jj], scale);
#pragma unroll
            for (int r = 0; r < NR; ++r) pacc[r] = fma(kv, ws[jj][r], pacc[r]);
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] += (double)pacc[r];
        __syncthreads();
    }
    if (i < iend) {
        for (int r = 0; r < nr; ++r) part[((int64_t)split * m + i) * nrhs + rhs0 + r] = acc[r];
    }
}

__global__ void k_reduce_splits(const double *__restrict__ part, int nsplit, int64_t mn, double beta,
                                double *__restrict__ out) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= mn) return;
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * mn + t];
    out[t] = (beta != 0.0) ? s + beta * out[t] : s;
}

template <class T, class C, int D, int NR>
void launch_kmv(const T *X, int64_t m, const T *Y, int64_t n, int d, C scale, double c2, const double *W,
                int nrhs, int rhs0, int nsplit, int64_t cps, double *part, hipStream_t s, const SampBlock *bt,
                int64_t nb) {
    dim3 grid(bt ? (unsigned)nb : ceil_div(m, MV_ROWS), nsplit);
    if (D > 0)
        k_kmv<T, C, (D > 0 ? D : 1), NR><<<grid, MV_ROWS, 0, s>>>(X, m, Y, n, d, scale, W, nrhs, rhs0, cps, part, bt);
    else
        k_kmv_wide<T, C, NR><<<grid, MV_ROWS, 0, s>>>(X, m, Y, n, d, scale, W, nrhs, rhs0, cps, part, bt);
    check_launch("k_kmv");
}

template <class T, class C, int NR>
void dispatch_d(const T *X, int64_t m, const T *Y, int64_t n, int d, C scale, double c2, const double *W, int nrhs,
                int rhs0, int nsplit, int64_t cps, double *part, hipStream_t s, const SampBlock *bt, int64_t nb) {
    if (d <= 8)
        launch_kmv<T, C, 8, NR>(X, m, Y, n, d, scale, c2, W, nrhs, rhs0, nsplit, cps, part, s, bt, nb);
    else if (d <= 16)
        launch_kmv<T, C, 16, NR>(X, m, Y, n, d, scale, c2, W, nrhs, rhs0, nsplit, cps, part, s, bt, nb);
    else if (d <= 32)
        launch_kmv<T, C, 32, NR>(X, m, Y, n, d, scale, c2, W, nrhs, rhs0, nsplit, cps, part, s, bt, nb);
    else if (d <= 64)
        launch_kmv<T, C, 64, NR>(X, m, Y, n, d, scale, c2, W, nrhs, rhs0, nsplit, cps, part, s, bt, nb);
    else
        launch_kmv<T, C, 0, NR>(X, m, Y, n, d, scale, c2, W, nrhs, rhs0, nsplit, cps, part, s, bt, nb);
}

// Widths of the scalar-operand kernel (coordinates padded with zeros).
template <class T, int NR, bool QM = false>
void launch_sc(int D, dim3 grid, const T *X, int64_t m, int d, double c2, const double *ya, const float *wf,
               int nrhs, int rhs0, int64_t n, int64_t cps, double *part, const SampBlock *bt, hipStream_t s) {
#define KRR_SC(DD)                                                                                              \
    case DD:                                                                                                     \
        k_kmv_sc<T, DD, NR, sc_rpt(DD), QM><<<grid, MV_ROWS, 0, s>>>(X, m, d, c2, ya, wf, nrhs, rhs0, n, cps,   \
                                                                     part, bt);                              \
        break;
    switch (D) {
        KRR_SC(4)
        KRR_SC(8)
        KRR_SC(12)
        KRR_SC(16)
        KRR_SC(20)
        KRR_SC(24)
        KRR_SC(32)
        KRR_SC(48)
        KRR_SC(56)
        KRR_SC(64)
        default: fail(KRR_E_INVAL, "kernel_matvec: no scalar-operand variant for width %d", D);
    }
#undef KRR_SC
    check_launch("k_kmv_sc");
}

int sc_width(int d) {
    if (d <= 24) return (d + 3) / 4 * 4;
    if (d <= 32) return 32;
    if (d <= 48) return 48;
    if (d <= 56) return 56;
    return 64;
}


// Column data ya and FP32 weights wf of the FP32-entry kernels.
template <class T>
void prep_columns(const T *Y, int64_t n, int d, int D, double c2, const double *W, int nrhs, const Batch *batch,
                  DBuf &ya, DBuf &wf, hipStream_t s) {
    const int LD = (D + 2) & ~1;  // ColLd
    ya = dalloc<double>((size_t)n * LD);
    wf = dalloc<float>((size_t)n * nrhs);
    DBuf pb, cp;
    if (batch) {
        std::vector<double> cpr(batch->np());
        for (int k = 0; k < batch->np(); ++k) cpr[k] = kernel_scale_log2(batch->h[k]);
        pb = upload(batch->pbeg, s);
        cp = upload(cpr, s);
        sync(s);  // `cpr` is released at the end of this scope
    }
    k_col_aug<T><<<ceil_div(n, 256), 256, 0, s>>>(Y, n, d, D, LD, c2, pb.as<int64_t>(), cp.as<double>(),
                                                  batch ? batch->np() : 0, ya.as<double>());
    check_launch("k_col_aug");
    k_w_to_float<<<ceil_div(n * nrhs, 256), 256, 0, s>>>(W, n * nrhs, wf.as<float>());
    check_launch("k_w_to_float");
    sync(s);  // pb / cp are released on return
}

template <class T, int D, int NR>
void launch_sym(dim3 gd, dim3 gs, dim3 gr, int rows_pb, const T *X, int d, double c2, const double *ya,
                const float *wf, int64_t n, const SampBlock *dt, const SymItem *it, const SymBlock *bl, double *diag,
                double *rowpart, float *colpart, double beta, double *Out, hipStream_t s) {
    constexpr int RPT = sc_rpt(D);
    k_kmv_sc<T, D, NR, RPT><<<gd, MV_ROWS, 0, s>>>(X, n, d, c2, ya, wf, NR, 0, n, 0, diag, dt);
    check_launch("k_kmv_sc (diagonal blocks)");
    if (gs.x > 0) {
        k_kmv_sym<T, D, NR, RPT><<<gs, MV_ROWS, 0, s>>>(X, d, ya, wf, NR, n, it, rowpart, colpart);
        check_launch("k_kmv_sym");
    }
    k_sym_reduce<NR><<<gr, 256, 0, s>>>(bl, rows_pb, diag, rowpart, colpart, n, beta, Out);
    check_launch("k_sym_reduce");
}

template <int D>
void launch_symm(dim3 gd, dim3 gs, dim3 gr, int rows_pb, const float *X, int d, double c2, const double *ya,
                 const float *wf, int64_t n, const SampBlock *dt, const SymItem *it, const SymBlock *bl, double *diag,
                 double *rowpart, float *colpart, double beta, double *Out, hipStream_t s) {
    k_kmv_sc<float, D, 1, sc_rpt(D)><<<gd, MV_ROWS, 0, s>>>(X, n, d, c2, ya, wf, 1, 0, n, 0, diag, dt);
    check_launch("k_kmv_sc (diagonal blocks)");
    if (gs.x > 0) {
        if (d < D)
            k_kmv_symm<D, true><<<gs, 64 * SM_WAVES, 0, s>>>(X, d, ya, wf, n, it, rowpart, colpart);
        else
            k_kmv_symm<D, false><<<gs, 64 * SM_WAVES, 0, s>>>(X, d, ya, wf, n, it, rowpart, colpart);
        check_launch("k_kmv_symm");
    }
    k_sym_reduce<1><<<gr, 256, 0, s>>>(bl, rows_pb, diag, rowpart, colpart, n, beta, Out);
    check_launch("k_sym_reduce");
}

template <int D>
void launch_symf(dim3 gd, dim3 gs, dim3 gr, int rows_pb, const float *X, int d, double c2, const double *ya,
                 const float *wf, int64_t n, const SampBlock *dt, const SymItem *it, const SymBlock *bl,
                 int64_t nblocks, double *diag, double *rowpart, float *colpart, double beta, double *Out,
                 hipStream_t s) {
    k_kmv_sc<float, D, 1, sc_rpt(D)><<<gd, MV_ROWS, 0, s>>>(X, n, d, c2, ya, wf, 1, 0, n, 0, diag, dt);
    check_launch("k_kmv_sc (diagonal blocks)");
    if (gs.x > 0) {
        DBuf anchors = dalloc<float>((size_t)nblocks * d);
        k_block_mean<<<(unsigned)nblocks, 256, 0, s>>>(X, d, bl, anchors.as<float>());
        check_launch("k_block_mean");
        if (d < D)
            k_kmv_symf<D, true><<<gs, 64 * SM_WAVES, 0, s>>>(X, d, anchors.as<float>(), wf, n, it, rowpart, colpart);
        else
            k_kmv_symf<D, false><<<gs, 64 * SM_WAVES, 0, s>>>(X, d, anchors.as<float>(), wf, n, it, rowpart, colpart);
        check_launch("k_kmv_symf");
        sync(s);  // the anchors are released on return
    }
    k_sym_reduce<1><<<gr, 256, 0, s>>>(bl, rows_pb, diag, rowpart, colpart, n, beta, Out);
    check_launch("k_sym_reduce");
}

// BF16 three-term exponents: K slots for d (the symmetric form's row tiles
// follow from them).  mk: the tile map's use (k_kmv_symb's MK; 3: record,
// then use, in one call).
template <int KT, bool QM>
void launch_symb_kernel(dim3 gs, const float *X, int d, const float *anchors, const float *wf, int64_t n,
                        const SymItem *it, double *rowpart, float *colpart, int mk, uint32_t *mask, int ppi,
                        hipStream_t s) {
    constexpr int RTM = symb_rt_sym(KT);
    if constexpr (QM) {
        k_kmv_symb<KT, RTM, true, true><<<gs, 64 * SM_WAVES, 0, s>>>(X, X, d, anchors, wf, n, it, rowpart, colpart);
    } else {
        if (mk == 0)
            k_kmv_symb<KT, RTM, false, true, 0><<<gs, 64 * SM_WAVES, 0, s>>>(X, X, d, anchors, wf, n, it, rowpart,
                                                                             colpart);
        if (mk == 1 || mk == 3)
            k_kmv_symb<KT, RTM, false, true, 1><<<gs, 64 * SM_WAVES, 0, s>>>(X, X, d, anchors, wf, n, it, rowpart,
                                                                             colpart, mask, ppi);
        if (mk == 2 || mk == 3)
            k_kmv_symb<KT, RTM, false, true, 2><<<gs, 64 * SM_WAVES, 0, s>>>(X, X, d, anchors, wf, n, it, rowpart,
                                                                             colpart, mask, ppi);
    }
}

template <int D, bool QM>
void launch_symb(dim3 gd, dim3 gs, dim3 gr, int rows_pb, const float *X, int d, double c2, const double *ya,
                 const float *wf, int64_t n, const SampBlock *dt, const SymItem *it, const SymBlock *bl,
                 int64_t nblocks, double *diag, double *rowpart, float *colpart, double beta, double *Out,
                 int mk, uint32_t *mask, int ppi, hipStream_t s) {
    k_kmv_sc<float, D, 1, sc_rpt(D), QM><<<gd, MV_ROWS, 0, s>>>(X, n, d, c2, ya, wf, 1, 0, n, 0, diag, dt);
    check_launch("k_kmv_sc (diagonal blocks)");
    if (gs.x > 0) {
        DBuf anchors = dalloc<float>((size_t)nblocks * d);
        k_block_mean<<<(unsigned)nblocks, 256, 0, s>>>(X, d, bl, anchors.as<float>());
        check_launch("k_block_mean");
        const int kt = (6 * d + 6 + 31) / 32 * 32;
        const float *an = anchors.as<float>();
#define KRR_SYMB(KT)                                                                                  \
    case KT:                                                                                          \
        launch_symb_kernel<KT, QM>(gs, X, d, an, wf, n, it, rowpart, colpart, mk, mask, ppi, s);             \
        break;
        switch (kt) {  // row tiles per wave: symb_rt_sym
            KRR_SYMB(32)
            KRR_SYMB(64)
            KRR_SYMB(96)
            KRR_SYMB(128)
            KRR_SYMB(160)
            KRR_SYMB(192)
            default: fail(KRR_E_INVAL, "kernel_matvec: no BF16 symmetric variant for width %d", d);
        }
#undef KRR_SYMB
        check_launch("k_kmv_symb");
        sync(s);  // the anchors are released on return
    }
    k_sym_reduce<1><<<gr, 256, 0, s>>>(bl, rows_pb, diag, rowpart, colpart, n, beta, Out);
    check_launch("k_sym_reduce");
}

// The symmetric product y = K(X, X) W + beta y (FP32 entries) when it
// applies (d <= 32, one or two right-hand sides, partial sums within budget);
// returns false otherwise.  FP32 points with one right-hand side take the
// matrix-core exponents (k_kmv_symm) unless the vector form is selected;
// the rest the vector form.  qm: the entry exp2(t) t, on the BF16 form only.
// skip: the negligible-tile map (BF16 form, qm false): used when it was
// recorded for the same item layout, otherwise recorded by this product.
template <class T>
bool kmv_sym(const T *X, int64_t n, int d, double h, const double *W, int nrhs, double beta, double *Out,
             hipStream_t s, const Batch *batch, bool qm = false, SymSkip *skip = nullptr) {
    const int D = sc_width(d);
    if (D > 32 || (nrhs != 1 && nrhs != 2)) return false;
    const bool mc = sizeof(T) == 4 && nrhs == 1 && tune_get(KRR_TUNE_SYMMETRIC) == 1;
    const int form = tune_get(KRR_TUNE_SYMMETRIC);
    const bool mb = sizeof(T) == 4 && nrhs == 1 && form == 4 && d <= symb_max_d;
    const bool mf = sizeof(T) == 4 && nrhs == 1 && (form == 3 || (form == 4 && d > symb_max_d));
    if (qm && !mb) return false;
    const int diag_rows = MV_ROWS * sc_rpt(D);  // rows of one k_kmv_sc workgroup
    // the tile map: the refinement's products (skip given) or every product
    // (knob 2)
    const int map_knob = tune_get(KRR_TUNE_SYM_SKIP);
    const bool map_on = mb && !qm && map_knob != 0 && (skip || map_knob == 2);
    const int rows_pb = mb ? symb_rows_sym(d) : ((mc || mf) ? symm_rows(D) : diag_rows);
    std::vector<int64_t> pb = batch ? batch->pbeg : std::vector<int64_t>{0, n};
    std::vector<double> hs = batch ? batch->h : std::vector<double>{h};
    const int np = (int)hs.size();
    // columns per item: a multiple of the tile width, halved (while it is a
    // multiple of 2048) as long as the grid would hold fewer than ~4096
    // items (sum of n_p^2 / (2 rows_pb CH)), so small products fill the chip
    int64_t CH = tune_get(KRR_TUNE_SYM_CHUNK);
    // with a tile map the item's map words sit in LDS: at most kMapPanels panels
    if (map_on) CH = std::min<int64_t>(CH, (int64_t)kMapPanels * symb_pn(symb_kt(d)));
    double sq = 0.0;
    for (int p = 0; p < np; ++p) sq += (double)(pb[p + 1] - pb[p]) * (double)(pb[p + 1] - pb[p]);
    while (CH % 2048 == 0 && sq / (2.0 * rows_pb * CH) < 4096.0) CH /= 2;
    std::vector<SymBlock> blocks;
    std::vector<SymItem> items;
    std::vector<SampBlock> diag;
    int64_t nchunks = 0, mids = 0;  // mids: items of every problem, left-out ones included
    for (int p = 0; p < np; ++p) {
        const bool out = batch && batch->skipped(p);  // rows left as they are
        const double c2 = kernel_scale_log2(hs[p]);
        const int64_t first = (int64_t)blocks.size(), pe = pb[p + 1];
        for (int64_t i0 = pb[p]; i0 < pe; i0 += rows_pb) {
            SymBlock b{};
            b.i0 = i0;
            b.iend = std::min<int64_t>(pe, i0 + rows_pb);
            b.first_blk = first;
            const int64_t blk = (int64_t)blocks.size(), off = b.iend;
            if (off < pe) {
                b.chunk_lo = off / CH;
                b.chunk_hi = (pe - 1) / CH + 1;
            }
            for (int64_t c = b.chunk_lo; c < b.chunk_hi; ++c) {
                SymItem it{};
                it.i0 = b.i0;
                it.iend = b.iend;
                it.j0 = std::max(off, c * CH);
                it.j1 = std::min(pe, (c + 1) * CH);
                it.blk = blk;
                it.chunk = c;
                it.c2 = c2;
                it.mid = mids++;
                if (!out) items.push_back(it);
            }
            if (out) continue;
            nchunks = std::max(nchunks, b.chunk_hi);
            blocks.push_back(b);
            for (int64_t r0 = b.i0; r0 < b.iend; r0 += diag_rows) {
                SampBlock sb{};
                sb.i0 = r0;
                sb.iend = std::min<int64_t>(b.iend, r0 + diag_rows);
                sb.jlo = b.i0;
                sb.jhi = b.iend;
                sb.cps = rows_pb;
                sb.c2 = c2;
                diag.push_back(sb);
            }
        }
    }
    if (blocks.empty()) return true;  // every problem left out: nothing to compute
    const double col_bytes = (double)blocks.size() * n * nrhs * sizeof(float);
    const double row_bytes = (double)nchunks * n * nrhs * sizeof(double);
    if (col_bytes + row_bytes > 24e9) return false;  // the plain product needs no partial sums
    // the tile map: mk as in launch_symb_kernel
    int mk = 0, ppi = 0;
    uint32_t *mask = nullptr;
    DBuf own_map;
    if (map_on) {
        ppi = (int)ceil_div(CH, (int64_t)symb_pn(symb_kt(d)));
        KRR_REQUIRE(ppi <= kMapPanels, "kernel_matvec: %d panels per item exceed the tile map's %d", ppi,
                    kMapPanels);
        const size_t words = (size_t)mids * ppi * SM_WAVES;
        std::vector<double> key{(double)(uintptr_t)X, (double)n, (double)d, (double)CH, (double)rows_pb,
                                (double)mids};
        for (int p = 0; p < np; ++p) {
            key.push_back((double)pb[p + 1]);
            key.push_back(hs[p]);
        }
        if (skip && skip->ready && skip->key == key) {
            mk = 2;
        } else if (!(batch && batch->any_skipped())) {  // a recording covers every item
            DBuf &map = skip ? skip->bits : own_map;
            map = dalloc<uint32_t>(std::max<size_t>(words, 1));
            // words past an item's last panel are never read; bits past a
            // panel's tiles stay 0
            KRR_HIP(hipMemsetAsync(map.get(), 0, std::max<size_t>(words, 1) * sizeof(uint32_t), s));
            mk = skip ? 1 : 3;
            if (skip) {
                const int64_t pn = symb_pn(symb_kt(d));
                int64_t panels = 0;
                for (const SymItem &it : items) panels += ceil_div(it.j1 - it.j0, pn);
                skip->key = key;
                skip->ready = true;
                skip->tiles = panels * SM_WAVES * (pn / 16);
                skip->entries_per_tile = (int64_t)rows_pb / SM_WAVES * 16;
            }
        }
        if (mk != 0) mask = (skip ? skip->bits : own_map).as<uint32_t>();
    }
    const double c2 = kernel_scale_log2(h);
    DBuf ya, wf;
    prep_columns<T>(X, n, d, D, c2, W, nrhs, batch, ya, wf, s);
    DBuf dd = dalloc<double>((size_t)n * nrhs), rp = dalloc<double>(std::max<size_t>((size_t)(row_bytes / 8), 1)),
         cpart = dalloc<float>(std::max<size_t>((size_t)(col_bytes / 4), 1));
    DBuf dt = upload(diag, s), it = upload(items, s), bl = upload(blocks, s);
    sync(s);  // the host tables are released on return
    dim3 gd((unsigned)diag.size()), gs((unsigned)items.size()), gr(ceil_div(rows_pb, 256), (unsigned)blocks.size());
#define KRR_SYM(DD, NRR)                                                                                        \
    if constexpr (sizeof(T) == 4 && NRR == 1) {                                                                 \
        if (mc) {                                                                                               \
            launch_symm<DD>(gd, gs, gr, rows_pb, X, d, c2, ya.as<double>(), wf.as<float>(), n,                 \
                                 dt.as<SampBlock>(), it.as<SymItem>(), bl.as<SymBlock>(), dd.as<double>(),      \
                                 rp.as<double>(), cpart.as<float>(), beta, Out, s);                             \
            break;                                                                                              \
        }                                                                                                       \
        if (mb) {                                                                                               \
            (qm ? launch_symb<DD, true> : launch_symb<DD, false>)(                                              \
                gd, gs, gr, rows_pb, X, d, c2, ya.as<double>(), wf.as<float>(), n, dt.as<SampBlock>(),          \
                it.as<SymItem>(), bl.as<SymBlock>(), (int64_t)blocks.size(), dd.as<double>(), rp.as<double>(),  \
                cpart.as<float>(), beta, Out, mk, mask, ppi, s);                                                \
            break;                                                                                              \
        }                                                                                                       \
        if (mf) {                                                                                               \
            launch_symf<DD>(gd, gs, gr, rows_pb, X, d, c2, ya.as<double>(), wf.as<float>(), n,                 \
                            dt.as<SampBlock>(), it.as<SymItem>(), bl.as<SymBlock>(), (int64_t)blocks.size(),    \
                            dd.as<double>(), rp.as<double>(), cpart.as<float>(), beta, Out, s);                 \
            break;                                                                                              \
        }                                                                                                       \
    }                                                                                                           \
    launch_sym<T, DD, NRR>(gd, gs, gr, rows_pb, X, d, c2, ya.as<double>(), wf.as<float>(), n, dt.as<SampBlock>(), \
                           it.as<SymItem>(), bl.as<SymBlock>(), dd.as<double>(), rp.as<double>(),              \
                           cpart.as<float>(), beta, Out, s)
    switch (D * 4 + nrhs) {
        case 4 * 4 + 1: KRR_SYM(4, 1); break;
        case 4 * 4 + 2: KRR_SYM(4, 2); break;
        case 8 * 4 + 1: KRR_SYM(8, 1); break;
        case 8 * 4 + 2: KRR_SYM(8, 2); break;
        case 12 * 4 + 1: KRR_SYM(12, 1); break;
        case 12 * 4 + 2: KRR_SYM(12, 2); break;
        case 16 * 4 + 1: KRR_SYM(16, 1); break;
        case 16 * 4 + 2: KRR_SYM(16, 2); break;
        case 20 * 4 + 1: KRR_SYM(20, 1); break;
        case 20 * 4 + 2: KRR_SYM(20, 2); break;
        case 24 * 4 + 1: KRR_SYM(24, 1); break;
        case 24 * 4 + 2: KRR_SYM(24, 2); break;
        case 32 * 4 + 1: KRR_SYM(32, 1); break;
        case 32 * 4 + 2: KRR_SYM(32, 2); break;
        default: fail(KRR_E_INVAL, "kernel_matvec: no symmetric variant for width %d", D);
    }
#undef KRR_SYM
    sync(s);  // temporaries are released on return
    return true;
}

// K(X, Y) w with the entry exp2(t) t for FP32 points of width d <= 31 (the
// fused backward's dh when X != Y): the BF16 matrix-core exponents of
// Set bits of a tile map (one 64-bit atomic per workgroup).
__global__ __launch_bounds__(256) void k_popcount(const uint32_t *__restrict__ w, int64_t nw,
                                                  unsigned long long *__restrict__ out) {
    __shared__ unsigned long long part[4];
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nw; i += (int64_t)gridDim.x * 256)
        c += (unsigned long long)__popc(w[i]);
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, part[0] + part[1] + part[2] + part[3]);
}

}  // namespace

int64_t sym_skip_kept(const SymSkip &m, hipStream_t s) {
    if (!m.ready) return 0;
    const int64_t nw = (int64_t)(m.bits.bytes() / sizeof(uint32_t));
    DBuf cnt = dalloc<unsigned long long>(1);
    KRR_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(unsigned long long), s));
    k_popcount<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, ceil_div(nw, 256))), 256, 0, s>>>(
        m.bits.as<uint32_t>(), nw, cnt.as<unsigned long long>());
    check_launch("k_popcount");
    unsigned long long h = 0;
    d2h(&h, cnt.as<unsigned long long>(), 1, s);
    sync(s);
    return (int64_t)h;
}

namespace {

// k_kmv_symb without column sums.  Items are (row block of X, chunk of Y's
// columns), the chunk sized so that the grid holds about 2048 workgroups;
// the chunks' FP64 row partials are summed in a fixed order.
bool kmv_q_rect(const float *X, int64_t m, const float *Y, int64_t n, int d, double h, const double *W, double *Out,
                hipStream_t s) {
    if (d > symb_max_d || tune_get(KRR_TUNE_SYMMETRIC) != 4 || m <= 0 || n <= 0) return false;
    const int kt = symb_kt(d), rows_pb = symb_rows(d);
    const int64_t pn = symb_pn(kt), nblocks = (m + rows_pb - 1) / rows_pb;
    const int64_t want = std::max<int64_t>(1, (2048 + nblocks - 1) / nblocks);
    int64_t ch = (n + want - 1) / want;
    ch = std::max<int64_t>(pn, (ch + pn - 1) / pn * pn);
    const int64_t nch = (n + ch - 1) / ch;
    const double c2 = kernel_scale_log2(h);
    std::vector<SymBlock> blocks;
    std::vector<SymItem> items;
    for (int64_t b = 0; b < nblocks; ++b) {
        SymBlock sb{};
        sb.i0 = b * rows_pb;
        sb.iend = std::min<int64_t>(m, sb.i0 + rows_pb);
        blocks.push_back(sb);
        for (int64_t c = 0; c < nch; ++c) {
            SymItem it{};
            it.i0 = sb.i0;
            it.iend = sb.iend;
            it.j0 = c * ch;
            it.j1 = std::min<int64_t>(n, (c + 1) * ch);
            it.blk = b;
            it.chunk = c;
            it.c2 = c2;
            items.push_back(it);
        }
    }
    DBuf wf = dalloc<float>((size_t)n), rp = dalloc<double>((size_t)(nch * m)), an = dalloc<float>((size_t)(nblocks * d));
    DBuf bl = upload(blocks, s), it = upload(items, s);
    sync(s);  // the host tables are released on return
    k_w_to_float<<<ceil_div(n, 256), 256, 0, s>>>(W, n, wf.as<float>());
    check_launch("k_w_to_float");
    k_block_mean<<<(unsigned)nblocks, 256, 0, s>>>(X, d, bl.as<SymBlock>(), an.as<float>());
    check_launch("k_block_mean");
    const dim3 gs((unsigned)items.size());
    const float *a = an.as<float>(), *w = wf.as<float>();
    const SymItem *ip = it.as<SymItem>();
    double *r = rp.as<double>();
#define KRR_QR(KT)                                                                                      \
    case KT:                                                                                            \
        k_kmv_symb<KT, symb_rt(KT), true, false><<<gs, 64 * SM_WAVES, 0, s>>>(X, Y, d, a, w, m, ip, r, \
                                                                               nullptr);                \
        break;
    switch (kt) {
        KRR_QR(32)
        KRR_QR(64)
        KRR_QR(96)
        KRR_QR(128)
        KRR_QR(160)
        KRR_QR(192)
        default: fail(KRR_E_INVAL, "kernel_matvec_q: no BF16 variant for width %d", d);
    }
#undef KRR_QR
    check_launch("k_kmv_symb (rectangular)");
    k_reduce_splits<<<ceil_div(m, 256), 256, 0, s>>>(r, (int)nch, m, 0.0, Out);
    check_launch("k_reduce_splits");
    sync(s);  // temporaries are released on return
    return true;
}

// The plain product K(X, Y) W (no batch, no symmetric form, d <= 64 for the
// FP32 entries' scalar-operand kernel): column splits so that the grid fills
// the chip, and the scratch it needs -- split-K partial sums, and for FP32
// entries the column data and FP32 weights.
struct KmvPlan {
    bool sc;
    int D, rows_pb, nsplit;
    int64_t cps;
    size_t part_elems, ya_elems, wf_elems;  // doubles, doubles, floats
};

KmvPlan kmv_plan(int64_t m, int64_t n, int d, int nrhs, bool f32) {
    KmvPlan P{};
    P.sc = f32 && d <= 64;
    P.D = P.sc ? sc_width(d) : 0;
    P.rows_pb = P.sc ? MV_ROWS * sc_rpt(P.D) : MV_ROWS;
    const int64_t row_blocks = ceil_div(m, P.rows_pb);
    int nsplit = (int)std::max<int64_t>(
        1, std::min<int64_t>(ceil_div(tune_get(KRR_TUNE_MV_BLOCKS), row_blocks), ceil_div(n, 4 * MV_TN)));
    int64_t cps = (int64_t)ceil_div(n, nsplit);
    cps = (cps + MV_TN - 1) / MV_TN * MV_TN;
    P.nsplit = (int)ceil_div(n, cps);
    P.cps = cps;
    P.part_elems = (size_t)P.nsplit * m * nrhs;
    const int LD = (P.D + 2) & ~1;  // ColLd
    P.ya_elems = P.sc ? (size_t)n * LD : 0;
    P.wf_elems = P.sc ? (size_t)n * nrhs : 0;
    return P;
}

// Runs a plan with caller-given scratch (part, and ya / wf for FP32 entries).
// Every scratch element read is written first by the same call; nothing is
// allocated and the stream is not synchronized.
template <class T, class C>
void kmv_run(const T *X, int64_t m, const T *Y, int64_t n, int d, double h, const double *W, int nrhs, double beta,
             double *Out, const KmvPlan &P, double *part, double *ya, float *wf, hipStream_t s, bool qmode = false) {
    const C scale = kernel_scale<C>(h);
    const double c2 = kernel_scale_log2(h);
    const int nsplit = P.nsplit;
    const int64_t cps = P.cps;
    if (P.sc) {
        const int D = P.D, LD = (D + 2) & ~1;
        k_col_aug<T><<<ceil_div(n, 256), 256, 0, s>>>(Y, n, d, D, LD, c2, nullptr, nullptr, 0, ya);
        check_launch("k_col_aug");
        k_w_to_float<<<ceil_div(n * nrhs, 256), 256, 0, s>>>(W, n * nrhs, wf);
        check_launch("k_w_to_float");
        dim3 grid(ceil_div(m, P.rows_pb), nsplit);
        if (qmode) {  // one right-hand side (checked by the caller)
            launch_sc<T, 1, true>(D, grid, X, m, d, c2, ya, wf, nrhs, 0, n, cps, part, nullptr, s);
        }
        for (int r0 = qmode ? nrhs : 0; r0 < nrhs;) {
            const int left = nrhs - r0;
            const int nr = left >= 16 ? 16 : left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
            switch (nr) {
                case 16: launch_sc<T, 16>(D, grid, X, m, d, c2, ya, wf, nrhs, r0, n, cps, part, nullptr, s); break;
                case 8: launch_sc<T, 8>(D, grid, X, m, d, c2, ya, wf, nrhs, r0, n, cps, part, nullptr, s); break;
                case 4: launch_sc<T, 4>(D, grid, X, m, d, c2, ya, wf, nrhs, r0, n, cps, part, nullptr, s); break;
                case 2: launch_sc<T, 2>(D, grid, X, m, d, c2, ya, wf, nrhs, r0, n, cps, part, nullptr, s); break;
                default: launch_sc<T, 1>(D, grid, X, m, d, c2, ya, wf, nrhs, r0, n, cps, part, nullptr, s); break;
            }
            r0 += nr;
        }
    } else {
        for (int r0 = 0; r0 < nrhs;) {
            const int left = nrhs - r0;
            const int nr = left >= 16 ? 16 : left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
            switch (nr) {
                case 16: dispatch_d<T, C, 16>(X, m, Y, n, d, scale, c2, W, nrhs, r0, nsplit, cps, part, s, nullptr, 0); break;
                case 8: dispatch_d<T, C, 8>(X, m, Y, n, d, scale, c2, W, nrhs, r0, nsplit, cps, part, s, nullptr, 0); break;
                case 4: dispatch_d<T, C, 4>(X, m, Y, n, d, scale, c2, W, nrhs, r0, nsplit, cps, part, s, nullptr, 0); break;
                case 2: dispatch_d<T, C, 2>(X, m, Y, n, d, scale, c2, W, nrhs, r0, nsplit, cps, part, s, nullptr, 0); break;
                default: dispatch_d<T, C, 1>(X, m, Y, n, d, scale, c2, W, nrhs, r0, nsplit, cps, part, s, nullptr, 0); break;
            }
            r0 += nr;
        }
    }
    const int64_t mn = m * nrhs;
    k_reduce_splits<<<ceil_div(mn, 256), 256, 0, s>>>(part, nsplit, mn, beta, Out);
    check_launch("k_reduce_splits");
}

template <class T, class C>
void kmv_typed(const T *X, int64_t m, const T *Y, int64_t n, int d, double h, const double *W, int nrhs,
               double beta, double *Out, hipStream_t s, const Batch *batch, SymSkip *skip) {
    if constexpr (sizeof(C) == 4 && sizeof(T) == 4) {
        if (d > 64) {  // wide points: the exponents as a matrix-core GEMM
            kmv_wide_mfma(X, m, Y, n, d, h, W, nrhs, beta, Out, s, batch);
            return;
        }
    }
    if constexpr (sizeof(C) == 8) {
        if (d > 64) {  // FP64 entries of wide points: an FP64 matrix-core GEMM
            kmv_wide_mfma64<T>(X, m, Y, n, d, h, W, nrhs, beta, Out, s, batch);
            return;
        }
    }
    if constexpr (sizeof(C) == 4) {
        // K(X, X): each off-diagonal entry once, for its row and its column
        if (X == Y && m == n && tune_get(KRR_TUNE_SYMMETRIC) &&
            kmv_sym<T>(X, n, d, h, W, nrhs, beta, Out, s, batch, false, skip))
            return;
    }
    if (!batch) {
        const KmvPlan P = kmv_plan(m, n, d, nrhs, sizeof(C) == 4);
        DBuf part = dalloc<double>(P.part_elems), ya = dalloc<double>(P.ya_elems), wf = dalloc<float>(P.wf_elems);
        kmv_run<T, C>(X, m, Y, n, d, h, W, nrhs, beta, Out, P, part.as<double>(), ya.as<double>(), wf.as<float>(),
                      s);
        sync(s);  // the temporaries are released on return
        return;
    }
    const C scale = kernel_scale<C>(h);
    const double c2 = kernel_scale_log2(h);
    const bool sc = sizeof(C) == 4 && d <= 64;
    const int D = sc ? sc_width(d) : 0;
    const int rows_pb = sc ? MV_ROWS * sc_rpt(D) : MV_ROWS;  // rows per workgroup
    // a batch: one block table row per (problem, row block), each problem's
    // columns split so that the grid has enough blocks to fill the chip
    int nsplit;
    int64_t cps = 0, nb = 0;
    DBuf btab;
    {
        std::vector<SampBlock> blocks = row_blocks(*batch, rows_pb);
        nb = (int64_t)blocks.size();
        int64_t nmax = 0;
        for (int k = 0; k < batch->np(); ++k) nmax = std::max(nmax, batch->size(k));
        nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(tune_get(KRR_TUNE_MV_BLOCKS), nb), ceil_div(nmax, 4 * MV_TN)));
        for (auto &b : blocks) {
            int64_t c = ceil_div(b.jhi - b.jlo, nsplit);
            b.cps = (c + MV_TN - 1) / MV_TN * MV_TN;
        }
        btab = upload(blocks, s);
        sync(s);
    }
    const SampBlock *bt = btab.as<SampBlock>();
    DBuf part = dalloc<double>((size_t)nsplit * m * nrhs);
    if (batch && batch->any_skipped())  // rows of left-out problems reduce to 0
        KRR_HIP(hipMemsetAsync(part.get(), 0, sizeof(double) * nsplit * m * nrhs, s));
    if (sc) {
        const int LD = (D + 2) & ~1;  // ColLd
        DBuf ya = dalloc<double>((size_t)n * LD), wf = dalloc<float>((size_t)n * nrhs), pb, cp;
        if (batch) {
            std::vector<double> cpr(batch->np());
            for (int k = 0; k < batch->np(); ++k) cpr[k] = kernel_scale_log2(batch->h[k]);
            pb = upload(batch->pbeg, s);
            cp = upload(cpr, s);
            sync(s);  // `cpr` is released at the end of this scope
        }
        k_col_aug<T><<<ceil_div(n, 256), 256, 0, s>>>(Y, n, d, D, LD, c2, pb.as<int64_t>(), cp.as<double>(),
                                                      batch ? batch->np() : 0, ya.as<double>());
        check_launch("k_col_aug");
        k_w_to_float<<<ceil_div(n * nrhs, 256), 256, 0, s>>>(W, n * nrhs, wf.as<float>());
        check_launch("k_w_to_float");
        dim3 grid(bt ? (unsigned)nb : ceil_div(m, rows_pb), nsplit);
        for (int r0 = 0; r0 < nrhs;) {
            const int left = nrhs - r0;
            const int nr = left >= 16 ? 16 : left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
            switch (nr) {
                case 16: launch_sc<T, 16>(D, grid, X, m, d, c2, ya.as<double>(), wf.as<float>(), nrhs, r0, n, cps,
                                          part.as<double>(), bt, s); break;
                case 8: launch_sc<T, 8>(D, grid, X, m, d, c2, ya.as<double>(), wf.as<float>(), nrhs, r0, n, cps,
                                        part.as<double>(), bt, s); break;
                case 4: launch_sc<T, 4>(D, grid, X, m, d, c2, ya.as<double>(), wf.as<float>(), nrhs, r0, n, cps,
                                        part.as<double>(), bt, s); break;
                case 2: launch_sc<T, 2>(D, grid, X, m, d, c2, ya.as<double>(), wf.as<float>(), nrhs, r0, n, cps,
                                        part.as<double>(), bt, s); break;
                default: launch_sc<T, 1>(D, grid, X, m, d, c2, ya.as<double>(), wf.as<float>(), nrhs, r0, n, cps,
                                         part.as<double>(), bt, s); break;
            }
            r0 += nr;
        }
        const int64_t mn = m * nrhs;
        k_reduce_splits<<<ceil_div(mn, 256), 256, 0, s>>>(part.as<double>(), nsplit, mn, beta, Out);
        check_launch("k_reduce_splits");
        sync(s);  // the temporaries are released on return
        return;
    }
    for (int r0 = 0; r0 < nrhs;) {
        int left = nrhs - r0;
        if (left >= 16) {
            dispatch_d<T, C, 16>(X, m, Y, n, d, scale, c2, W, nrhs, r0, nsplit, cps, part.as<double>(), s, bt, nb);
            r0 += 16;
        } else if (left >= 8) {
            dispatch_d<T, C, 8>(X, m, Y, n, d, scale, c2, W, nrhs, r0, nsplit, cps, part.as<double>(), s, bt, nb);
            r0 += 8;
        } else if (left >= 4) {
            dispatch_d<T, C, 4>(X, m, Y, n, d, scale, c2, W, nrhs, r0, nsplit, cps, part.as<double>(), s, bt, nb);
            r0 += 4;
        } else if (left >= 2) {
            dispatch_d<T, C, 2>(X, m, Y, n, d, scale, c2, W, nrhs, r0, nsplit, cps, part.as<double>(), s, bt, nb);
            r0 += 2;
        } else {
            dispatch_d<T, C, 1>(X, m, Y, n, d, scale, c2, W, nrhs, r0, nsplit, cps, part.as<double>(), s, bt, nb);
            r0 += 1;
        }
    }
    const int64_t mn = m * nrhs;
    k_reduce_splits<<<ceil_div(mn, 256), 256, 0, s>>>(part.as<double>(), nsplit, mn, beta, Out);
    check_launch("k_reduce_splits");
    sync(s);  // `part` is released on return
}
}  // namespace

void kernel_matvec_impl(const void *X, int64_t m, const void *Y, int64_t n, int d, int xprec, double h,
                        const double *W, int nrhs, double beta, double *Out, int prec, hipStream_t s,
                        const Batch *batch, SymSkip *skip) {
    if (m == 0) return;
    if (batch && batch->np() == 1) batch = nullptr;  // one problem: the plain launch
    KRR_REQUIRE(!batch || (X == Y && m == n), "kernel_matvec: a batch multiplies its own points");
    if (n == 0) {
        fail(KRR_E_INVAL, "kernel_matvec: n == 0");
    }
    if (xprec == KRR_F64) {
        auto Xd = static_cast<const double *>(X);
        auto Yd = static_cast<const double *>(Y);
        if (prec == KRR_F64)
            kmv_typed<double, double>(Xd, m, Yd, n, d, h, W, nrhs, beta, Out, s, batch, skip);
        else
            kmv_typed<double, float>(Xd, m, Yd, n, d, h, W, nrhs, beta, Out, s, batch, skip);
    } else {
        auto Xf = static_cast<const float *>(X);
        auto Yf = static_cast<const float *>(Y);
        if (prec == KRR_F64)
            kmv_typed<float, double>(Xf, m, Yf, n, d, h, W, nrhs, beta, Out, s, batch, skip);
        else
            kmv_typed<float, float>(Xf, m, Yf, n, d, h, W, nrhs, beta, Out, s, batch, skip);
    }
}

size_t kernel_matvec_ws_bytes(int64_t m, int64_t n, int d, int nrhs, int prec) {
    const KmvPlan P = kmv_plan(m, n, d, nrhs, prec != KRR_F64);
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    return up(P.part_elems * sizeof(double)) + up(P.ya_elems * sizeof(double)) + up(P.wf_elems * sizeof(float));
}

void kernel_matvec_ws(const void *X, int64_t m, const void *Y, int64_t n, int d, int xprec, double h,
                      const double *W, int nrhs, double *Out, int prec, void *ws, size_t ws_bytes, hipStream_t s) {
    KRR_REQUIRE(d <= 64, "kernel_matvec_ws: d = %d > 64 is not supported", d);
    const bool f32 = prec != KRR_F64;
    const KmvPlan P = kmv_plan(m, n, d, nrhs, f32);
    const size_t need = kernel_matvec_ws_bytes(m, n, d, nrhs, prec);
    KRR_REQUIRE(need <= ws_bytes, "kernel_matvec_ws: needs %zu bytes of scratch, %zu available", need, ws_bytes);
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    char *base = static_cast<char *>(ws);
    double *part = reinterpret_cast<double *>(base);
    double *ya = reinterpret_cast<double *>(base + up(P.part_elems * sizeof(double)));
    float *wf = reinterpret_cast<float *>(base + up(P.part_elems * sizeof(double)) + up(P.ya_elems * sizeof(double)));
    if (xprec == KRR_F64) {
        auto Xd = static_cast<const double *>(X);
        auto Yd = static_cast<const double *>(Y);
        if (f32)
            kmv_run<double, float>(Xd, m, Yd, n, d, h, W, nrhs, 0.0, Out, P, part, ya, wf, s);
        else
            kmv_run<double, double>(Xd, m, Yd, n, d, h, W, nrhs, 0.0, Out, P, part, ya, wf, s);
    } else {
        auto Xf = static_cast<const float *>(X);
        auto Yf = static_cast<const float *>(Y);
        if (f32)
            kmv_run<float, float>(Xf, m, Yf, n, d, h, W, nrhs, 0.0, Out, P, part, ya, wf, s);
        else
            kmv_run<float, double>(Xf, m, Yf, n, d, h, W, nrhs, 0.0, Out, P, part, ya, wf, s);
    }
}

void kernel_matvec_q(const void *X, int64_t m, const void *Y, int64_t n, int d, int xprec, double h,
                     const double *W, double *Out, hipStream_t s) {
    KRR_REQUIRE(d <= 64, "kernel_matvec_q: d = %d > 64", d);
    // K(X, X) with FP32 points: the symmetric matrix-core form, each
    // off-diagonal entry once
    if (X == Y && m == n && xprec == KRR_F32 && tune_get(KRR_TUNE_SYMMETRIC) &&
        kmv_sym<float>(static_cast<const float *>(X), n, d, h, W, 1, 0.0, Out, s, nullptr, true))
        return;
    // other FP32 operands: the same exponents without column sums
    if (xprec == KRR_F32 &&
        kmv_q_rect(static_cast<const float *>(X), m, static_cast<const float *>(Y), n, d, h, W, Out, s))
        return;
    const KmvPlan P = kmv_plan(m, n, d, 1, true);
    DBuf part = dalloc<double>(P.part_elems), ya = dalloc<double>(P.ya_elems), wf = dalloc<float>(P.wf_elems);
    if (xprec == KRR_F64)
        kmv_run<double, float>(static_cast<const double *>(X), m, static_cast<const double *>(Y), n, d, h, W, 1, 0.0,
                               Out, P, part.as<double>(), ya.as<double>(), wf.as<float>(), s, true);
    else
        kmv_run<float, float>(static_cast<const float *>(X), m, static_cast<const float *>(Y), n, d, h, W, 1, 0.0,
                              Out, P, part.as<double>(), ya.as<double>(), wf.as<float>(), s, true);
    sync(s);  // the temporaries are released on return
}

// ------------------------------------------------- tiled VALU sampling

namespace {
constexpr int SP_TM = 64, SP_TR = 64, SP_TK = 16;

// S[i, c] = sum_{j not in own leaf} K(x_i, x_j) R[j, c] for the block's 64 rows
// and 64 columns.  Thread (ty, tx) owns rows 4 ty.. and columns 4 tx..
template <class T, class C, class RT, class ST>
__global__ __launch_bounds__(256) void k_sample_valu(const T *__restrict__ X, int64_t n, int d, C scale,
                                                     const RT *__restrict__ R, int r,
                                                     const int32_t *__restrict__ lb,
                                                     const int32_t *__restrict__ le, ST *__restrict__ S,
                                                     const SampBlock *__restrict__ bt) {
    __shared__ C es[SP_TK][SP_TM + 1];
    __shared__ C rs[SP_TK][SP_TR];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    // rows [i0, iend) against columns [jlo, jhi): the whole matrix, or one
    // problem's diagonal block in a batch
    int64_t i0, iend, jlo, jhi;
    if (bt) {
        const SampBlock sb = bt[blockIdx.x];
        i0 = sb.i0;
        iend = sb.iend;
        jlo = sb.jlo;
        jhi = sb.jhi;
        if constexpr (sizeof(C) == 8)
            scale = sb.inv;
        else
            scale = sb.cs;
    } else {
        i0 = (int64_t)blockIdx.x * SP_TM;
        iend = n;
        jlo = 0;
        jhi = n;
    }
    const int c0 = blockIdx.y * SP_TR;
    C acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (C)0;
    // the entry this thread evaluates in each E tile: row er, column ej
    const int er = tid & 63, ej = tid >> 6;  // 64 rows x 4 column groups (4 entries each)
    const int64_t gi = i0 + er;
    const bool row_ok = gi < iend;
    const int32_t my_lb = row_ok && lb ? lb[gi] : 0, my_le = row_ok && le ? le[gi] : 0;
    for (int64_t jt = jlo; jt < jhi; jt += SP_TK) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int jj = ej * 4 + u;
            int64_t j = jt + jj;
            C v = (C)0;
            if (row_ok && j < jhi && !(j >= my_lb && j < my_le)) {
                C q = (C)0;
                for (int k = 0; k < d; ++k) {
                    C t = (C)X[gi * d + k] - (C)X[j * d + k];
                    q = fma(t, t, q);
                }
                v = kexp(q, scale);
            }
            es[jj][er] = v;
        }
        for (int t = tid; t < SP_TK * SP_TR; t += 256) {
            int jj = t / SP_TR, c = t % SP_TR;
            int64_t j = jt + jj;
            rs[jj][c] = (j < jhi && c0 + c < r) ? (C)R[j * r + c0 + c] : (C)0;
        }
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < SP_TK; ++jj) {
            C ev[4], rv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) ev[a] = es[jj][4 * ty + a];
#pragma unroll
            for (int b = 0; b < 4; ++b) rv[b] = rs[jj][4 * tx + b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = fma(ev[a], rv[b], acc[a][b]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        int64_t i = i0 + 4 * ty + a;
        if (i >= iend) continue;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            int c = c0 + 4 * tx + b;
            if (c < r) S[i * r + c] = (ST)acc[a][b];
        }
    }
}
}  // namespace

void sample_valu(const void *X, int64_t n, int d, int xprec, double h, const float *R, int r,
                 const int32_t *lb, const int32_t *le, void *S, int prec, hipStream_t s, const Batch *batch) {
    DBuf btab;
    int64_t nb = ceil_div(n, SP_TM);
    if (batch) {
        std::vector<SampBlock> blocks = row_blocks(*batch, SP_TM);
        nb = (int64_t)blocks.size();
        btab = upload(blocks, s);
        sync(s);
    }
    const SampBlock *bt = btab.as<SampBlock>();
    dim3 grid((unsigned)nb, ceil_div(r, SP_TR));
    if (prec == KRR_F64) {
        double sc = kernel_scale<double>(h);
        if (xprec == KRR_F64)
            k_sample_valu<double, double, float, double><<<grid, 256, 0, s>>>(
                static_cast<const double *>(X), n, d, sc, R, r, lb, le, static_cast<double *>(S), bt);
        else
            k_sample_valu<float, double, float, double><<<grid, 256, 0, s>>>(
                static_cast<const float *>(X), n, d, sc, R, r, lb, le, static_cast<double *>(S), bt);
    } else {
        float sc = kernel_scale<float>(h);
        if (xprec == KRR_F64)
            k_sample_valu<double, float, float, float><<<grid, 256, 0, s>>>(
                static_cast<const double *>(X), n, d, sc, R, r, lb, le, static_cast<float *>(S), bt);
        else
            k_sample_valu<float, float, float, float><<<grid, 256, 0, s>>>(
                static_cast<const float *>(X), n, d, sc, R, r, lb, le, static_cast<float *>(S), bt);
    }
    check_launch("k_sample_valu");
    sync(s);  // the block table is released on return
}

// ------------------------------------------------------------ helpers

namespace {
__device__ __forceinline__ uint64_t rb_mix(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_random_block(uint64_t seed, int64_t n, int r, int c0, float *__restrict__ R, int ldr) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * r) return;
    int64_t i = t / r;
    int c = (int)(t % r);
    uint64_t v = rb_mix(rb_mix(rb_mix(seed) ^ (uint64_t)i) ^ (uint64_t)(c0 + c));
    R[i * ldr + c] = (v >> 63) ? -1.0f : 1.0f;
}

template <class T>
__global__ void k_gather(const T *__restrict__ src, int64_t n, int cols, const int64_t *__restrict__ perm,
                         T *__restrict__ dst, int scatter) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * cols) return;
    int64_t i = t / cols;
    int c = (int)(t % cols);
    if (scatter)
        dst[perm[i] * cols + c] = src[t];
    else
        dst[t] = src[perm[i] * cols + c];
}

constexpr int DOT_BLOCK = 256, DOT_ROWS = 4096;

__global__ void k_dot_partial(const double *__restrict__ a, const double *__restrict__ b, int64_t n, int k,
                              double *__restrict__ part) {
    __shared__ double red[DOT_BLOCK / 64];
    const int c = blockIdx.y;
    const int64_t r0 = (int64_t)blockIdx.x * DOT_ROWS;
    const int64_t r1 = min(n, r0 + DOT_ROWS);
    double s = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += DOT_BLOCK) s += a[i * k + c] * b[i * k + c];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < DOT_BLOCK / 64; ++w) t += red[w];
        part[(int64_t)c * gridDim.x + blockIdx.x] = t;
    }
}

__global__ void k_dot_final(const double *__restrict__ part, int nb, int k, double *__restrict__ out) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= k) return;
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += part[(int64_t)c * nb + b];
    out[c] = t;
}
}  // namespace

void random_block(uint64_t seed, int64_t n, int r, int c0, float *R, int ldr, hipStream_t s) {
    if (n * r == 0) return;
    k_random_block<<<ceil_div(n * r, 256), 256, 0, s>>>(seed, n, r, c0, R, ldr);
    check_launch("k_random_block");
}

void gather_rows(const void *src, int prec, int64_t n, int cols, const int64_t *perm, void *dst, bool scatter,
                 hipStream_t s) {
    if (n * cols == 0) return;
    unsigned g = ceil_div(n * cols, 256);
    switch (prec) {
        case KRR_F64:
            k_gather<double><<<g, 256, 0, s>>>(static_cast<const double *>(src), n, cols, perm,
                                               static_cast<double *>(dst), scatter);
            break;
        case KRR_F32:
            k_gather<float><<<g, 256, 0, s>>>(static_cast<const float *>(src), n, cols, perm,
                                              static_cast<float *>(dst), scatter);
            break;
        default:
            fail(KRR_E_INVAL, "gather: unsupported dtype %d", prec);
    }
    check_launch("k_gather");
}

void dot_columns(const double *a, const double *b, int64_t n, int k, double *out, DBuf &scratch, hipStream_t s) {
    int nb = (int)std::max<int64_t>(1, ceil_div(n, DOT_ROWS));
    scratch.reserve(sizeof(double) * (size_t)nb * k);
    k_dot_partial<<<dim3(nb, k), DOT_BLOCK, 0, s>>>(a, b, n, k, scratch.as<double>());
    check_launch("k_dot_partial");
    k_dot_final<<<ceil_div(k, 64), 64, 0, s>>>(scratch.as<double>(), nb, k, out);
    check_launch("k_dot_final");
}

}  // namespace krr
