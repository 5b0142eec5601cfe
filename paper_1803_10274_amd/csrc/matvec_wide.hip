// FP32-entry kernel product Out = K(X, Y; h) W for wide points (d > 64) on
// the matrix cores.  The exponents are a GEMM of prepared coordinates (see
// wide.hpp), each split into three BF16 terms (hi + mid + lo: 24 bits, FP32's
// range) and the six cross products down to 2^-16 (hh, hm, mh, hl, lh, mm)
// accumulated by v_mfma_f32_32x32x16_bf16, which gives FP32-accurate
// exponents at about 2.6 times the FP32 matrix-core rate.  Only the three
// terms are stored and staged (6 bytes per coordinate); each pair reads its
// operands from the matching term block.  A workgroup owns
// 128 rows (4 waves x 32) and walks the columns in panels of 128 points,
// accumulating t = x~_i . y~_j over K chunks staged through LDS (points as A
// rows, the wave's rows as B columns).  Each lane then holds, for its row,
// the exponents of 16 points of every 32-point tile; exp2 turns them into
// FP32 entries that are directly the A operand of a v_mfma_f32_32x32x2_f32
// product with the panel's weights (B: the weights of the same points, up to
// 32 right-hand sides), so E never leaves registers.  Products are summed in
// FP32 over a panel and in FP64 across panels; the columns are split across
// workgroups (split-K) and reduced in order afterwards.
#include "internal.hpp"
#include "wide.hpp"

namespace krr {
namespace {

typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int KW = 4;           // waves per workgroup
constexpr int KROWS = 32 * KW;  // rows per workgroup
constexpr int KPT = 4;          // 32-point tiles per panel
constexpr int KKC = 64;         // augmented coordinates: KP is a multiple of this
constexpr int BC = 32;          // augmented coordinates per LDS chunk
constexpr int BCS = 3 * BC;     // BF16 terms per chunk
constexpr int BLD = BCS + 8;    // staged row (16 bytes of padding)

typedef __bf16 bf8w __attribute__((ext_vector_type(8)));

// Three-term BF16 rows: for coordinate k = 32 c + j, slot 96 c + j holds its
// hi term, 96 c + 32 + j the mid term and 96 c + 64 + j the lo term.
__global__ void k_wide_pack(const float *__restrict__ A, int64_t n, int KP, __bf16 *__restrict__ P) {
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    for (int k = threadIdx.x; k < KP; k += blockDim.x) {
        const float v = A[i * KP + k];
        const __bf16 h = (__bf16)v;
        const float r1 = v - (float)h;
        const __bf16 mid = (__bf16)r1;
        const __bf16 lo = (__bf16)(r1 - (float)mid);
        __bf16 *row = P + i * (int64_t)KP * 3 + (int64_t)(k / BC) * BCS + (k % BC);
        row[0] = h;
        row[BC] = mid;
        row[2 * BC] = lo;
    }
}

// point of register s of a lane in half g of the wave (the C layout of the
// exponent GEMM): 8 (s / 4) + 4 g + s % 4
__device__ __forceinline__ int reg_point(int s, int g) { return 8 * (s >> 2) + 4 * g + (s & 3); }

__global__ __launch_bounds__(64 * KW) void k_kmv_wmfma(const __bf16 *__restrict__ XB, int64_t m,
                                                       const __bf16 *__restrict__ YB, int64_t n, int KP,
                                                       const float *__restrict__ wf, int nrhs, int rhs0, int nrc,
                                                       int64_t cols_per_split, double *__restrict__ part,
                                                       const SampBlock *__restrict__ bt) {
    constexpr int TH = 64 * KW;
    __shared__ __attribute__((aligned(16))) __bf16 lds[2 * KROWS * BLD];
    __bf16 *xs = lds;                  // [KROWS][BLD] rows
    __bf16 *ys = lds + KROWS * BLD;    // [KROWS][BLD] points
    float(*ws)[33] = reinterpret_cast<float(*)[33]>(lds);  // the panel's weights, after the GEMM

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 5;
    const int split = blockIdx.y;
    int64_t i0, iend, j0, j1;
    if (bt) {
        const SampBlock sb = bt[blockIdx.x];
        i0 = sb.i0;
        iend = sb.iend;
        j0 = sb.jlo + split * sb.cps;
        j1 = min(sb.jhi, j0 + sb.cps);
    } else {
        i0 = (int64_t)blockIdx.x * KROWS;
        iend = m;
        j0 = split * cols_per_split;
        j1 = min(n, j0 + cols_per_split);
    }
    const int64_t KP3 = (int64_t)KP * 3;
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    for (int64_t p0 = (j0 / 32) * 32; p0 < j1; p0 += 32 * KPT) {
        f16v t[KPT];
#pragma unroll
        for (int pt = 0; pt < KPT; ++pt)
#pragma unroll
            for (int q = 0; q < 16; ++q) t[pt][q] = 0.0f;
        for (int kc = 0; kc < KP; kc += BC) {
            // 16-byte pieces: KROWS rows x BCS / 8 pieces each, for both sides
            const int64_t coff = (int64_t)(kc / BC) * BCS;
            for (int u = tid; u < KROWS * (BCS / 8); u += TH) {
                const int rr = u / (BCS / 8), e8 = (u % (BCS / 8)) * 8;
                const int64_t gi = i0 + rr, gj = p0 + rr;
                const uint4 zero = {0u, 0u, 0u, 0u};
                *reinterpret_cast<uint4 *>(xs + rr * BLD + e8) =
                    gi < iend ? *reinterpret_cast<const uint4 *>(XB + gi * KP3 + coff + e8) : zero;
                *reinterpret_cast<uint4 *>(ys + rr * BLD + e8) =
                    (gj >= j0 && gj < j1) ? *reinterpret_cast<const uint4 *>(YB + gj * KP3 + coff + e8) : zero;
            }
            __syncthreads();
            // K halves of 16 coordinates; operands: term block (0 hi, 1 mid,
            // 2 lo) at 32 x block + 16 x half + 8 g within a staged row
            const __bf16 *xr = xs + (32 * w + (lane & 31)) * BLD + 8 * g;
#pragma unroll
            for (int kh = 0; kh < 2; ++kh) {
                const bf8w bh = *reinterpret_cast<const bf8w *>(xr + 16 * kh);
                const bf8w bm = *reinterpret_cast<const bf8w *>(xr + BC + 16 * kh);
                const bf8w bl = *reinterpret_cast<const bf8w *>(xr + 2 * BC + 16 * kh);
#pragma unroll
                for (int pt = 0; pt < KPT; ++pt) {
                    const __bf16 *yr = ys + (32 * pt + (lane & 31)) * BLD + 8 * g + 16 * kh;
                    const bf8w ah = *reinterpret_cast<const bf8w *>(yr);
                    const bf8w am = *reinterpret_cast<const bf8w *>(yr + BC);
                    const bf8w al = *reinterpret_cast<const bf8w *>(yr + 2 * BC);
                    t[pt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bm, t[pt], 0, 0, 0);
                    t[pt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, t[pt], 0, 0, 0);
                    t[pt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, t[pt], 0, 0, 0);
                    t[pt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bh, t[pt], 0, 0, 0);
                    t[pt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bm, t[pt], 0, 0, 0);
                    t[pt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, t[pt], 0, 0, 0);
                }
            }
            __syncthreads();
        }
    // the panel's weights (zero outside the column range and past nrc)
        for (int u = tid; u < 32 * KPT * 32; u += TH) {
            const int pp = u / 32, col = u % 32;
            const int64_t gj = p0 + pp;
            ws[pp][col] = (col < nrc && gj >= j0 && gj < j1) ? wf[gj * nrhs + rhs0 + col] : 0.0f;
        }
        __syncthreads();
        f16v pa;
#pragma unroll
        for (int q = 0; q < 16; ++q) pa[q] = 0.0f;
#pragma unroll
        for (int pt = 0; pt < KPT; ++pt)
#pragma unroll
            for (int sidx = 0; sidx < 16; ++sidx) {
                const int pp = 32 * pt + reg_point(sidx, g);
                const float e = __builtin_amdgcn_exp2f(t[pt][sidx]);  // masked points meet zero weights
                pa = __builtin_amdgcn_mfma_f32_32x32x2f32(e, ws[pp][lane & 31], pa, 0, 0, 0);
            }
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] += (double)pa[q];
        __syncthreads();
    }
    // lane: right-hand side lane % 32, rows 8 (q / 4) + 4 g + q % 4 of the wave's 32
    const int col = lane & 31;
    if (col < nrc) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int64_t row = i0 + 32 * w + 8 * (q >> 2) + 4 * g + (q & 3);
            if (row < iend) part[((int64_t)split * m + row) * nrhs + rhs0 + col] = acc[q];
        }
    }
}

__global__ void k_w_to_float_wide(const double *__restrict__ W, int64_t len, float *__restrict__ wf) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < len) wf[t] = (float)W[t];
}

__global__ void k_reduce_parts(const double *__restrict__ part, int nsplit, int64_t mn, double beta,
                               double *__restrict__ out) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= mn) return;
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * mn + t];
    out[t] = (beta != 0.0) ? s + beta * out[t] : s;
}

// FP64 entries: the exponent GEMM in FP64 on v_mfma_f64_16x16x4_f64.  A
// workgroup of 8 waves owns 128 rows (16 per wave) and walks the columns in
// panels of 128 points, accumulating t = x~_i . y~_j (natural-log units) over K
// chunks of 32 staged through LDS; in the FP64 C layout register q of lane l
// holds row l % 16 of the wave's rows against point l / 16 + 4 q of each
// 16-point tile.  exp (FP64) turns t into the entry, and the panel's weights
// (FP64, up to 16 right-hand sides per pass) are multiplied in on the vector
// ALUs: for d > 64 the GEMM's d + 2 FMAs per entry dominate the entry's cost.
constexpr int W64 = 8;            // waves per workgroup
constexpr int W64ROWS = 16 * W64;  // rows per workgroup
constexpr int W64PN = 128;         // points per panel (8 tiles of 16)
constexpr int W64KC = 32;          // augmented coordinates per LDS chunk
typedef double d4v __attribute__((ext_vector_type(4)));

template <int NR>
__global__ __launch_bounds__(64 * W64) void k_kmv_wmfma64(const double *__restrict__ XA, int64_t m,
                                                          const double *__restrict__ YA, int64_t n, int KP,
                                                          const double *__restrict__ W, int nrhs, int rhs0, int nrc,
                                                          int64_t cols_per_split, double *__restrict__ part,
                                                          const SampBlock *__restrict__ bt) {
    constexpr int TH = 64 * W64;
    constexpr int LDK = W64KC + 1;
    constexpr int PT = W64PN / 16;
    __shared__ double xs[W64ROWS][LDK];
    __shared__ double ys[W64PN][LDK];
    __shared__ double wsh[W64PN][NR];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = lane >> 4, lr = lane & 15;
    const int split = blockIdx.y;
    int64_t i0, iend, j0, j1;
    if (bt) {
        const SampBlock sb = bt[blockIdx.x];
        i0 = sb.i0;
        iend = sb.iend;
        j0 = sb.jlo + split * sb.cps;
        j1 = min(sb.jhi, j0 + sb.cps);
    } else {
        i0 = (int64_t)blockIdx.x * W64ROWS;
        iend = m;
        j0 = split * cols_per_split;
        j1 = min(n, j0 + cols_per_split);
    }
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = 0.0;
    for (int64_t p0 = j0; p0 < j1; p0 += W64PN) {
        d4v t[PT];
#pragma unroll
        for (int pt = 0; pt < PT; ++pt) t[pt] = d4v{0.0, 0.0, 0.0, 0.0};
        for (int kc = 0; kc < KP; kc += W64KC) {
            for (int u = tid; u < W64ROWS * W64KC; u += TH) {
                const int rr = u / W64KC, kk = u % W64KC;
                const int64_t gi = i0 + rr, gj = p0 + rr;  // W64ROWS == W64PN
                xs[rr][kk] = gi < iend ? XA[gi * KP + kc + kk] : 0.0;
                ys[rr][kk] = gj < j1 ? YA[gj * KP + kc + kk] : 0.0;
            }
            __syncthreads();
#pragma unroll 2
            for (int kk = 0; kk < W64KC; kk += 4) {
                const double b = xs[16 * wv + lr][kk + g];
#pragma unroll
                for (int pt = 0; pt < PT; ++pt)
                    t[pt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ys[16 * pt + lr][kk + g], b, t[pt], 0, 0, 0);
            }
            __syncthreads();
        }
        // the panel's weights (zero past the column range and past nrc)
        for (int u = tid; u < W64PN * NR; u += TH) {
            const int pp = u / NR, r = u % NR;
            const int64_t gj = p0 + pp;
            wsh[pp][r] = (r < nrc && gj < j1) ? W[gj * nrhs + rhs0 + r] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int pt = 0; pt < PT; ++pt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double e = exp(t[pt][q]);  // padded points meet zero weights
                const int pp = 16 * pt + g + 4 * q;
#pragma unroll
                for (int r = 0; r < NR; ++r) acc[r] = fma(e, wsh[pp][r], acc[r]);
            }
        // the next panel rewrites the weights only after its K loop's barriers
    }
    const int64_t row = i0 + 16 * wv + lr;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        double v = acc[r];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (g == 0 && r < nrc && row < iend) part[((int64_t)split * m + row) * nrhs + rhs0 + r] = v;
    }
}

}  // namespace

// Out = K(X, Y; h) W + beta Out with FP64 entries for d > 64 (T: the points'
// type; a batch multiplies its own points).
template <class T>
void kmv_wide_mfma64(const T *X, int64_t m, const T *Y, int64_t n, int d, double h, const double *W, int nrhs,
                     double beta, double *Out, hipStream_t s, const Batch *batch) {
    const int KP = (d + 2 + W64KC - 1) / W64KC * W64KC;
    const double cn = 1.0 / (2.0 * h * h);
    DBuf mean = dalloc<double>(d), XA = dalloc<double>((size_t)m * KP), YA = dalloc<double>((size_t)n * KP);
    DBuf pb, cp, btab;
    int64_t nb = 0, cps = 0;
    int nsplit;
    if (batch) {
        std::vector<double> cpr(batch->np());
        for (int k = 0; k < batch->np(); ++k) cpr[k] = 1.0 / (2.0 * batch->h[k] * batch->h[k]);
        pb = upload(batch->pbeg, s);
        cp = upload(cpr, s);
        std::vector<SampBlock> blocks = row_blocks(*batch, W64ROWS);
        nb = (int64_t)blocks.size();
        int64_t nmax = 0;
        for (int k = 0; k < batch->np(); ++k) nmax = std::max(nmax, batch->size(k));
        nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(tune_get(KRR_TUNE_MV_BLOCKS), nb),
                                                             ceil_div(nmax, 4 * W64PN)));
        for (auto &b : blocks) {
            int64_t c = ceil_div(b.jhi - b.jlo, nsplit);
            b.cps = (c + W64PN - 1) / W64PN * W64PN;
        }
        btab = upload(blocks, s);
        sync(s);
    } else {
        const int64_t rb = ceil_div(m, W64ROWS);
        nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(tune_get(KRR_TUNE_MV_BLOCKS), rb),
                                                             ceil_div(n, 4 * W64PN)));
        cps = (ceil_div(n, nsplit) + W64PN - 1) / W64PN * W64PN;
        nsplit = (int)ceil_div(n, cps);
    }
    k_col_mean<T><<<d, 256, 0, s>>>(Y, n, d, mean.as<double>());
    check_launch("k_col_mean");
    k_wide_aug64<T><<<(unsigned)m, 256, 0, s>>>(X, m, d, KP, mean.as<double>(), cn, pb.as<int64_t>(),
                                                cp.as<double>(), batch ? batch->np() : 0, 0, XA.as<double>());
    check_launch("k_wide_aug64");
    k_wide_aug64<T><<<(unsigned)n, 256, 0, s>>>(Y, n, d, KP, mean.as<double>(), cn, pb.as<int64_t>(),
                                                cp.as<double>(), batch ? batch->np() : 0, 1, YA.as<double>());
    check_launch("k_wide_aug64");
    DBuf part = dalloc<double>((size_t)nsplit * m * nrhs);
    if (batch && batch->any_skipped())  // rows of left-out problems reduce to 0
        KRR_HIP(hipMemsetAsync(part.get(), 0, sizeof(double) * nsplit * m * nrhs, s));
    dim3 grid((unsigned)(batch ? nb : ceil_div(m, W64ROWS)), nsplit);
    for (int r0 = 0; r0 < nrhs; r0 += 16) {
        const int nrc = std::min(16, nrhs - r0);
        if (nrc > 8) {
            k_kmv_wmfma64<16><<<grid, 64 * W64, 0, s>>>(XA.as<double>(), m, YA.as<double>(), n, KP, W, nrhs, r0, nrc,
                                                        cps, part.as<double>(), btab.as<SampBlock>());
        } else if (nrc > 2) {
            k_kmv_wmfma64<8><<<grid, 64 * W64, 0, s>>>(XA.as<double>(), m, YA.as<double>(), n, KP, W, nrhs, r0, nrc,
                                                       cps, part.as<double>(), btab.as<SampBlock>());
        } else {
            k_kmv_wmfma64<2><<<grid, 64 * W64, 0, s>>>(XA.as<double>(), m, YA.as<double>(), n, KP, W, nrhs, r0, nrc,
                                                       cps, part.as<double>(), btab.as<SampBlock>());
        }
        check_launch("k_kmv_wmfma64");
    }
    const int64_t mn = m * nrhs;
    k_reduce_parts<<<ceil_div(mn, 256), 256, 0, s>>>(part.as<double>(), nsplit, mn, beta, Out);
    check_launch("k_reduce_parts");
    sync(s);  // temporaries are released on return
}
template void kmv_wide_mfma64<float>(const float *, int64_t, const float *, int64_t, int, double, const double *, int,
                                     double, double *, hipStream_t, const Batch *);
template void kmv_wide_mfma64<double>(const double *, int64_t, const double *, int64_t, int, double, const double *,
                                      int, double, double *, hipStream_t, const Batch *);

// Out = K(X, Y; h) W + beta Out with FP32 entries for d > 64 (X: m FP32
// points, Y: n FP32 points; a batch multiplies its own points).
void kmv_wide_mfma(const float *X, int64_t m, const float *Y, int64_t n, int d, double h, const double *W, int nrhs,
                   double beta, double *Out, hipStream_t s, const Batch *batch) {
    const int KP = (d + 2 + KKC - 1) / KKC * KKC;
    const double c2 = 1.4426950408889634 / (2.0 * h * h);
    DBuf mean = dalloc<double>(d), XA = dalloc<float>((size_t)m * KP), YA = dalloc<float>((size_t)n * KP);
    DBuf wf = dalloc<float>((size_t)n * nrhs), pb, cp, btab;
    int64_t nb = 0, cps = 0;
    int nsplit;
    if (batch) {
        std::vector<double> cpr(batch->np());
        for (int k = 0; k < batch->np(); ++k) cpr[k] = 1.4426950408889634 / (2.0 * batch->h[k] * batch->h[k]);
        pb = upload(batch->pbeg, s);
        cp = upload(cpr, s);
        std::vector<SampBlock> blocks = row_blocks(*batch, KROWS);
        nb = (int64_t)blocks.size();
        int64_t nmax = 0;
        for (int k = 0; k < batch->np(); ++k) nmax = std::max(nmax, batch->size(k));
        nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(tune_get(KRR_TUNE_MV_BLOCKS), nb),
                                                             ceil_div(nmax, 4 * 32 * KPT)));
        for (auto &b : blocks) {
            int64_t c = ceil_div(b.jhi - b.jlo, nsplit);
            b.cps = (c + 127) / 128 * 128;
        }
        btab = upload(blocks, s);
        sync(s);
    } else {
        const int64_t rb = ceil_div(m, KROWS);
        nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(tune_get(KRR_TUNE_MV_BLOCKS), rb),
                                                             ceil_div(n, 4 * 32 * KPT)));
        cps = (ceil_div(n, nsplit) + 127) / 128 * 128;
        nsplit = (int)ceil_div(n, cps);
    }
    // one anchor for rows and columns: the mean of the columns' points
    k_col_mean<float><<<d, 256, 0, s>>>(Y, n, d, mean.as<double>());
    check_launch("k_col_mean");
    k_wide_aug<<<(unsigned)m, 256, 0, s>>>(X, m, d, KP, mean.as<double>(), c2, pb.as<int64_t>(), cp.as<double>(),
                                          batch ? batch->np() : 0, 0.0f, 0, XA.as<float>());
    check_launch("k_wide_aug");
    k_wide_aug<<<(unsigned)n, 256, 0, s>>>(Y, n, d, KP, mean.as<double>(), c2, pb.as<int64_t>(), cp.as<double>(),
                                          batch ? batch->np() : 0, 0.0f, 1, YA.as<float>());
    check_launch("k_wide_aug");
    k_w_to_float_wide<<<ceil_div(n * nrhs, 256), 256, 0, s>>>(W, n * nrhs, wf.as<float>());
    check_launch("k_w_to_float_wide");
    DBuf XB = dalloc<__bf16>((size_t)m * KP * 3), YB = dalloc<__bf16>((size_t)n * KP * 3);
    k_wide_pack<<<(unsigned)m, 256, 0, s>>>(XA.as<float>(), m, KP, XB.as<__bf16>());
    check_launch("k_wide_pack");
    k_wide_pack<<<(unsigned)n, 256, 0, s>>>(YA.as<float>(), n, KP, YB.as<__bf16>());
    check_launch("k_wide_pack");
    DBuf part = dalloc<double>((size_t)nsplit * m * nrhs);
    if (batch && batch->any_skipped())  // rows of left-out problems reduce to 0
        KRR_HIP(hipMemsetAsync(part.get(), 0, sizeof(double) * nsplit * m * nrhs, s));
    dim3 grid((unsigned)(batch ? nb : ceil_div(m, KROWS)), nsplit);
    for (int r0 = 0; r0 < nrhs; r0 += 32) {
        const int nrc = std::min(32, nrhs - r0);
        k_kmv_wmfma<<<grid, 64 * KW, 0, s>>>(XB.as<__bf16>(), m, YB.as<__bf16>(), n, KP, wf.as<float>(), nrhs, r0,
                                            nrc, cps, part.as<double>(), btab.as<SampBlock>());
        check_launch("k_kmv_wmfma");
    }
    const int64_t mn = m * nrhs;
    k_reduce_parts<<<ceil_div(mn, 256), 256, 0, s>>>(part.as<double>(), nsplit, mn, beta, Out);
    check_launch("k_reduce_parts");
    sync(s);  // temporaries are released on return
}

}  // namespace krr
