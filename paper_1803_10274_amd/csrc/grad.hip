// Backward of the fused kernel product Out = K(X, Y; h) W for an upstream
// gradient G.  With P = K o (G W^T) (never stored):
//   dW   = K(X, Y)^T G = K(Y, X) G                     (a kernel product)
//   dX_i = -(1/h^2) [ (sum_j P_ij) x_i - (P Y)_i ]
//   dY_j = -(1/h^2) [ (sum_i P_ij) y_j - (P^T X)_j ]   (same form, roles swapped)
//   dh   = sum_ij P_ij ||x_i - y_j||^2 / h^3
// One thread per row of the left operand; right-operand tiles in LDS; FP32
// entries from exact differences inside a 64-column tile, FP64 across tiles
// (FP64 throughout for prec = KRR_F64).  dh alone with FP32 entries and one
// right-hand side (the validation-loss gradient) is a kernel product instead:
// the entry exp2(t) t on the products' split-K kernel, then a dot with G.
#include "internal.hpp"

namespace krr {


namespace {
constexpr int GB_ROWS = 256, GB_TN = 32, GB_DMAX = 64, GB_RMAX = 16;

__device__ __forceinline__ float gexp(float q, float s2) { return __builtin_amdgcn_exp2f(-q * s2); }
__device__ __forceinline__ double gexp(double q, double s) { return exp(-q * s); }

// For rows a of A: s_a = sum_b P_ab, t_a = sum_b P_ab B_b, u_a = sum_b P_ab ||A_a - B_b||^2
// with P_ab = K(A_a, B_b) (GA_a . GB_b).  Writes dA_a = -(1/h^2)(s_a A_a - t_a)
// and u_a (for dh) when the pointers are given.
// D: the point width padded up (8, 16, 32 or 64); NR: 1 or up to 16
// right-hand sides.
template <class T, class C, int D, int NR>
__global__ __launch_bounds__(GB_ROWS) void k_bwd_rows(const T *__restrict__ A, int64_t ma, const T *__restrict__ B,
                                                      int64_t nb, int d, C scale, const double *__restrict__ GA,
                                                      const double *__restrict__ GB, int nrhs, double inv_h2,
                                                      double *__restrict__ dA, double *__restrict__ u_out) {
    __shared__ C bs[GB_TN][D];
    __shared__ C gbs[GB_TN][NR];
    const int tid = threadIdx.x;
    const int64_t a = (int64_t)blockIdx.x * GB_ROWS + tid;
    C xa[D];
    C ga[NR];
#pragma unroll
    for (int k = 0; k < D; ++k) xa[k] = (a < ma && k < d) ? (C)A[a * d + k] : (C)0;
#pragma unroll
    for (int r = 0; r < NR; ++r) ga[r] = (a < ma && r < nrhs) ? (C)GA[a * nrhs + r] : (C)0;
    double s = 0.0, u = 0.0;
    double t[D];
#pragma unroll
    for (int k = 0; k < D; ++k) t[k] = 0.0;
    for (int64_t j0 = 0; j0 < nb; j0 += GB_TN) {
        for (int e = tid; e < GB_TN * D; e += GB_ROWS) {
            int jj = e / D, k = e % D;
            int64_t j = j0 + jj;
            bs[jj][k] = (j < nb && k < d) ? (C)B[j * d + k] : (C)0;
        }
        for (int e = tid; e < GB_TN * NR; e += GB_ROWS) {
            int jj = e / NR, r = e % NR;
            int64_t j = j0 + jj;
            gbs[jj][r] = (j < nb && r < nrhs) ? (C)GB[j * nrhs + r] : (C)0;
        }
        __syncthreads();
        C ps = 0, pu = 0;
        C pt[D];
#pragma unroll
        for (int k = 0; k < D; ++k) pt[k] = 0;
        for (int jj = 0; jj < GB_TN; ++jj) {
            C q = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                C df = xa[k] - bs[jj][k];
                q = fma(df, df, q);
            }
            C g = 0;
#pragma unroll
            for (int r = 0; r < NR; ++r) g = fma(ga[r], gbs[jj][r], g);
            C p = gexp(q, scale) * g;
            ps += p;
            pu = fma(p, q, pu);
#pragma unroll
            for (int k = 0; k < D; ++k) pt[k] = fma(p, bs[jj][k], pt[k]);
        }
        s += (double)ps;
        u += (double)pu;
#pragma unroll
        for (int k = 0; k < D; ++k) t[k] += (double)pt[k];
        __syncthreads();
    }
    if (a >= ma) return;
    if (dA)
        for (int k = 0; k < d; ++k) dA[a * d + k] = -inv_h2 * (s * (double)A[a * d + k] - t[k]);
    if (u_out) u_out[a] = u;
}

__global__ void k_sum_scaled(const double *__restrict__ u, int64_t m, double scale, double *__restrict__ out) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) acc += u[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) *out = scale * (red[0] + red[1] + red[2] + red[3]);
}

template <class T, class C, int D>
void bwd_rows_d(const T *A, int64_t ma, const T *B, int64_t nb, int d, C scale, const double *GA, const double *GB,
                int nrhs, double inv_h2, double *dA, double *u, hipStream_t s) {
    if (nrhs == 1)
        k_bwd_rows<T, C, D, 1><<<ceil_div(ma, GB_ROWS), GB_ROWS, 0, s>>>(A, ma, B, nb, d, scale, GA, GB, nrhs, inv_h2,
                                                                         dA, u);
    else
        k_bwd_rows<T, C, D, GB_RMAX><<<ceil_div(ma, GB_ROWS), GB_ROWS, 0, s>>>(A, ma, B, nb, d, scale, GA, GB, nrhs,
                                                                               inv_h2, dA, u);
    check_launch("k_bwd_rows");
}

template <class T, class C>
void bwd_rows(const T *A, int64_t ma, const T *B, int64_t nb, int d, double h, const double *GA, const double *GB,
              int nrhs, double *dA, double *u, hipStream_t s) {
    C scale = (sizeof(C) == 4) ? (C)(1.4426950408889634 / (2.0 * h * h)) : (C)(1.0 / (2.0 * h * h));
    const double ih2 = 1.0 / (h * h);
    if (d <= 8)
        bwd_rows_d<T, C, 8>(A, ma, B, nb, d, scale, GA, GB, nrhs, ih2, dA, u, s);
    else if (d <= 16)
        bwd_rows_d<T, C, 16>(A, ma, B, nb, d, scale, GA, GB, nrhs, ih2, dA, u, s);
    else if (d <= 32)
        bwd_rows_d<T, C, 32>(A, ma, B, nb, d, scale, GA, GB, nrhs, ih2, dA, u, s);
    else
        bwd_rows_d<T, C, GB_DMAX>(A, ma, B, nb, d, scale, GA, GB, nrhs, ih2, dA, u, s);
}

// dh = scale sum_a G_a v_a (one block, fixed order: deterministic)
// One workgroup of up to 1024 threads; the waves' sums are added in a fixed
// order, so the result is deterministic.
__global__ __launch_bounds__(1024) void k_dot_scaled(const double *__restrict__ g, const double *__restrict__ v,
                                                     int64_t m, double scale, double *__restrict__ out) {
    __shared__ double red[16];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) acc += g[i] * v[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        *out = scale * t;
    }
}

template <class T>
void bwd_typed(const T *X, int64_t m, const T *Y, int64_t n, int d, double h, const double *W, const double *G,
               int nrhs, double *dX, double *dY, double *dh, int prec, hipStream_t s) {
    DBuf u;
    if (dh) u = dalloc<double>(m);
    if (dX || dh) {
        if (prec == KRR_F64)
            bwd_rows<T, double>(X, m, Y, n, d, h, G, W, nrhs, dX, dh ? u.as<double>() : nullptr, s);
        else
            bwd_rows<T, float>(X, m, Y, n, d, h, G, W, nrhs, dX, dh ? u.as<double>() : nullptr, s);
    }
    if (dY) {
        if (prec == KRR_F64)
            bwd_rows<T, double>(Y, n, X, m, d, h, W, G, nrhs, dY, nullptr, s);
        else
            bwd_rows<T, float>(Y, n, X, m, d, h, W, G, nrhs, dY, nullptr, s);
    }
    if (dh) {
        k_sum_scaled<<<1, 256, 0, s>>>(u.as<double>(), m, 1.0 / (h * h * h), dh);
        check_launch("k_sum_scaled");
        sync(s);
    }
}
}  // namespace

namespace {
// Validation residual of one column: e = f - y_v, ge = (2 / m) e and
// loss = |e|^2 / m, summed in a fixed order (strided per thread, then a tree
// over the block) so the result is deterministic.
__global__ __launch_bounds__(256) void k_val_residual(const double *__restrict__ f, const double *__restrict__ yv,
                                                      int64_t m, int k, double *__restrict__ ge,
                                                      double *__restrict__ loss) {
    __shared__ double part[256];
    const int c = blockIdx.x, tid = threadIdx.x;
    const double sc = 2.0 / (double)m;
    double acc = 0.0;
    for (int64_t i = tid; i < m; i += 256) {
        const double e = f[i * k + c] - yv[i * k + c];
        ge[i * k + c] = sc * e;
        acc += e * e;
    }
    part[tid] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) part[tid] += part[tid + o];
        __syncthreads();
    }
    if (tid == 0) loss[c] = part[0] / (double)m;
}

// (dL/dlog h, dL/dlog lambda) = g (h (dh_v - dh_t), -lambda beta^T alpha)
__global__ void k_val_grad_finish(const double *bta, const double *dh_v, const double *dh_t, const double *gscale,
                                  double h, double lam, double *out) {
    if (threadIdx.x != 0) return;
    const double g = gscale ? gscale[0] : 1.0;
    out[0] = g * (h * (dh_v[0] - dh_t[0]));
    out[1] = g * (-lam * bta[0]);
}
}  // namespace

void val_residual(const double *f, const double *yv, int64_t m, int k, double *ge, double *loss, hipStream_t s) {
    k_val_residual<<<k, 256, 0, s>>>(f, yv, m, k, ge, loss);
    check_launch("k_val_residual");
}

void val_grad_finish(const double *bta, const double *dh_v, const double *dh_t, const double *gscale, double h,
                     double lam, double *out, hipStream_t s) {
    k_val_grad_finish<<<1, 64, 0, s>>>(bta, dh_v, dh_t, gscale, h, lam, out);
    check_launch("k_val_grad_finish");
}

void kernel_matvec_bwd_impl(const void *X, int64_t m, const void *Y, int64_t n, int d, int xprec, double h,
                            const double *W, const double *G, int nrhs, double *dX, double *dY, double *dW,
                            double *dh, int prec, hipStream_t s) {
    KRR_REQUIRE(d <= GB_DMAX, "kernel_matvec_bwd: d = %d exceeds %d", d, GB_DMAX);
    KRR_REQUIRE(nrhs <= GB_RMAX, "kernel_matvec_bwd: nrhs = %d exceeds %d", nrhs, GB_RMAX);
    if (dW) kernel_matvec_impl(Y, n, X, m, d, xprec, h, G, nrhs, 0.0, dW, prec, s);
    if (dh && !dX && !dY && prec == KRR_F32 && nrhs == 1) {
        // dh alone: sum_ab P_ab q_ab / h^3 = sum_a G_a [(K o Q) W]_a / h^3, and
        // K o Q = -(1 / c) exp2(t) t with t = -c q in log2 units: a kernel
        // product whose entry is exp2(t) t, on the products' fast kernel
        DBuf v = dalloc<double>(m);
        kernel_matvec_q(X, m, Y, n, d, xprec, h, W, v.as<double>(), s);
        const double c = 1.4426950408889634 / (2.0 * h * h);
        k_dot_scaled<<<1, 1024, 0, s>>>(G, v.as<double>(), m, -1.0 / (c * h * h * h), dh);
        check_launch("k_dot_scaled");
        sync(s);
        return;
    }
    if (xprec == KRR_F64)
        bwd_typed<double>(static_cast<const double *>(X), m, static_cast<const double *>(Y), n, d, h, W, G, nrhs, dX,
                          dY, dh, prec, s);
    else
        bwd_typed<float>(static_cast<const float *>(X), m, static_cast<const float *>(Y), n, d, h, W, G, nrhs, dX, dY,
                         dh, prec, s);
}

}  // namespace krr
