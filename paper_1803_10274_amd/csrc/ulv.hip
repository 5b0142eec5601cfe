// ULV factorization and solve of K_hss + lambda I (Section 3.1; lambda is
// added to the leaf diagonal blocks only, Section 5.3).
//
// Bottom-up over the levels, one workgroup per node (levels with few, large
// nodes spread their products over many workgroups: kPhasedNodes), with the
// node's dense block Dw (m x m) and basis Uw (m x k):
//   leaf    Dw = D + lambda I,  Uw = U
//   parent  Dw = [[S_a, Rh_a B_ab Rh_b^T], [(.)^T, S_b]],  Uw = diag(Rh_a, Rh_b) U
// 1. Householder QR  Q^T Uw = [Rh; 0]  (Rh k x k is passed to the parent);
// 2. Dw <- Q^T Dw Q;  the last m - k rows no longer couple to the rest of the
//    matrix, so with Dw = [[A_cc, A_ce], [A_ec, A_ee]]:
// 3. A_ee = L L^T (Cholesky), W = A_ce L^{-T}, S = A_cc - W W^T (passed up);
// the root factors its whole Dw.  The factor keeps Q in compact WY form
// (Q = I - V T V^T) and L^{-1} explicitly, so that every step of the solve
// is a parallel matrix-vector product.  Solve: forward sweep b <- Q^T b,
// z = L^{-1} b_e, c = b_c - W z passed up; root solve; backward sweep
// x_e = L^{-T} (z - W^T x_c), x = Q [x_c; x_e].
#include <algorithm>
#include <cstring>
#include <memory>

#include "dense.hpp"
#include "internal.hpp"

namespace krr {
namespace {

// Levels with fewer nodes than this factor in phases with their products
// spread over many workgroups (k_tile_gemms).
constexpr int kPhasedNodes = 64;

struct UlvDesc {
    int32_t m, k, kl, kr, leaf, root;
    int32_t prob;                      // the node's problem (batch)
    int32_t qr_done;                   // V, tau, Tw and Rh_out are in place from an earlier pass
    double lambda, pivot_floor;        // of the node's problem
    const double *D, *U, *B;           // HSS generators
    const double *S_l, *S_r, *Rh_l, *Rh_r;
    double *Dw, *Uw, *Tmp;             // scratch
    double *Yw, *Zw;                   // scratch of the blocked transform: k x m, k x m
    double *Sw;                        // scratch of the blocked inverse: 32 x m
    double *V, *tau, *Tw, *L, *W;      // factor (Tw: the WY T, k x k; L: the inverse Cholesky factor)
    double *S_out, *Rh_out;            // passed to the parent
};

constexpr int QR_NB = 16;  // panel width of the blocked QR (and block of T)
constexpr int CH_NB = 32;  // panel width of the blocked Cholesky and of L^{-1}'s blocks

// The diagonal block T_p (pb x pb, pb <= 32) of the compact WY factor from
// G_p = V_p^T V_p (row-major pb x pb) and the reflectors' tau, by the
// recurrence T(i, j) = -tau_j sum_{l=i}^{j-1} T(i, l) G(l, j), T(j, j) = tau_j,
// in LDS; written to T (leading dimension ldt).
__device__ void wy_diag_block(const double *tau, const double *G, int pb, double *T, int ldt, double (*blk)[33]) {
    double(*g)[33] = blk, (*t)[33] = blk + 32;
    const int tid = threadIdx.x;
    for (int e = tid; e < pb * pb; e += BG_T) {
        g[e / pb][e % pb] = G[e];
        t[e / pb][e % pb] = 0.0;
    }
    __syncthreads();
    for (int j = 0; j < pb; ++j) {
        if (tid < j) {
            double acc = 0.0;
            for (int l = tid; l < j; ++l) acc += t[tid][l] * g[l][j];
            t[tid][j] = -tau[j] * acc;
        }
        if (tid == j) t[j][j] = tau[j];
        __syncthreads();
    }
    for (int e = tid; e < pb * pb; e += BG_T) T[(int64_t)(e / pb) * ldt + e % pb] = t[e / pb][e % pb];
    __syncthreads();
}

// Phase 1: assemble Dw and Uw, Householder QR of Uw (V, tau, Rh_out) and the
// compact WY factor T (Tw).
__device__ void ulv_assemble_qr(const UlvDesc &q, double *smem, double *red, double (*blk)[33]) {
    const int m = q.m, k = q.k, tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
    double *Dw = q.Dw, *Uw = q.Uw;
    // ---- assemble
    if (q.leaf) {
        for (int t = tid; t < m * m; t += BG_T) Dw[t] = q.D[t] + ((t / m == t % m) ? q.lambda : 0.0);
        if (!q.qr_done)
            for (int t = tid; t < m * k; t += BG_T) Uw[t] = q.U[t];
    } else {
        const int kl = q.kl, kr = q.kr;
        for (int t = tid; t < kl * kl; t += BG_T) Dw[(t / kl) * m + t % kl] = q.S_l[t];
        for (int t = tid; t < kr * kr; t += BG_T) Dw[(kl + t / kr) * m + kl + t % kr] = q.S_r[t];
        __syncthreads();
        // Tmp = B Rh_r^T (kl x kr);  Dw[0:kl, kl:] = Rh_l Tmp
        block_gemm(kl, kr, kr, 1.0, q.B, kr, 1, q.Rh_r, 1, kr, 0.0, q.Tmp, kr, smem);
        block_gemm(kl, kr, kl, 1.0, q.Rh_l, kl, 1, q.Tmp, kr, 1, 0.0, Dw + kl, m, smem);
        for (int t = tid; t < kl * kr; t += BG_T) {
            int i = t / kr, j = t % kr;
            Dw[(int64_t)(kl + j) * m + i] = Dw[(int64_t)i * m + kl + j];
        }
        if (!q.root && !q.qr_done) {
            block_gemm(kl, k, kl, 1.0, q.Rh_l, kl, 1, q.U, k, 1, 0.0, Uw, k, smem);
            block_gemm(kr, k, kr, 1.0, q.Rh_r, kr, 1, q.U + (int64_t)kl * k, k, 1, 0.0, Uw + (int64_t)kl * k, k, smem);
        }
    }
    __syncthreads();
    if (q.qr_done) return;  // the basis's QR does not depend on lambda or the shift
    // ---- Householder QR of Uw (reflectors in V, tau), blocked: panels of
    // QR_NB columns are factored column by column, the columns right of a
    // panel get its block reflector Q_p^T = I - V_p T_p^T V_p^T as three
    // products.  T_p is the diagonal block of the compact WY factor T of
    // Q = H_0 ... H_(k-1) = I - V T V^T, whose column j is T(0:j, j) =
    // -tau_j T(0:j, 0:j) G(0:j, j), T(j, j) = tau_j, G = V^T V.
    for (int t = tid; t < k * k; t += BG_T) q.Tw[t] = 0.0;
    __syncthreads();
    for (int p0 = 0; p0 < k; p0 += QR_NB) {
        const int p1 = min(k, p0 + QR_NB), pb = p1 - p0;
        for (int j = p0; j < p1; ++j) {
            double part = 0.0;
            for (int i = j + 1 + tid; i < m; i += BG_T) part += Uw[(int64_t)i * k + j] * Uw[(int64_t)i * k + j];
            double sig = block_sum(part, red);
            double alpha = Uw[(int64_t)j * k + j];
            double tau, beta, scal;
            if (sig == 0.0) {
                tau = 0.0;
                beta = alpha;
                scal = 0.0;
            } else {
                double nrm = sqrt(alpha * alpha + sig);
                beta = alpha >= 0.0 ? -nrm : nrm;
                tau = (beta - alpha) / beta;
                scal = 1.0 / (alpha - beta);
            }
            // reflector v: v[j] = 1, v[i > j] = x[i] * scal; stored in column j of V
            for (int i = tid; i < m; i += BG_T) {
                double v = (i < j) ? 0.0 : (i == j ? 1.0 : Uw[(int64_t)i * k + j] * scal);
                q.V[(int64_t)i * k + j] = v;
            }
            if (tid == 0) q.tau[j] = tau;
            __syncthreads();
            // the panel's columns c > j: a wave per column, lanes over rows
            const double *v = q.V + j;  // stride k
            for (int c = j + 1 + wv; c < p1; c += BG_T / 64) {
                double w = 0.0;
                for (int i = j + ln; i < m; i += 64) w += v[(int64_t)i * k] * Uw[(int64_t)i * k + c];
                w = tau * wave_sum(w);
                for (int i = j + ln; i < m; i += 64) Uw[(int64_t)i * k + c] -= w * v[(int64_t)i * k];
            }
            __syncthreads();
            if (tid == 0) Uw[(int64_t)j * k + j] = beta;
            for (int i = j + 1 + tid; i < m; i += BG_T) Uw[(int64_t)i * k + j] = 0.0;
            __syncthreads();
        }
        // T_p from G_p = V_p^T V_p (rows p0..m) by the recurrence, in LDS
        double *Gs = q.Yw;  // pb x pb
        block_gemm(pb, pb, m - p0, 1.0, q.V + (int64_t)p0 * k + p0, 1, k, q.V + (int64_t)p0 * k + p0, k, 1, 0.0, Gs,
                   pb, smem);
        wy_diag_block(q.tau + p0, Gs, pb, q.Tw + (int64_t)p0 * k + p0, k, blk);
        if (p1 < k) {
            // Uw(p0:m, p1:k) -= V_p (T_p^T (V_p^T Uw(p0:m, p1:k)))
            const int nt = k - p1;
            double *W1 = q.Yw, *W2 = q.Zw;  // pb x nt each
            block_gemm(pb, nt, m - p0, 1.0, q.V + (int64_t)p0 * k + p0, 1, k, Uw + (int64_t)p0 * k + p1, k, 1, 0.0,
                       W1, nt, smem);
            block_gemm(pb, nt, pb, 1.0, q.Tw + (int64_t)p0 * k + p0, 1, k, W1, nt, 1, 0.0, W2, nt, smem);
            block_gemm(m - p0, nt, pb, -1.0, q.V + (int64_t)p0 * k + p0, k, 1, W2, nt, 1, 1.0,
                       Uw + (int64_t)p0 * k + p1, k, smem);
        }
    }
    // ---- the rest of T, block column by block column:
    // T(0:p0, p0:p1) = -T(0:p0, 0:p0) G(0:p0, p0:p1) T_p
    for (int p0 = QR_NB; p0 < k; p0 += QR_NB) {
        const int p1 = min(k, p0 + QR_NB), pb = p1 - p0;
        double *Gc = q.Yw, *Z = q.Zw;  // p0 x pb each
        block_gemm(p0, pb, m - p0, 1.0, q.V + (int64_t)p0 * k, 1, k, q.V + (int64_t)p0 * k + p0, k, 1, 0.0, Gc, pb,
                   smem);
        block_gemm(p0, pb, pb, 1.0, Gc, pb, 1, q.Tw + (int64_t)p0 * k + p0, k, 1, 0.0, Z, pb, smem);
        block_gemm(p0, pb, p0, -1.0, q.Tw, k, 1, Z, pb, 1, 0.0, q.Tw + p0, k, smem);
    }
    if (!q.root)
        for (int t = tid; t < k * k; t += BG_T) {
            int i = t / k, c = t % k;
            q.Rh_out[t] = (c >= i) ? Uw[(int64_t)i * k + c] : 0.0;
        }
    __syncthreads();
}

// Phase 2: Dw <- Q^T Dw Q as GEMMs: left Dw -= V (T^T (V^T Dw)), right
// Dw -= ((Dw V) T) V^T.  The six products, as batch jobs (j < 6) or one
// workgroup's block products.
__device__ __forceinline__ GemmJob ulv_transform_job(const UlvDesc &q, int j) {
    const int m = q.m, k = q.k;
    double *Y = q.Yw, *Z = q.Zw, *Dw = q.Dw;
    switch (j) {
        case 0: return {k, m, m, 1.0, 0.0, q.V, 1, k, Dw, m, 1, Y, m};        // Y = V^T Dw   (k x m)
        case 1: return {k, m, k, 1.0, 0.0, q.Tw, 1, k, Y, m, 1, Z, m};       // Z = T^T Y    (k x m)
        case 2: return {m, m, k, -1.0, 1.0, q.V, k, 1, Z, m, 1, Dw, m};      // Dw -= V Z
        case 3: return {m, k, m, 1.0, 0.0, Dw, m, 1, q.V, k, 1, Y, k};       // Y = Dw V     (m x k)
        case 4: return {m, k, k, 1.0, 0.0, Y, k, 1, q.Tw, k, 1, Z, k};       // Z = Y T      (m x k)
        default: return {m, m, k, -1.0, 1.0, Z, k, 1, q.V, 1, k, Dw, m};     // Dw -= Z V^T
    }
}

__device__ void ulv_transform(const UlvDesc &q, double *smem) {
    if (q.k <= 0) return;
    for (int j = 0; j < 6; ++j) {
        const GemmJob J = ulv_transform_job(q, j);
        block_gemm(J.M, J.N, J.K, J.alpha, J.A, J.as0, J.as1, J.B, J.bs0, J.bs1, J.beta, J.C, J.ldc, smem);
    }
}

// Phase 3: Cholesky of A_ee and its inverse; false (and the flag raised) on a
// non-positive pivot.
__device__ bool ulv_chol_inv(const UlvDesc &q, int32_t *flag, unsigned long long *clamped,
                             unsigned long long *worst, double *red, double *smem, double (*blk)[33]) {
    const double pivot_floor = q.pivot_floor;
    const int m = q.m, k = q.k, ne = m - k, tid = threadIdx.x;
    double *Dw = q.Dw;
    // ---- Cholesky of A_ee = Dw[k:, k:] (right-looking, in place).  With a
    // pivot floor, a pivot d below it is replaced, as in the modified Cholesky
    // of Gill, Murray and Wright, by max(floor, |d|, theta^2 / beta^2), theta
    // the largest entry below the pivot and beta^2 the largest diagonal entry
    // of A_ee: this bounds the factor's entries by beta (no growth) and adds a
    // nonnegative diagonal term.
    bool bad = false;
    double beta2 = 0.0;
    if (pivot_floor > 0.0) {
        double mx = 0.0;
        for (int i = tid; i < ne; i += BG_T) mx = fmax(mx, fabs(Dw[(int64_t)(k + i) * m + k + i]));
        mx = wave_max(mx);
        __syncthreads();
        if ((tid & 63) == 0) red[tid >> 6] = mx;
        __syncthreads();
        for (int i = 0; i < BG_T / 64; ++i) beta2 = fmax(beta2, red[i]);
        beta2 = fmax(beta2, pivot_floor);
        __syncthreads();
    }
    // blocked: panels of CH_NB columns factored column by column (each
    // column updates the rest of its panel), then the trailing block gets
    // A22 -= L21 L21^T as one product
    for (int p0 = 0; p0 < ne && !bad; p0 += CH_NB) {
        const int p1 = min(ne, p0 + CH_NB);
        for (int j = p0; j < p1; ++j) {
            double *Ajj = Dw + (int64_t)(k + j) * m + k + j;
            double djj = *Ajj;
            if (!(djj == djj) || isinf(djj)) {
                bad = true;
                break;
            }
            if (pivot_floor > 0.0 && !(djj >= pivot_floor)) {
                double th = 0.0;
                for (int i = j + 1 + tid; i < ne; i += BG_T) th = fmax(th, fabs(Dw[(int64_t)(k + i) * m + k + j]));
                th = wave_max(th);
                __syncthreads();
                if ((tid & 63) == 0) red[tid >> 6] = th;
                __syncthreads();
                double theta = 0.0;
                for (int i = 0; i < BG_T / 64; ++i) theta = fmax(theta, red[i]);
                if (tid == 0) {
                    atomicAdd(clamped + q.prob, 1ull);
                    // largest deficit below the floor (non-negative, so its bits order like integers)
                    atomicMax(worst + q.prob, (unsigned long long)__double_as_longlong(pivot_floor - djj));
                }
                djj = fmax(fmax(pivot_floor, fabs(djj)), theta * theta / beta2);
            }
            if (!(djj > 0.0)) {
                bad = true;
                break;
            }
            double ljj = sqrt(djj);
            __syncthreads();
            if (tid == 0) *Ajj = ljj;
            for (int i = j + 1 + tid; i < ne; i += BG_T) Dw[(int64_t)(k + i) * m + k + j] /= ljj;
            __syncthreads();
            for (int i = j + 1 + tid; i < ne; i += BG_T) {
                double lij = Dw[(int64_t)(k + i) * m + k + j];
                double *rowi = Dw + (int64_t)(k + i) * m + k;
                const int cend = min(i, p1 - 1);
                for (int c = j + 1; c <= cend; ++c) rowi[c] -= lij * Dw[(int64_t)(k + c) * m + k + j];
            }
            __syncthreads();
        }
        if (!bad && p1 < ne)
            block_gemm(ne - p1, ne - p1, p1 - p0, -1.0, Dw + (int64_t)(k + p1) * m + k + p0, m, 1,
                       Dw + (int64_t)(k + p1) * m + k + p0, 1, m, 1.0, Dw + (int64_t)(k + p1) * m + k + p1, m, smem);
    }
    if (bad) {
        if (tid == 0) atomicOr(flag, 1);
        return false;
    }
    // L^{-1} (lower triangular, zeros stored above the diagonal) in blocks of
    // CH_NB: the diagonal block X_II = L_II^{-1} by substitution in LDS, then
    // X(I, 0:I) = -X_II (L(I, 0:I) X(0:I, 0:I)) as two products
    for (int t = tid; t < ne * ne; t += BG_T) q.L[t] = 0.0;
    __syncthreads();
    for (int I0 = 0; I0 < ne; I0 += CH_NB) {
        const int nb = min(CH_NB, ne - I0);
        double(*lb)[33] = blk, (*xb)[33] = blk + 32;
        for (int e = tid; e < nb * nb; e += BG_T) {
            const int i = e / nb, c = e % nb;
            lb[i][c] = Dw[(int64_t)(k + I0 + i) * m + k + I0 + c];
            xb[i][c] = 0.0;
        }
        __syncthreads();
        if (tid < nb) {
            const int c = tid;
            for (int i = c; i < nb; ++i) {
                double t = (i == c) ? 1.0 : 0.0;
                for (int l = c; l < i; ++l) t -= lb[i][l] * xb[l][c];
                xb[i][c] = t / lb[i][i];
            }
        }
        __syncthreads();
        for (int e = tid; e < nb * nb; e += BG_T) {
            const int i = e / nb, c = e % nb;
            if (c <= i) q.L[(int64_t)(I0 + i) * ne + I0 + c] = xb[i][c];
        }
        __syncthreads();
        if (I0 > 0) {
            double *S = q.Sw;  // nb x I0
            block_gemm(nb, I0, I0, 1.0, Dw + (int64_t)(k + I0) * m + k, m, 1, q.L, ne, 1, 0.0, S, I0, smem);
            block_gemm(nb, I0, nb, -1.0, q.L + (int64_t)I0 * ne + I0, ne, 1, S, I0, 1, 0.0, q.L + (int64_t)I0 * ne, ne,
                       smem);
        }
    }
    __syncthreads();
    return true;
}

// Phase 4: W = A_ce L^{-T}, S = A_cc - W W^T (jobs 0, 1), and S passed up
// symmetrized.
__device__ __forceinline__ GemmJob ulv_schur_job(const UlvDesc &q, int j) {
    const int m = q.m, k = q.k, ne = m - k;
    if (j == 0) return {k, ne, ne, 1.0, 0.0, q.Dw + k, m, 1, q.L, 1, ne, q.W, ne};  // W = A_ce L^{-T}
    return {k, k, ne, -1.0, 1.0, q.W, ne, 1, q.W, 1, ne, q.Dw, m};                   // A_cc -= W W^T
}

__device__ void ulv_schur_out(const UlvDesc &q) {
    const int m = q.m, k = q.k;
    for (int t = threadIdx.x; t < k * k; t += BG_T) {
        int i = t / k, c = t % k;
        q.S_out[t] = 0.5 * (q.Dw[(int64_t)i * m + c] + q.Dw[(int64_t)c * m + i]);
    }
}

// The whole elimination of a level's nodes, one workgroup per node.
__global__ __launch_bounds__(BG_T) void k_ulv_factor(const UlvDesc *dsc, int32_t *flag, unsigned long long *clamped,
                                                     unsigned long long *worst) {
    __shared__ double smem[2 * 16 * 65];
    __shared__ double red[BG_T / 64];
    __shared__ double blk[64][33];
    const UlvDesc q = dsc[blockIdx.x];
    ulv_assemble_qr(q, smem, red, blk);
    ulv_transform(q, smem);
    if (!ulv_chol_inv(q, flag, clamped, worst, red, smem, blk)) return;
    if (q.root) return;
    for (int j = 0; j < 2; ++j) {
        const GemmJob J = ulv_schur_job(q, j);
        block_gemm(J.M, J.N, J.K, J.alpha, J.A, J.as0, J.as1, J.B, J.bs0, J.bs1, J.beta, J.C, J.ldc, smem);
    }
    ulv_schur_out(q);
}

// The same phases for levels of few, large nodes: phases 1 and 3 one
// workgroup per node, the products of phases 2 and 4 one workgroup per tile
// of every node of the level (k_tile_gemms), the output last.
__global__ __launch_bounds__(BG_T) void k_ulv_phase1(const UlvDesc *dsc) {
    __shared__ double smem[2 * 16 * 65];
    __shared__ double red[BG_T / 64];
    __shared__ double blk[64][33];
    const UlvDesc q = dsc[blockIdx.x];
    ulv_assemble_qr(q, smem, red, blk);
}

__global__ __launch_bounds__(BG_T) void k_ulv_phase3(const UlvDesc *dsc, int32_t *flag, unsigned long long *clamped,
                                                     unsigned long long *worst) {
    __shared__ double smem[2 * 16 * 65];
    __shared__ double red[BG_T / 64];
    __shared__ double blk[64][33];
    const UlvDesc q = dsc[blockIdx.x];
    ulv_chol_inv(q, flag, clamped, worst, red, smem, blk);
}

__global__ __launch_bounds__(BG_T) void k_ulv_schur_out(const UlvDesc *dsc) {
    const UlvDesc q = dsc[blockIdx.x];
    if (!q.root) ulv_schur_out(q);
}

// One 64 x 64 tile of one job per workgroup; jobs are filled in on the device
// from the level's descriptors (step: 0-5 the transform, 6-7 the Schur
// complement).
__global__ __launch_bounds__(BG_T) void k_tile_gemms(const UlvDesc *dsc, const GemmTile *tiles, int step) {
    __shared__ double smem[2 * 16 * 65];
    const GemmTile t = tiles[blockIdx.x];
    const UlvDesc q = dsc[t.job];
    const GemmJob J = step < 6 ? ulv_transform_job(q, step) : ulv_schur_job(q, step - 6);
    tile_gemm(J.M, J.N, J.K, t.i0, t.j0, J.alpha, J.A, J.as0, J.as1, J.B, J.bs0, J.bs1, J.beta, J.C, J.ldc, smem);
}

struct SolveDesc {
    int32_t m, k, leaf, root;
    int64_t b;
    const double *V, *T, *Li, *W;  // Q = I - V T V^T; Li = L^{-1}
    double *bw;              // m x nrhs: rhs on the way up, solution on the way down
    double *z;               // (m - k) x nrhs
    double *c_out;           // k x nrhs (passed up)
    double *y1, *y2;         // k x nrhs scratch of the WY products
    const double *c_l, *c_r; // children's reduced rhs
    int32_t kl, kr;
    const double *x_par;     // parent's solution rows for this node (k x nrhs), set for the backward sweep
};

// out(o) = sum over l in [lo(o), hi(o)) of term(o, l), for o < nout: each
// output is summed by a team of ts consecutive lanes (ts the largest power of
// two <= blockDim / nout, at most 64, so a team stays inside a wave), which
// shortens the dependent chain of the big nodes near the root.
template <class Range, class Term, class Store>
__device__ __forceinline__ void team_sum(int nout, Range range, Term term, Store store) {
    const int nt = blockDim.x, tid = threadIdx.x;
    int ts = 1;
    while (ts < 64 && 2 * ts * nout <= nt) ts *= 2;
    const int team = tid / ts, li = tid % ts, nteams = nt / ts;
    for (int o0 = 0; o0 < nout; o0 += nteams) {  // uniform trip count: every lane takes part in the shuffles
        const int o = o0 + team;
        double acc = 0.0;
        if (o < nout) {
            int lo, hi;
            range(o, lo, hi);
            for (int l = lo + li; l < hi; l += ts) acc += term(o, l);
        }
        for (int off = ts / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (o < nout && li == 0) store(o, acc);
    }
}

// bw (m x nrhs) <- (I - V op(T) V^T) bw with op(T) = T^T (Q^T, `trans`) or T
// (Q).  V (m x k) holds unit lower-trapezoidal reflectors (zeros above the
// diagonal, ones on it).
__device__ void apply_wy(const double *__restrict__ V, const double *__restrict__ T, int m, int k, double *bw,
                         int nrhs, double *y1, double *y2, bool trans) {
    // y1 = V^T bw
    team_sum(k * nrhs, [&](int o, int &lo, int &hi) { lo = o / nrhs; hi = m; },
             [&](int o, int i) { return V[(int64_t)i * k + o / nrhs] * bw[(int64_t)i * nrhs + o % nrhs]; },
             [&](int o, double v) { y1[o] = v; });
    __syncthreads();
    // y2 = op(T) y1, T upper triangular
    if (trans)
        team_sum(k * nrhs, [&](int o, int &lo, int &hi) { lo = 0; hi = o / nrhs + 1; },
                 [&](int o, int l) { return T[(int64_t)l * k + o / nrhs] * y1[(int64_t)l * nrhs + o % nrhs]; },
                 [&](int o, double v) { y2[o] = v; });
    else
        team_sum(k * nrhs, [&](int o, int &lo, int &hi) { lo = o / nrhs; hi = k; },
                 [&](int o, int l) { return T[(int64_t)(o / nrhs) * k + l] * y1[(int64_t)l * nrhs + o % nrhs]; },
                 [&](int o, double v) { y2[o] = v; });
    __syncthreads();
    // bw -= V y2
    team_sum(m * nrhs, [&](int o, int &lo, int &hi) { lo = 0; hi = min(o / nrhs + 1, k); },
             [&](int o, int j) { return V[(int64_t)(o / nrhs) * k + j] * y2[(int64_t)j * nrhs + o % nrhs]; },
             [&](int o, double v) { bw[o] -= v; });
    __syncthreads();
}

__global__ __launch_bounds__(1024) void k_ulv_fwd(const SolveDesc *dsc, const double *__restrict__ Bin, int nrhs,
                                                  double *__restrict__ Xout) {
    const SolveDesc q = dsc[blockIdx.x];
    const int m = q.m, k = q.k, ne = m - k, tid = threadIdx.x, nt = blockDim.x;
    if (q.leaf) {
        for (int64_t t = tid; t < (int64_t)m * nrhs; t += nt) q.bw[t] = Bin[q.b * nrhs + t];
    } else {
        for (int64_t t = tid; t < (int64_t)q.kl * nrhs; t += nt) q.bw[t] = q.c_l[t];
        for (int64_t t = tid; t < (int64_t)q.kr * nrhs; t += nt) q.bw[(int64_t)q.kl * nrhs + t] = q.c_r[t];
    }
    __syncthreads();
    if (k > 0) apply_wy(q.V, q.T, m, k, q.bw, nrhs, q.y1, q.y2, true);
    // z = L^{-1} b_e
    const double *bwe = q.bw + (int64_t)k * nrhs;
    team_sum(ne * nrhs, [&](int o, int &lo, int &hi) { lo = 0; hi = o / nrhs + 1; },
             [&](int o, int l) { return q.Li[(int64_t)(o / nrhs) * ne + l] * bwe[(int64_t)l * nrhs + o % nrhs]; },
             [&](int o, double v) { q.z[o] = v; });
    __syncthreads();
    if (q.root) {
        // whole solve at the root (k = 0): x = L^{-T} z
        team_sum(m * nrhs, [&](int o, int &lo, int &hi) { lo = o / nrhs; hi = m; },
                 [&](int o, int l) { return q.Li[(int64_t)l * m + o / nrhs] * q.z[(int64_t)l * nrhs + o % nrhs]; },
                 [&](int o, double v) {
                     q.bw[o] = v;
                     if (q.leaf) Xout[q.b * nrhs + o] = v;  // a one-node tree has no backward sweep
                 });
        return;
    }
    // c = b_c - W z
    team_sum(k * nrhs, [&](int o, int &lo, int &hi) { lo = 0; hi = ne; },
             [&](int o, int l) { return q.W[(int64_t)(o / nrhs) * ne + l] * q.z[(int64_t)l * nrhs + o % nrhs]; },
             [&](int o, double v) { q.c_out[o] = q.bw[o] - v; });
}

__global__ __launch_bounds__(1024) void k_ulv_bwd(const SolveDesc *dsc, double *__restrict__ Xout, int nrhs) {
    const SolveDesc q = dsc[blockIdx.x];
    const int m = q.m, k = q.k, ne = m - k, tid = threadIdx.x, nt = blockDim.x;
    // x_c from the parent; z <- z - W^T x_c
    for (int64_t t = tid; t < (int64_t)k * nrhs; t += nt) q.bw[t] = q.x_par[t];
    team_sum(ne * nrhs, [&](int o, int &lo, int &hi) { lo = 0; hi = k; },
             [&](int o, int i) { return q.W[(int64_t)i * ne + o / nrhs] * q.x_par[(int64_t)i * nrhs + o % nrhs]; },
             [&](int o, double v) { q.z[o] -= v; });
    __syncthreads();
    // x_e = L^{-T} z
    double *bwe = q.bw + (int64_t)k * nrhs;
    team_sum(ne * nrhs, [&](int o, int &lo, int &hi) { lo = o / nrhs; hi = ne; },
             [&](int o, int l) { return q.Li[(int64_t)l * ne + o / nrhs] * q.z[(int64_t)l * nrhs + o % nrhs]; },
             [&](int o, double v) { bwe[o] = v; });
    __syncthreads();
    if (k > 0) apply_wy(q.V, q.T, m, k, q.bw, nrhs, q.y1, q.y2, false);
    if (q.leaf)
        for (int64_t t = tid; t < (int64_t)m * nrhs; t += nt) Xout[q.b * nrhs + t] = q.bw[t];
}

}  // namespace

int64_t ulv_factor(const hss_s *H, const std::vector<double> &lam, const std::vector<double> &floor, hipStream_t s,
                   hss_ulv_s *F, std::vector<double> *deficit, bool stop_at_floor, std::vector<uint8_t> *active) {
    const int nn = (int)H->node.size();
    const int np = (int)H->hprob.size();
    KRR_REQUIRE((int)lam.size() == np && (int)floor.size() == np, "ULV: one lambda and floor per problem");
    KRR_REQUIRE(!active || (int)active->size() == np, "ULV: one activity flag per problem");
    const bool reuse = !F->node.empty();  // a later pass over some problems of the same factor
    KRR_REQUIRE(!reuse || (F->node.size() == H->node.size() && F->n == H->n), "ULV: factor of another matrix");
    F->n = H->n;
    F->lambda = lam[0];
    if (!reuse) F->lamprob = lam;
    for (int p = 0; p < np; ++p)
        if (!active || (*active)[p]) F->lamprob[p] = lam[p];
    F->plans.clear();  // solve plans describe the previous values
    if (!reuse) {
        F->node = H->node;
        F->levels = H->levels;
        F->offV.assign(nn, 0);
        F->offT.assign(nn, 0);
        F->offL.assign(nn, 0);
        F->offW.assign(nn, 0);
        F->offY.assign(nn, 0);
    }
    // per-node sizes: m (rows of the reduced block) and k
    std::vector<int> m(nn), k(nn);
    for (int i = 0; i < nn; ++i) {
        const HNode &q = H->node[i];
        k[i] = (q.parent < 0) ? 0 : q.k;
        m[i] = (q.left < 0) ? (int)(q.e - q.b) : k[q.left] + k[q.right];
        F->node[i].m = m[i];
        F->node[i].k = k[i];
    }
    if (!reuse) {
        int64_t nv = 0, nt = 0, nl = 0, nw = 0, ny = 0;
        for (int i = 0; i < nn; ++i) {
            int ne = m[i] - k[i];
            F->offV[i] = nv; nv += (int64_t)m[i] * k[i];
            F->offT[i] = nt; nt += k[i];
            F->offL[i] = nl; nl += (int64_t)ne * ne;
            F->offW[i] = nw; nw += (int64_t)k[i] * ne;
            F->offY[i] = ny; ny += (int64_t)k[i] * k[i];
    }
    F->V.alloc(8 * std::max<int64_t>(nv, 1));
    F->T.alloc(8 * std::max<int64_t>(nt, 1));
    F->L.alloc(8 * std::max<int64_t>(nl, 1));
    F->W.alloc(8 * std::max<int64_t>(nw, 1));
    F->Y.alloc(8 * std::max<int64_t>(ny, 1));
    F->R.alloc(8 * std::max<int64_t>(ny, 1));
    F->nV = nv; F->nT = nt; F->nL = nl; F->nW = nw; F->nY = ny;
    F->qr_ok.assign(nn, 0);
    }
    std::vector<uint8_t> act(np, 1);
    if (active) act = *active;
    // S of every non-root node lives until the parent is done (Rh lives in
    // the factor, at offY)
    std::vector<int64_t> offS(nn, 0);
    int64_t ns = 0;
    for (int i = 0; i < nn; ++i) {
        offS[i] = ns;
        ns += (int64_t)k[i] * k[i];
    }
    DBuf Sb = dalloc<double>(std::max<int64_t>(ns, 1));
    // counters: raised pivots per problem, then each problem's largest deficit
    DBuf flag = dalloc<int32_t>(1), nclamp = dalloc<unsigned long long>(2 * np);
    KRR_HIP(hipMemsetAsync(flag.get(), 0, sizeof(int32_t), s));
    KRR_HIP(hipMemsetAsync(nclamp.get(), 0, 2 * np * sizeof(unsigned long long), s));
    std::vector<uint8_t> raised(np, 0);
    for (const auto &lv_all : H->levels) {
        std::vector<int> lv;  // this level's nodes of the problems still being factored
        for (int id : lv_all)
            if (act[H->nprob[id]]) lv.push_back(id);
        if (lv.empty()) continue;
        const int cnt = (int)lv.size();
        int64_t dsz = 0, usz = 0, tsz = 0, ysz = 0, ssz = 0;
        for (int id : lv) {
            dsz += (int64_t)m[id] * m[id];
            usz += (int64_t)m[id] * k[id];
            const HNode &q = H->node[id];
            if (q.left >= 0) tsz += (int64_t)k[q.left] * k[q.right];
            ysz += (int64_t)std::max(m[id], k[id]) * k[id];
            ssz += (int64_t)CH_NB * m[id];
        }
        DBuf Dw = dalloc<double>(std::max<int64_t>(dsz, 1)), Uw = dalloc<double>(std::max<int64_t>(usz, 1)),
             Tm = dalloc<double>(std::max<int64_t>(tsz, 1)), Yb = dalloc<double>(std::max<int64_t>(ysz, 1)),
             Zb = dalloc<double>(std::max<int64_t>(ysz, 1)), Sb2 = dalloc<double>(std::max<int64_t>(ssz, 1));
        std::vector<UlvDesc> dsc(cnt);
        int64_t od = 0, ou = 0, ot = 0, oy = 0, os = 0;
        for (int a = 0; a < cnt; ++a) {
            const int id = lv[a];
            const HNode &q = H->node[id];
            UlvDesc &u = dsc[a];
            std::memset(&u, 0, sizeof u);
            u.m = m[id];
            u.k = k[id];
            u.leaf = q.left < 0;
            u.root = q.parent < 0;
            u.prob = H->nprob[id];
            u.lambda = lam[H->nprob[id]];
            u.pivot_floor = floor[H->nprob[id]];
            if (u.leaf) {
                u.D = H->D.as<double>() + q.offD;
            } else {
                u.kl = k[q.left];
                u.kr = k[q.right];
                u.B = H->B.as<double>() + q.offB;
                u.S_l = Sb.as<double>() + offS[q.left];
                u.S_r = Sb.as<double>() + offS[q.right];
                u.Rh_l = F->R.as<double>() + F->offY[q.left];
                u.Rh_r = F->R.as<double>() + F->offY[q.right];
                u.Tmp = Tm.as<double>() + ot;
                ot += (int64_t)u.kl * u.kr;
            }
            if (!u.root) u.U = H->U.as<double>() + q.offU;
            u.Dw = Dw.as<double>() + od;
            u.Uw = Uw.as<double>() + ou;
            u.Yw = Yb.as<double>() + oy;
            u.Zw = Zb.as<double>() + oy;
            u.Sw = Sb2.as<double>() + os;
            os += (int64_t)CH_NB * u.m;
            u.Tw = F->Y.as<double>() + F->offY[id];
            od += (int64_t)u.m * u.m;
            ou += (int64_t)u.m * u.k;
            oy += (int64_t)std::max(u.m, u.k) * u.k;
            u.V = F->V.as<double>() + F->offV[id];
            u.tau = F->T.as<double>() + F->offT[id];
            u.L = F->L.as<double>() + F->offL[id];
            u.W = F->W.as<double>() + F->offW[id];
            u.S_out = Sb.as<double>() + offS[id];
            u.Rh_out = F->R.as<double>() + F->offY[id];
            u.qr_done = F->qr_ok[id];
        }
        DBuf dd = upload(dsc, s);
        if (cnt >= kPhasedNodes) {
            k_ulv_factor<<<cnt, BG_T, 0, s>>>(dd.as<UlvDesc>(), flag.as<int32_t>(), nclamp.as<unsigned long long>(),
                                              nclamp.as<unsigned long long>() + np);
            check_launch("k_ulv_factor");
        } else {
            // few, large nodes (near the root): the products of each phase
            // spread over one workgroup per 64 x 64 tile of every node
            std::vector<GemmTile> tiles;
            std::vector<int64_t> step_off(9, 0);
            for (int step = 0; step < 8; ++step) {
                step_off[step] = (int64_t)tiles.size();
                for (int a = 0; a < cnt; ++a) {
                    const UlvDesc &u = dsc[a];
                    const int ne = u.m - u.k;
                    if (u.k <= 0 || (step >= 6 && u.root)) continue;
                    int M, N;
                    if (step < 6) {
                        M = (step <= 1) ? u.k : u.m;
                        N = (step == 3 || step == 4) ? u.k : u.m;
                    } else {
                        M = u.k;
                        N = step == 6 ? ne : u.k;
                    }
                    for (int i0 = 0; i0 < M; i0 += 64)
                        for (int j0 = 0; j0 < N; j0 += 64) tiles.push_back({a, i0, j0});
                }
            }
            step_off[8] = (int64_t)tiles.size();
            DBuf dt = upload(tiles, s);
            auto gemms = [&](int step) {
                const int64_t nt = step_off[step + 1] - step_off[step];
                if (nt == 0) return;
                k_tile_gemms<<<(unsigned)nt, BG_T, 0, s>>>(dd.as<UlvDesc>(), dt.as<GemmTile>() + step_off[step], step);
                check_launch("k_tile_gemms");
            };
            k_ulv_phase1<<<cnt, BG_T, 0, s>>>(dd.as<UlvDesc>());
            check_launch("k_ulv_phase1");
            for (int step = 0; step < 6; ++step) gemms(step);
            k_ulv_phase3<<<cnt, BG_T, 0, s>>>(dd.as<UlvDesc>(), flag.as<int32_t>(), nclamp.as<unsigned long long>(),
                                              nclamp.as<unsigned long long>() + np);
            check_launch("k_ulv_phase3");
            gemms(6);
            gemms(7);
            k_ulv_schur_out<<<cnt, BG_T, 0, s>>>(dd.as<UlvDesc>());
            check_launch("k_ulv_schur_out");
            sync(s);  // `tiles` is released at the end of this scope
        }
        sync(s);
        for (int id : lv) F->qr_ok[id] = 1;  // the level's QR ran whatever its pivots did
        if (stop_at_floor) {
            // a problem with a pivot below its floor stops here (its factor
            // is left incomplete); the others go on
            std::vector<unsigned long long> c(np);
            d2h(c.data(), nclamp.as<unsigned long long>(), np, s);
            sync(s);
            for (int p = 0; p < np; ++p)
                if (act[p] && c[p]) {
                    act[p] = 0;
                    raised[p] = 1;
                }
        }
    }
    int32_t bad = 0;
    std::vector<unsigned long long> cl(2 * np);
    d2h(&bad, flag.as<int32_t>(), 1, s);
    d2h(cl.data(), nclamp.as<unsigned long long>(), 2 * np, s);
    sync(s);
    if (deficit) {
        deficit->assign(np, 0.0);
        for (int p = 0; p < np; ++p)
            (*deficit)[p] = cl[np + p] ? __builtin_bit_cast(double, (uint64_t)cl[np + p]) : 0.0;
    }
    if (bad) fail(KRR_E_NUMERIC, "ULV: non-positive pivot in a Cholesky factor (K_hss + lambda I not SPD)");
    if (active && stop_at_floor) *active = raised;
    int64_t tot = 0;
    for (int p = 0; p < np; ++p) tot += (int64_t)cl[p];
    return tot;
}

// A solve plan for one factor and one number of right-hand sides: the sweep
// workspace and the per-level descriptor arrays live on the device for the
// factor's lifetime, so that a solve issues only its kernel launches (no
// allocation, upload or synchronization); with graphs on, those launches are
// captured once into a HIP graph and replayed (the right-hand side is copied
// into the plan's input block and the solution out of its output block).
struct UlvSolvePlan {
    int nrhs = 0;
    int64_t n = 0;
    DBuf bw, zb, cb, y1, y2, in, out;
    std::vector<DBuf> desc;             // forward levels, then backward levels
    std::vector<int> cnt, fwd;          // per launch: blocks, 1 = forward
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~UlvSolvePlan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

namespace {

std::shared_ptr<UlvSolvePlan> make_plan(const hss_ulv_s *F, int nrhs, hipStream_t s) {
    auto P = std::make_shared<UlvSolvePlan>();
    P->nrhs = nrhs;
    P->n = F->n;
    const int nn = (int)F->node.size();
    std::vector<int64_t> ob(nn), oz(nn), oc(nn);
    int64_t nb = 0, nz = 0, nc = 0;
    for (int i = 0; i < nn; ++i) {
        const HNode &q = F->node[i];
        ob[i] = nb; nb += (int64_t)q.m * nrhs;
        oz[i] = nz; nz += (int64_t)(q.m - q.k) * nrhs;
        oc[i] = nc; nc += (int64_t)q.k * nrhs;
    }
    P->bw = dalloc<double>(std::max<int64_t>(nb, 1));
    P->zb = dalloc<double>(std::max<int64_t>(nz, 1));
    P->cb = dalloc<double>(std::max<int64_t>(nc, 1));
    P->y1 = dalloc<double>(std::max<int64_t>(nc, 1));
    P->y2 = dalloc<double>(std::max<int64_t>(nc, 1));
    double *bw = P->bw.as<double>(), *zb = P->zb.as<double>(), *cb = P->cb.as<double>();
    double *y1 = P->y1.as<double>(), *y2 = P->y2.as<double>();
    auto make = [&](int id) {
        const HNode &q = F->node[id];
        SolveDesc d;
        std::memset(&d, 0, sizeof d);
        d.m = q.m;
        d.k = q.k;
        d.leaf = q.left < 0;
        d.root = q.parent < 0;
        d.b = q.b;
        d.V = F->V.as<double>() + F->offV[id];
        d.T = F->Y.as<double>() + F->offY[id];
        d.Li = F->L.as<double>() + F->offL[id];
        d.W = F->W.as<double>() + F->offW[id];
        d.bw = bw + ob[id];
        d.z = zb + oz[id];
        d.c_out = cb + oc[id];
        d.y1 = y1 + oc[id];
        d.y2 = y2 + oc[id];
        if (!d.leaf) {
            d.kl = F->node[q.left].k;
            d.kr = F->node[q.right].k;
            d.c_l = cb + oc[q.left];
            d.c_r = cb + oc[q.right];
        }
        if (!d.root) {
            const HNode &p = F->node[q.parent];
            int64_t off = (p.left == id) ? 0 : (int64_t)F->node[p.left].k;
            d.x_par = bw + ob[q.parent] + off * nrhs;
        }
        return d;
    };
    auto add = [&](const std::vector<SolveDesc> &v, int forward) {
        if (v.empty()) return;
        P->desc.push_back(upload(v, s));
        P->cnt.push_back((int)v.size());
        P->fwd.push_back(forward);
        sync(s);  // `v` is a temporary of the caller
    };
    for (const auto &lv : F->levels) {
        std::vector<SolveDesc> v;
        for (int id : lv) v.push_back(make(id));
        add(v, 1);
    }
    for (int h = (int)F->levels.size() - 1; h >= 0; --h) {
        std::vector<SolveDesc> v;
        for (int id : F->levels[h])
            if (F->node[id].parent >= 0) v.push_back(make(id));
        add(v, 0);
    }
    return P;
}

void enqueue_solve(const UlvSolvePlan &P, const double *Bin, double *Xout, hipStream_t s) {
    for (size_t l = 0; l < P.desc.size(); ++l) {
        // levels of few nodes (near the root, big nodes) get 1024 threads per node
        const int nt = P.cnt[l] >= 1024 ? BG_T : 1024;
        if (P.fwd[l]) {
            k_ulv_fwd<<<(unsigned)P.cnt[l], nt, 0, s>>>(P.desc[l].as<SolveDesc>(), Bin, P.nrhs, Xout);
            check_launch("k_ulv_fwd");
        } else {
            k_ulv_bwd<<<(unsigned)P.cnt[l], nt, 0, s>>>(P.desc[l].as<SolveDesc>(), Xout, P.nrhs);
            check_launch("k_ulv_bwd");
        }
    }
}

void capture(UlvSolvePlan &P) {
    P.in = dalloc<double>((size_t)P.n * P.nrhs);
    P.out = dalloc<double>((size_t)P.n * P.nrhs);
    hipStream_t cs = nullptr;
    KRR_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    try {
        KRR_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_solve(P, P.in.as<double>(), P.out.as<double>(), cs);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(cs, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        KRR_HIP(hipStreamEndCapture(cs, &P.graph));
        KRR_HIP(hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0));
    } catch (...) {
        (void)hipStreamDestroy(cs);
        throw;
    }
    KRR_HIP(hipStreamDestroy(cs));
}

}  // namespace

void ulv_solve(const hss_ulv_s *F, const double *Bin, int nrhs, double *Xout, hipStream_t s) {
    auto *Fm = const_cast<hss_ulv_s *>(F);  // the plan cache is not part of the factor's value
    std::shared_ptr<UlvSolvePlan> P;
    for (auto &q : Fm->plans)
        if (q->nrhs == nrhs) P = q;
    if (!P) {
        P = make_plan(F, nrhs, s);
        Fm->plans.push_back(P);
    }
    if (!F->use_graph) {
        enqueue_solve(*P, Bin, Xout, s);
        return;
    }
    if (!P->exec) capture(*P);
    const size_t bytes = sizeof(double) * (size_t)F->n * nrhs;
    KRR_HIP(hipMemcpyAsync(P->in.get(), Bin, bytes, hipMemcpyDeviceToDevice, s));
    KRR_HIP(hipGraphLaunch(P->exec, s));
    KRR_HIP(hipMemcpyAsync(Xout, P->out.get(), bytes, hipMemcpyDeviceToDevice, s));
}

}  // namespace krr
