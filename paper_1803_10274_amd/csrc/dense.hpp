// Workgroup-level FP64 dense kernels for the per-node work of the HSS
// compression and ULV factorization.  One workgroup of 256 threads owns one
// tree node; operands live in global memory (they are small and stay in L2)
// and are staged through LDS in 64 x 16 panels.
#pragma once

#include "common.hpp"

namespace krr {

constexpr int BG_T = 256;  // threads per node workgroup

// One 64 x 64 tile (rows i0.., columns j0..) of
// C(i, j) = beta * C(i, j) + alpha * sum_k A(i, k) B(k, j)
// with A(i, k) = A[i * as0 + k * as1], B(k, j) = B[k * bs0 + j * bs1],
// C row-major with leading dimension ldc.  beta == 0 never reads C.
// smem: at least 2 * 16 * 65 doubles.  All 256 threads must call it.
template <class TA, class TB>
__device__ __forceinline__ void tile_gemm(int M, int N, int K, int i0, int j0, double alpha, const TA *__restrict__ A, int64_t as0,
                          int64_t as1, const TB *__restrict__ B, int64_t bs0, int64_t bs1, double beta,
                          double *__restrict__ C, int64_t ldc, double *smem) {
    double(*As)[65] = reinterpret_cast<double(*)[65]>(smem);
    double(*Bs)[65] = reinterpret_cast<double(*)[65]>(smem + 16 * 65);
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int k0 = 0; k0 < K; k0 += 16) {
        for (int t = tid; t < 16 * 64; t += BG_T) {
            int kk = t >> 6, ii = t & 63;
            int gi = i0 + ii, gk = k0 + kk;
            As[kk][ii] = (gi < M && gk < K) ? (double)A[gi * as0 + gk * as1] : 0.0;
            int gj = j0 + ii;
            Bs[kk][ii] = (gj < N && gk < K) ? (double)B[gk * bs0 + gj * bs1] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = As[kk][ty + 16 * a];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = Bs[kk][tx + 16 * b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        int gi = i0 + ty + 16 * a;
        if (gi >= M) continue;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            int gj = j0 + tx + 16 * b;
            if (gj >= N) continue;
            double *c = C + (int64_t)gi * ldc + gj;
            *c = (beta == 0.0) ? alpha * acc[a][b] : beta * (*c) + alpha * acc[a][b];
        }
    }
}

// The whole product by one workgroup, tile after tile.
template <class TA, class TB>
__device__ __forceinline__ void block_gemm(int M, int N, int K, double alpha, const TA *__restrict__ A, int64_t as0,
                           int64_t as1, const TB *__restrict__ B, int64_t bs0, int64_t bs1, double beta,
                           double *__restrict__ C, int64_t ldc, double *smem) {
    for (int i0 = 0; i0 < M; i0 += 64)
        for (int j0 = 0; j0 < N; j0 += 64)
            tile_gemm(M, N, K, i0, j0, alpha, A, as0, as1, B, bs0, bs1, beta, C, ldc, smem);
    __syncthreads();
}

// A product of a batch of independent ones, spread over workgroups: one
// 64 x 64 tile per workgroup (the levels of the ULV factorization with few,
// large nodes).
struct GemmJob {
    int M, N, K;
    double alpha, beta;
    const double *A;
    int64_t as0, as1;
    const double *B;
    int64_t bs0, bs1;
    double *C;
    int64_t ldc;
};
struct GemmTile {
    int job, i0, j0;
};

// Block-wide reductions (256 threads); red: at least 8 doubles / ints of smem.
__device__ inline double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < BG_T / 64; ++i) t += red[i];
    __syncthreads();
    return t;
}

// Arg-max of v over threads (ties to the smaller index); idx = -1 entries ignored.
__device__ inline void block_argmax(double v, int idx, double *redv, int *redi, double &best, int &bidx) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        double ov = __shfl_xor(v, o, 64);
        int oi = __shfl_xor(idx, o, 64);
        bool take = (oi >= 0) && (idx < 0 || ov > v || (ov == v && oi < idx));
        if (take) {
            v = ov;
            idx = oi;
        }
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        redv[w] = v;
        redi[w] = idx;
    }
    __syncthreads();
    best = -1.0;
    bidx = -1;
    for (int i = 0; i < BG_T / 64; ++i) {
        if (redi[i] < 0) continue;
        if (bidx < 0 || redv[i] > best || (redv[i] == best && redi[i] < bidx)) {
            best = redv[i];
            bidx = redi[i];
        }
    }
    __syncthreads();
}

}  // namespace krr
