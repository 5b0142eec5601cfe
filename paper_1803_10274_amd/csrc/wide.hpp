// Prepared coordinates of wide points (d > 64) for the matrix-core exponent
// GEMMs: points are centred on one anchor (the mean point; the Gaussian kernel
// is translation invariant) and augmented so that t = x~_i . y~_j is the
// log2-scaled exponent -c |x_i - y_j|^2:
//   rows    x~ = (2 c x', -c |x'|^2 + off, 1, 0 ..)
//   columns y~ = (x', 1, -c |x'|^2, 0 ..)
// in rows of KP floats (KP a multiple of the GEMM's K chunk); c per problem
// for a batch (pbeg / cprob), off = 14 for the 2^14-scaled FP16 entries.
// k_wide_aug64 is the FP64 form (natural-log units, no offset).
#pragma once

#include "internal.hpp"

namespace krr {
namespace {

template <class T>
__global__ void k_col_mean(const T *__restrict__ X, int64_t n, int d, double *__restrict__ mean) {
    __shared__ double red[4];
    const int k = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += (double)X[i * d + k];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) mean[k] = ((red[0] + red[1]) + (red[2] + red[3])) / (double)n;
}

// side 0: the row form into A; side 1: the column form into A.  One
// workgroup of 256 threads per point.
__global__ void k_wide_aug(const float *__restrict__ X, int64_t n, int d, int KP, const double *__restrict__ mean,
                           double c2, const int64_t *__restrict__ pbeg, const double *__restrict__ cprob, int np,
                           float off, int side, float *__restrict__ A) {
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    double c = c2;
    if (pbeg) {
        int lo = 0, hi = np - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) / 2;
            if (pbeg[mid] <= i)
                lo = mid;
            else
                hi = mid - 1;
        }
        c = cprob[lo];
    }
    __shared__ double red[4];
    double nrm = 0.0;
    for (int k = threadIdx.x; k < KP; k += 256) {
        float v = k < d ? (float)((double)X[i * d + k] - mean[k]) : 0.0f;
        if (k < d) nrm += (double)v * (double)v;
        A[i * KP + k] = k < d ? (side == 0 ? (float)(2.0 * c * v) : v) : 0.0f;
    }
    nrm = wave_sum(nrm);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double q = (red[0] + red[1]) + (red[2] + red[3]);
        A[i * KP + d] = side == 0 ? (float)(-c * q) + off : 1.0f;
        A[i * KP + d + 1] = side == 0 ? 1.0f : (float)(-c * q);
    }
}

// FP64 form for the FP64-entry product: rows x~ = (2 c x', -c |x'|^2, 1, 0 ..),
// columns y~ = (x', 1, -c |y'|^2, 0 ..), c = 1 / (2 h^2) (natural-log units),
// coordinates centred on `mean` in FP64.
template <class T>
__global__ void k_wide_aug64(const T *__restrict__ X, int64_t n, int d, int KP, const double *__restrict__ mean,
                             double c2, const int64_t *__restrict__ pbeg, const double *__restrict__ cprob, int np,
                             int side, double *__restrict__ A) {
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    double c = c2;
    if (pbeg) {
        int lo = 0, hi = np - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) / 2;
            if (pbeg[mid] <= i)
                lo = mid;
            else
                hi = mid - 1;
        }
        c = cprob[lo];
    }
    __shared__ double red[4];
    double nrm = 0.0;
    for (int k = threadIdx.x; k < KP; k += 256) {
        const double v = k < d ? (double)X[i * d + k] - mean[k] : 0.0;
        nrm = fma(v, v, nrm);
        A[i * KP + k] = side == 0 ? 2.0 * c * v : v;
    }
    nrm = wave_sum(nrm);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double q = (red[0] + red[1]) + (red[2] + red[3]);
        A[i * KP + d] = side == 0 ? -c * q : 1.0;
        A[i * KP + d + 1] = side == 0 ? 1.0 : -c * q;
    }
}

}  // namespace
}  // namespace krr
