// Sampling product dispatch: S = K(X, X; h) R with each row's own leaf block
// removed (the off-diagonal sample of the randomized HSS construction,
// Section 3.1).  FP64 samples use the tiled VALU kernel; the FP32 and the
// FP16 / BF16 split modes use the matrix-core kernel when it applies.
#include "internal.hpp"

namespace krr {

void sample_valu(const void *X, int64_t n, int d, int xprec, double h, const float *R, int r, const int32_t *lb,
                 const int32_t *le, void *S, int prec, hipStream_t s);

bool sample_mfma_supported(int d, int prec);
void sample_mfma(const void *X, int64_t n, int d, int xprec, double h, const float *R, int r, const int32_t *lb,
                 const int32_t *le, float *S, int prec, int split, hipStream_t s);

void sample_product(const void *X, int64_t n, int d, int xprec, double h, const float *R, int r, const int32_t *lb,
                    const int32_t *le, void *S, int prec, int split, hipStream_t s) {
    if (n == 0 || r == 0) return;
    if (sample_mfma_supported(d, prec))
        sample_mfma(X, n, d, xprec, h, R, r, lb, le, static_cast<float *>(S), prec, split, s);
    else
        sample_valu(X, n, d, xprec, h, R, r, lb, le, S, prec == KRR_F64 ? KRR_F64 : KRR_F32, s);
}

}  // namespace krr
