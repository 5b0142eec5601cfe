// Sampling product dispatch: S = K(X, X; h) R with each row's own leaf block
// removed (the off-diagonal sample of the randomized HSS construction,
// Section 3.1).  FP64 samples use the tiled VALU kernel; the FP32 and the
// FP16 / BF16 split modes use the matrix-core kernel when it applies.  A
// batch of independent problems is sampled in one launch: each workgroup
// takes rows of one problem and sums over that problem's columns only (the
// kernel matrix of a batch is block diagonal).
#include <algorithm>
#include <numeric>

#include "internal.hpp"

namespace krr {

void sample_valu(const void *X, int64_t n, int d, int xprec, double h, const float *R, int r, const int32_t *lb,
                 const int32_t *le, void *S, int prec, hipStream_t s, const Batch *batch);

bool sample_mfma_supported(int d, int prec);
void sample_mfma(const void *X, int64_t n, int d, int xprec, double h, const float *R, int r, const int32_t *lb,
                 const int32_t *le, float *S, int prec, int split, hipStream_t s, const Batch *batch);

std::vector<SampBlock> row_blocks(const Batch &b, int rows) {
    const int np = b.np();
    std::vector<int> ord(np);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) { return b.size(a) > b.size(c); });
    std::vector<SampBlock> out;
    for (int k : ord) {
        if (b.skipped(k)) continue;
        const double h = b.h[k];
        SampBlock sb{};
        sb.jlo = b.pbeg[k];
        sb.jhi = b.pbeg[k + 1];
        sb.inv = 1.0 / (2.0 * h * h);
        sb.c2 = 1.4426950408889634 / (2.0 * h * h);
        sb.cs = (float)sb.c2;
        for (int64_t i = sb.jlo; i < sb.jhi; i += rows) {
            sb.i0 = i;
            sb.iend = std::min<int64_t>(sb.jhi, i + rows);
            out.push_back(sb);
        }
    }
    return out;
}

void sample_product(const void *X, int64_t n, int d, int xprec, double h, const float *R, int r, const int32_t *lb,
                    const int32_t *le, void *S, int prec, int split, hipStream_t s, const Batch *batch) {
    if (n == 0 || r == 0) return;
    if (batch && batch->np() == 1) batch = nullptr;  // one problem: the plain launch
    if (sample_mfma_supported(d, prec))
        sample_mfma(X, n, d, xprec, h, R, r, lb, le, static_cast<float *>(S), prec, split, s, batch);
    else
        sample_valu(X, n, d, xprec, h, R, r, lb, le, S, prec == KRR_F64 ? KRR_F64 : KRR_F32, s, batch);
}

}  // namespace krr
