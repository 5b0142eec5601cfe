// krr_predict_noalloc: prediction scores and labels without any device
// allocation, for callers that cannot allocate (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc).  The split-K partial sums
// and the column data of the kernel product live in one file-scope device
// array, `scratch`, of KRR_NOALLOC_SCRATCH_BYTES per device; each device that
// calls this entry point holds it until the process ends.
#include <mutex>

#include "internal.hpp"

namespace krr {
namespace {

static __device__ __align__(256) unsigned char scratch[KRR_NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` per device.  In host code the array's name is
// only a stand-in for the device symbol, so kernels get this address instead.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

void *scratch_address() {
    int dev = 0;
    KRR_HIP(hipGetDevice(&dev));
    KRR_REQUIRE(dev >= 0 && dev < kMaxDevices, "krr_predict_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[dev]) {
        void *p = nullptr;
        KRR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        KRR_REQUIRE(p != nullptr, "krr_predict_noalloc: no device address for the scratch array");
        g_addr[dev] = p;
    }
    return g_addr[dev];
}

}  // namespace

void predict_noalloc(const void *Xt, int64_t m, const void *Xp, int64_t n, int d, int xprec, double h,
                     const double *alpha, int nrhs, double *scores, int32_t *labels, int prec, hipStream_t s) {
    const size_t need = kernel_matvec_ws_bytes(m, n, d, nrhs, prec);
    KRR_REQUIRE(need <= (size_t)KRR_NOALLOC_SCRATCH_BYTES,
                "krr_predict_noalloc: this size needs %zu bytes of scratch, the limit is %zu (use krr_predict)",
                need, (size_t)KRR_NOALLOC_SCRATCH_BYTES);
    void *ws = scratch_address();
    kernel_matvec_ws(Xt, m, Xp, n, d, xprec, h, alpha, nrhs, scores, prec, ws, (size_t)KRR_NOALLOC_SCRATCH_BYTES, s);
    if (labels) predict_labels(scores, m, nrhs, labels, s);
}

}  // namespace krr
