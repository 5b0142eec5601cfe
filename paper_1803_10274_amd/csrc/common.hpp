// Shared host/device plumbing of libkrr: error propagation, device buffers,
// launch checks and wave-level reductions for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "krr.h"

namespace krr {

// Internal failures travel as exceptions and are turned into status codes at
// the C boundary (capi.cpp); nothing throws across it.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(int code, const char *fmt, ...);

#define KRR_HIP(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            ::krr::fail(KRR_E_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                           \
    } while (0)

#define KRR_REQUIRE(cond, ...)                                                         \
    do {                                                                               \
        if (!(cond)) ::krr::fail(KRR_E_INVAL, __VA_ARGS__);                            \
    } while (0)

inline void check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(KRR_E_HIP, "launch of %s failed: %s", what, hipGetErrorString(e));
}

// A caller's stream-ordered device allocator (krr_set_allocator); all
// members NULL: hipMalloc / hipFree.
struct Allocator {
    void *(*alloc)(size_t, void *, void *) = nullptr;
    void (*dealloc)(void *, void *, void *) = nullptr;
    void *ctx = nullptr;
};
Allocator current_allocator();           // the one new buffers use
hipStream_t call_stream();                // the stream of the C-ABI call in progress (this thread)
void note_allocation(bool by_caller);     // allocation counters (krr_alloc_counts)

// Owning device allocation, move-only: from the registered allocator on the
// current call's stream (returned to that same allocator and stream), else
// hipMalloc / hipFree.
class DBuf {
  public:
    DBuf() = default;
    explicit DBuf(size_t bytes) { alloc(bytes); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p_(o.p_), n_(o.n_), own_(o.own_), s_(o.s_) {
        o.p_ = nullptr;
        o.n_ = 0;
    }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) {
            release();
            p_ = o.p_; n_ = o.n_; own_ = o.own_; s_ = o.s_;
            o.p_ = nullptr; o.n_ = 0;
        }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t bytes) {
        release();
        if (bytes == 0) return;
        const Allocator a = current_allocator();
        if (a.alloc) {
            s_ = call_stream();
            p_ = a.alloc(bytes, static_cast<void *>(s_), a.ctx);
            if (!p_) fail(KRR_E_NOMEM, "the registered allocator returned NULL for %zu bytes", bytes);
            own_ = a;
            note_allocation(true);
        } else {
            if (hipMalloc(&p_, bytes) != hipSuccess) {
                (void)hipGetLastError();
                p_ = nullptr;
                fail(KRR_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
            }
            own_ = Allocator{};
            note_allocation(false);
        }
        n_ = bytes;
    }
    // Grows (discarding contents) when smaller than `bytes`.
    void reserve(size_t bytes) {
        if (bytes > n_) alloc(bytes);
    }
    void release() {
        if (p_) {
            if (own_.dealloc)
                own_.dealloc(p_, static_cast<void *>(s_), own_.ctx);
            else
                (void)hipFree(p_);
        }
        p_ = nullptr;
        n_ = 0;
    }
    template <class T> T *as() const { return static_cast<T *>(p_); }
    void *get() const { return p_; }
    size_t bytes() const { return n_; }

  private:
    void *p_ = nullptr;
    size_t n_ = 0;
    Allocator own_{};         // the allocator that made the buffer
    hipStream_t s_ = nullptr; // and the stream it was made on
};

template <class T> inline DBuf dalloc(size_t count) { return DBuf(count * sizeof(T)); }

template <class T>
inline void h2d(T *dst, const T *src, size_t count, hipStream_t s) {
    if (count) KRR_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, s));
}
template <class T>
inline void d2h(T *dst, const T *src, size_t count, hipStream_t s) {
    if (count) KRR_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDeviceToHost, s));
}
template <class T> inline DBuf upload(const std::vector<T> &v, hipStream_t s) {
    DBuf b(v.size() * sizeof(T));
    h2d(b.as<T>(), v.data(), v.size(), s);
    return b;
}
inline void sync(hipStream_t s) { KRR_HIP(hipStreamSynchronize(s)); }

inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// Timing with HIP events on a stream.
struct EventTimer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit EventTimer(hipStream_t st) : s(st) {
        KRR_HIP(hipEventCreate(&a));
        KRR_HIP(hipEventCreate(&b));
        KRR_HIP(hipEventRecord(a, s));
    }
    double stop_ms() {
        float ms = 0;
        KRR_HIP(hipEventRecord(b, s));
        KRR_HIP(hipEventSynchronize(b));
        KRR_HIP(hipEventElapsedTime(&ms, a, b));
        return ms;
    }
    ~EventTimer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// ------------------------------------------------------------ device helpers

template <class T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <class T> __device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, 64);
        v = v > w ? v : w;
    }
    return v;
}

template <class T> __device__ __forceinline__ T load_pt(const T *p) { return *p; }

// Converts a point coordinate of either dtype to float / double.
__device__ __forceinline__ double to_f64(float v) { return (double)v; }
__device__ __forceinline__ double to_f64(double v) { return v; }

}  // namespace krr
