// The extern "C" boundary of libkrr (declared in include/krr.h): argument
// checks, handle lifetime, and translation of internal failures into status
// codes with a per-thread message.  Nothing throws across this boundary.
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "internal.hpp"

namespace krr {

thread_local std::string g_last_error;
thread_local hipStream_t g_call_stream = nullptr;

std::mutex g_alloc_mu;
Allocator g_alloc;
std::atomic<int64_t> g_alloc_direct{0}, g_alloc_caller{0};

Allocator current_allocator() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc;
}
hipStream_t call_stream() { return g_call_stream; }
void note_allocation(bool by_caller) { (by_caller ? g_alloc_caller : g_alloc_direct).fetch_add(1); }

std::atomic<int> g_tune[KRR_TUNE_COUNT] = {{4}, {8}, {2048}, {16384}, {1}, {1}};

int tune_get(int knob) { return g_tune[knob].load(std::memory_order_relaxed); }

bool verbose() {
    static const bool v = [] {
        const char *e = std::getenv("KRR_VERBOSE");
        return e && *e && *e != '0';
    }();
    return v;
}

void fail(int code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Error(code, buf);
}


namespace {

template <class F> int guard(F &&f) {
    try {
        g_last_error.clear();
        g_call_stream = nullptr;
        return f();
    } catch (const Error &e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return KRR_E_NOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return KRR_E_HIP;
    } catch (...) {
        g_last_error = "unknown failure";
        return KRR_E_HIP;
    }
}

void require_device() {
    int cnt = 0;
    if (hipGetDeviceCount(&cnt) != hipSuccess || cnt == 0) {
        (void)hipGetLastError();
        fail(KRR_E_NODEVICE, "no HIP device available");
    }
}

// The call's stream; library temporaries are allocated on it.
hipStream_t S(void *p) {
    g_call_stream = static_cast<hipStream_t>(p);
    return g_call_stream;
}

void check_xprec(int32_t xprec) {
    KRR_REQUIRE(xprec == KRR_F32 || xprec == KRR_F64, "point dtype must be KRR_F32 or KRR_F64 (got %d)", xprec);
}

void check_hss_opts(const hss_opts &o, const char *who) {
    KRR_REQUIRE(o.rtol >= 0.0 && o.atol >= 0.0, "%s: tolerances must be >= 0", who);
    KRR_REQUIRE(o.r0 >= 32 && o.r0 % 32 == 0, "%s: r0 must be a positive multiple of 32", who);
    KRR_REQUIRE(o.dr >= 32 && o.dr % 32 == 0, "%s: dr must be a positive multiple of 32", who);
    KRR_REQUIRE(o.r_max >= o.r0, "%s: r_max < r0", who);
    KRR_REQUIRE(o.oversample >= 0 && o.oversample < o.r0, "%s: bad oversample", who);
    KRR_REQUIRE(o.prec >= KRR_F64 && o.prec <= KRR_BF16_SPLIT, "%s: bad prec", who);
    KRR_REQUIRE(o.split_terms == 1 || o.split_terms == 2, "%s: split_terms must be 1 or 2", who);
    KRR_REQUIRE(o.cap_policy == 0 || o.cap_policy == 1, "%s: cap_policy must be 0 or 1", who);
}

// Problem offsets (host, np + 1 entries from 0, non-decreasing) with
// per-problem widths and, where given, ridge parameters.
Batch make_batch(const int64_t *offsets, int32_t np, const double *h, const double *lam, const char *who) {
    KRR_REQUIRE(np >= 1 && offsets && h, "%s: need np >= 1, offsets and h", who);
    KRR_REQUIRE(offsets[0] == 0, "%s: offsets[0] must be 0", who);
    Batch b;
    b.pbeg.assign(offsets, offsets + np + 1);
    b.h.assign(h, h + np);
    if (lam) b.lam.assign(lam, lam + np);
    for (int k = 0; k < np; ++k) {
        KRR_REQUIRE(offsets[k + 1] > offsets[k], "%s: problem %d is empty", who, k);
        KRR_REQUIRE(h[k] > 0.0 && h[k] == h[k], "%s: h[%d] must be positive", who, k);
        if (lam) KRR_REQUIRE(lam[k] >= 0.0, "%s: lambda[%d] must be >= 0", who, k);
    }
    KRR_REQUIRE(offsets[np] <= INT32_MAX, "%s: total size must fit in int32", who);
    return b;
}

// Factor with lambda_k (1 + s_k) for use as a preconditioner, s_k found by a
// bracketed search per problem (a pass refactors only the problems still
// searching, each from its first level; a failing problem stops at its first
// level with a pivot below lambda_k / 2):
//   1. s = 0; on failure jump to the first of 1, 4, 16, ... covering the
//      largest deficit seen (lambda_k / 2 - pivot), and so on until a pass
//      succeeds at s = hi;
//   2. Schur-complement pivots grow faster than the shift, so hi overshoots
//      the smallest usable shift: try hi / 8, then hi / 2, keeping the first
//      that succeeds (else hi).
// A smaller shift is a better preconditioner: on the 16-Gaussian workload at
// n = 2^20 the search ends at s = 32 (40 conjugate-gradient iterations)
// where hi = 256 gives 57.  mult receives every s_k.
hss_ulv_s *factor_shifted(const hss_s *H, const std::vector<double> &lam, hipStream_t s, std::vector<double> &mult) {
    const int np = (int)lam.size();
    std::vector<double> floor(np), lam_s(np), sh(np, 0.0), hi(np, 0.0);
    for (int k = 0; k < np; ++k) floor[k] = 0.5 * lam[k];
    // per problem: 0 try 0, 1 growing, 2 tried hi / 8, 3 tried hi / 2, 4 back at hi, 5 done
    std::vector<int> stage(np, 0);
    auto *F = new hss_ulv_s();
    try {
        for (int attempt = 0; attempt < 20; ++attempt) {
            std::vector<uint8_t> act(np, 0);
            for (int k = 0; k < np; ++k) {
                lam_s[k] = lam[k] * (1.0 + sh[k]);
                act[k] = stage[k] < 5;
            }
            std::vector<double> deficit;
            ulv_factor(H, lam_s, floor, s, F, &deficit, true, &act);
            int left = 0;
            for (int k = 0; k < np; ++k) {
                if (stage[k] == 5) continue;
                const bool ok = !act[k];
                auto grow = [&] {  // next grid shift covering the deficit
                    const double target = sh[k] * lam[k] + deficit[k];
                    double next = sh[k] == 0.0 ? 1.0 : 4.0 * sh[k];
                    while (next * lam[k] < target && next < 1e12) next *= 4.0;
                    sh[k] = next;
                    stage[k] = 1;
                };
                switch (stage[k]) {
                    case 0:
                        if (ok) stage[k] = 5; else grow();
                        break;
                    case 1:
                        if (!ok) { grow(); break; }
                        hi[k] = sh[k];
                        if (hi[k] / 8.0 >= 1.0) { sh[k] = hi[k] / 8.0; stage[k] = 2; } else stage[k] = 5;
                        break;
                    case 2:
                        if (ok) stage[k] = 5; else { sh[k] = hi[k] / 2.0; stage[k] = 3; }
                        break;
                    case 3:
                        if (ok) stage[k] = 5; else { sh[k] = hi[k]; stage[k] = 4; }
                        break;
                    default:  // 4: hi passed before; grow again if it does not now
                        if (ok) stage[k] = 5; else grow();
                        break;
                }
                if (stage[k] != 5) ++left;
            }
            if (verbose()) fprintf(stderr, "[krr] ulv shift pass %d: %d of %d problems retry\n", attempt, left, np);
            if (left == 0) {
                mult = sh;
                return F;
            }
        }
    } catch (...) {
        delete F;
        throw;
    }
    delete F;
    fail(KRR_E_NUMERIC, "ULV: no positive definite shift found in 20 passes");
}

}  // namespace
}  // namespace krr

using namespace krr;

extern "C" {

const char *krr_last_error(void) { return g_last_error.c_str(); }

int krr_set_allocator(void *(*alloc)(size_t, void *, void *), void (*dealloc)(void *, void *, void *), void *ctx) {
    return guard([&] {
        KRR_REQUIRE((alloc == nullptr) == (dealloc == nullptr), "krr_set_allocator: give both functions or neither");
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        g_alloc = Allocator{alloc, dealloc, ctx};
        return KRR_OK;
    });
}

int krr_alloc_counts(int64_t *direct, int64_t *by_caller) {
    return guard([&] {
        KRR_REQUIRE(direct != nullptr && by_caller != nullptr, "krr_alloc_counts: NULL argument");
        *direct = g_alloc_direct.load();
        *by_caller = g_alloc_caller.load();
        return KRR_OK;
    });
}

int krr_device_count(void) {
    int cnt = 0;
    if (hipGetDeviceCount(&cnt) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return cnt;
}

int krr_cluster_2mn(const void *X, int32_t xprec, int64_t n, int32_t d, const krr_cluster_opts *opts, void *stream,
                    int64_t *perm, krr_tree *out) {
    return guard([&] {
        KRR_REQUIRE(out != nullptr && opts != nullptr, "krr_cluster_2mn: NULL opts or out");
        *out = nullptr;
        check_xprec(xprec);
        KRR_REQUIRE(n >= 1 && d >= 1, "krr_cluster_2mn: need n >= 1 and d >= 1");
        KRR_REQUIRE(n <= INT32_MAX, "krr_cluster_2mn: n must fit in int32");
        KRR_REQUIRE(X != nullptr && perm != nullptr, "krr_cluster_2mn: NULL X or perm");
        KRR_REQUIRE(opts->leaf_size >= 1 && opts->max_iter >= 1, "krr_cluster_2mn: leaf_size and max_iter must be >= 1");
        require_device();
        auto *t = new krr_tree_s();
        try {
            cluster_2mn(X, xprec, n, d, std::vector<int64_t>{0, n}, *opts, S(stream), perm, *t);
        } catch (...) {
            delete t;
            throw;
        }
        *out = t;
        return KRR_OK;
    });
}

int krr_cluster_order(const void *X, int32_t xprec, int64_t n, int32_t d, int32_t method, const int64_t *offsets,
                      int32_t np, const krr_cluster_opts *opts, void *stream, int64_t *perm, krr_tree *out) {
    return guard([&] {
        KRR_REQUIRE(out != nullptr && opts != nullptr, "krr_cluster_order: NULL opts or out");
        *out = nullptr;
        check_xprec(xprec);
        KRR_REQUIRE(method >= KRR_ORDER_2MN && method <= KRR_ORDER_PCA, "krr_cluster_order: unknown method %d",
                    method);
        std::vector<int64_t> roots{0, n};
        if (offsets) {
            KRR_REQUIRE(np >= 1 && offsets[0] == 0, "krr_cluster_order: need np >= 1 and offsets[0] = 0");
            for (int k = 0; k < np; ++k)
                KRR_REQUIRE(offsets[k + 1] > offsets[k], "krr_cluster_order: problem %d is empty", k);
            KRR_REQUIRE(offsets[np] == n, "krr_cluster_order: offsets[np] must equal n");
            roots.assign(offsets, offsets + np + 1);
        }
        KRR_REQUIRE(n >= 1 && d >= 1, "krr_cluster_order: need n >= 1 and d >= 1");
        KRR_REQUIRE(n <= INT32_MAX, "krr_cluster_order: n must fit in int32");
        KRR_REQUIRE(X != nullptr && perm != nullptr, "krr_cluster_order: NULL X or perm");
        KRR_REQUIRE(opts->leaf_size >= 1, "krr_cluster_order: leaf_size must be >= 1");
        KRR_REQUIRE(method != KRR_ORDER_2MN || opts->max_iter >= 1, "krr_cluster_order: max_iter must be >= 1");
        require_device();
        auto *t = new krr_tree_s();
        try {
            cluster_2mn(X, xprec, n, d, roots, *opts, S(stream), perm, *t, method);
        } catch (...) {
            delete t;
            throw;
        }
        *out = t;
        return KRR_OK;
    });
}

int krr_tree_from_host(const int64_t *nodes_host, int64_t n_nodes, krr_tree *out) {
    return guard([&] {
        KRR_REQUIRE(out != nullptr && nodes_host != nullptr && n_nodes >= 1, "krr_tree_from_host: bad arguments");
        *out = nullptr;
        auto *t = new krr_tree_s();
        t->nodes.assign(nodes_host, nodes_host + 5 * n_nodes);
        // every node without a parent is the root of one tree of a forest
        for (int64_t i = 0; i < n_nodes; ++i)
            if (t->parent(i) < 0) t->roots.push_back(i);
        t->n = t->roots.empty() ? 0 : t->e(t->roots.back());
        try {
            validate_tree(t);
        } catch (...) {
            delete t;
            throw;
        }
        *out = t;
        return KRR_OK;
    });
}

int krr_tree_size(krr_tree t, int64_t *n_host, int64_t *n_nodes_host) {
    return guard([&] {
        KRR_REQUIRE(t != nullptr, "krr_tree_size: NULL tree");
        if (n_host) *n_host = t->n;
        if (n_nodes_host) *n_nodes_host = t->n_nodes();
        return KRR_OK;
    });
}

int krr_tree_export(krr_tree t, int64_t *nodes_host, int64_t *stats_host) {
    return guard([&] {
        KRR_REQUIRE(t != nullptr, "krr_tree_export: NULL tree");
        if (nodes_host) std::memcpy(nodes_host, t->nodes.data(), sizeof(int64_t) * t->nodes.size());
        if (stats_host) std::memcpy(stats_host, t->stats.data(), sizeof(int64_t) * 4);
        return KRR_OK;
    });
}

void krr_tree_destroy(krr_tree t) { delete t; }

int krr_gather_rows(const void *src, int32_t prec, int64_t n, int32_t cols, const int64_t *perm, void *dst,
                    void *stream) {
    return guard([&] {
        KRR_REQUIRE(n >= 0 && cols >= 1, "krr_gather_rows: bad sizes");
        KRR_REQUIRE(n == 0 || (src && dst && perm), "krr_gather_rows: NULL pointer");
        check_xprec(prec);
        require_device();
        gather_rows(src, prec, n, cols, perm, dst, false, S(stream));
        return KRR_OK;
    });
}

int krr_scatter_rows(const void *src, int32_t prec, int64_t n, int32_t cols, const int64_t *perm, void *dst,
                     void *stream) {
    return guard([&] {
        KRR_REQUIRE(n >= 0 && cols >= 1, "krr_scatter_rows: bad sizes");
        KRR_REQUIRE(n == 0 || (src && dst && perm), "krr_scatter_rows: NULL pointer");
        check_xprec(prec);
        require_device();
        gather_rows(src, prec, n, cols, perm, dst, true, S(stream));
        return KRR_OK;
    });
}

int kernel_matvec(const void *X, int64_t m, const void *Y, int64_t n, int32_t d, int32_t xprec, double h,
                  const double *W, int32_t nrhs, double beta, double *Out, int32_t prec, void *stream) {
    return guard([&] {
        check_xprec(xprec);
        KRR_REQUIRE(m >= 0 && n >= 1 && d >= 1, "kernel_matvec: need m >= 0, n >= 1, d >= 1");
        KRR_REQUIRE(nrhs >= 1 && nrhs <= 64, "kernel_matvec: nrhs must be in [1, 64]");
        KRR_REQUIRE(h > 0.0 && h == h, "kernel_matvec: h must be positive");
        KRR_REQUIRE(prec == KRR_F32 || prec == KRR_F64, "kernel_matvec: prec must be KRR_F32 or KRR_F64");
        KRR_REQUIRE(m == 0 || (X && Y && W && Out), "kernel_matvec: NULL pointer");
        require_device();
        kernel_matvec_impl(X, m, Y, n, d, xprec, h, W, nrhs, beta, Out, prec, S(stream));
        return KRR_OK;
    });
}

struct krr_tile_map_s {
    krr::SymSkip map;
};

int krr_tile_map_create(krr_tile_map_t *map_out) {
    return guard([&] {
        KRR_REQUIRE(map_out, "krr_tile_map_create: NULL pointer");
        *map_out = new krr_tile_map_s();
        return KRR_OK;
    });
}

int krr_tile_map_destroy(krr_tile_map_t map) {
    return guard([&] {
        KRR_REQUIRE(map, "krr_tile_map_destroy: NULL handle");
        delete map;
        return KRR_OK;
    });
}

int kernel_matvec_mapped(const void *X, int64_t n, int32_t d, int32_t xprec, double h, const double *W,
                         int32_t nrhs, double beta, double *Out, krr_tile_map_t map, void *stream) {
    return guard([&] {
        check_xprec(xprec);
        KRR_REQUIRE(map, "kernel_matvec_mapped: NULL map");
        KRR_REQUIRE(n >= 1 && d >= 1, "kernel_matvec_mapped: need n >= 1, d >= 1");
        KRR_REQUIRE(nrhs >= 1 && nrhs <= 64, "kernel_matvec_mapped: nrhs must be in [1, 64]");
        KRR_REQUIRE(h > 0.0 && h == h, "kernel_matvec_mapped: h must be positive");
        KRR_REQUIRE(X && W && Out, "kernel_matvec_mapped: NULL pointer");
        require_device();
        kernel_matvec_impl(X, n, X, n, d, xprec, h, W, nrhs, beta, Out, KRR_F32, S(stream), nullptr, &map->map);
        return KRR_OK;
    });
}

int krr_tile_map_counts(krr_tile_map_t map, int64_t *counts_host, void *stream) {
    return guard([&] {
        KRR_REQUIRE(map && counts_host, "krr_tile_map_counts: NULL pointer");
        require_device();
        const bool rec = map->map.ready;
        counts_host[0] = rec ? krr::sym_skip_kept(map->map, S(stream)) : 0;
        counts_host[1] = rec ? map->map.tiles : 0;
        counts_host[2] = rec ? map->map.entries_per_tile : 0;
        return KRR_OK;
    });
}

int kernel_sample(const void *X, int64_t n, int32_t d, int32_t xprec, double h, const float *R, int32_t r,
                  const int32_t *leaf_begin, const int32_t *leaf_end, void *Sout, int32_t prec, int32_t split_terms,
                  void *stream) {
    return guard([&] {
        check_xprec(xprec);
        KRR_REQUIRE(n >= 1 && d >= 1, "kernel_sample: need n >= 1 and d >= 1");
        KRR_REQUIRE(r >= 32 && r % 32 == 0, "kernel_sample: r must be a positive multiple of 32");
        KRR_REQUIRE(h > 0.0, "kernel_sample: h must be positive");
        KRR_REQUIRE(prec >= KRR_F64 && prec <= KRR_BF16_SPLIT, "kernel_sample: bad prec %d", prec);
        KRR_REQUIRE(split_terms == 1 || split_terms == 2, "kernel_sample: split_terms must be 1 or 2");
        KRR_REQUIRE((leaf_begin == nullptr) == (leaf_end == nullptr), "kernel_sample: give both leaf arrays or none");
        KRR_REQUIRE(X && R && Sout, "kernel_sample: NULL pointer");
        require_device();
        sample_product(X, n, d, xprec, h, R, r, leaf_begin, leaf_end, Sout, prec, split_terms, S(stream));
        return KRR_OK;
    });
}

int krr_random_block(uint64_t seed, int64_t n, int32_t r, int32_t c0, float *R, void *stream) {
    return guard([&] {
        KRR_REQUIRE(n >= 0 && r >= 1 && c0 >= 0 && (n == 0 || R), "krr_random_block: bad arguments");
        require_device();
        random_block(seed, n, r, c0, R, r, S(stream));
        return KRR_OK;
    });
}

int kernel_matvec_bwd(const void *X, int64_t m, const void *Y, int64_t n, int32_t d, int32_t xprec, double h,
                      const double *W, const double *G, int32_t nrhs, double *dX, double *dY, double *dW,
                      double *dh, int32_t prec, void *stream) {
    return guard([&] {
        check_xprec(xprec);
        KRR_REQUIRE(m >= 1 && n >= 1 && d >= 1 && nrhs >= 1, "kernel_matvec_bwd: bad sizes");
        KRR_REQUIRE(h > 0.0, "kernel_matvec_bwd: h must be positive");
        KRR_REQUIRE(prec == KRR_F32 || prec == KRR_F64, "kernel_matvec_bwd: prec must be KRR_F32 or KRR_F64");
        KRR_REQUIRE(X && Y && W && G, "kernel_matvec_bwd: NULL pointer");
        require_device();
        kernel_matvec_bwd_impl(X, m, Y, n, d, xprec, h, W, G, nrhs, dX, dY, dW, dh, prec, S(stream));
        return KRR_OK;
    });
}

int hss_compress(krr_tree t, const void *Xp, int32_t xprec, int32_t d, double h, const hss_opts *opts, void *stream,
                 hss_t *out, hss_stats *stats_host) {
    return guard([&] {
        KRR_REQUIRE(out != nullptr, "hss_compress: NULL out");
        *out = nullptr;
        KRR_REQUIRE(t != nullptr && opts != nullptr && Xp != nullptr, "hss_compress: NULL argument");
        check_xprec(xprec);
        KRR_REQUIRE(d >= 1 && h > 0.0, "hss_compress: need d >= 1 and h > 0");
        const hss_opts &o = *opts;
        check_hss_opts(o, "hss_compress");
        validate_tree(t);
        require_device();
        auto *H = new hss_s();
        try {
            compress(t, Xp, xprec, d, std::vector<double>(t->roots.size(), h), o, S(stream), H, stats_host);
        } catch (...) {
            delete H;
            throw;
        }
        *out = H;
        return KRR_OK;
    });
}

// Handle storage goes back to its allocator once every stream is done with
// it (hipFree synchronizes implicitly; a stream-ordered allocator does not).
void hss_destroy(hss_t H) {
    if (!H) return;
    (void)hipDeviceSynchronize();
    delete H;
}

int hss_matvec(hss_t H, const double *x, int32_t nrhs, double *y, void *stream) {
    return guard([&] {
        KRR_REQUIRE(H != nullptr && x && y && nrhs >= 1, "hss_matvec: bad arguments");
        require_device();
        hss_matvec_impl(H, x, nrhs, y, S(stream));
        return KRR_OK;
    });
}

int hss_export_sizes(hss_t H, int64_t *n_nodes_host, int64_t *n_dbl_host, int64_t *n_int_host) {
    return guard([&] {
        KRR_REQUIRE(H != nullptr, "hss_export_sizes: NULL handle");
        if (n_nodes_host) *n_nodes_host = (int64_t)H->node.size();
        if (n_dbl_host) *n_dbl_host = H->nU + H->nD + H->nB;
        if (n_int_host) *n_int_host = H->nJ;
        return KRR_OK;
    });
}

int hss_export(hss_t H, int64_t *table_host, double *dbl_host, int64_t *int_host, void *stream) {
    return guard([&] {
        KRR_REQUIRE(H != nullptr && table_host && dbl_host && int_host, "hss_export: NULL argument");
        hipStream_t s = S(stream);
        const int64_t nn = (int64_t)H->node.size();
        const int64_t baseD = H->nU, baseB = H->nU + H->nD;
        for (int64_t i = 0; i < nn; ++i) {
            const HNode &q = H->node[i];
            int64_t *row = table_host + 10 * i;
            row[0] = q.b;
            row[1] = q.e;
            row[2] = q.left;
            row[3] = q.right;
            row[4] = q.m;
            row[5] = q.k;
            row[6] = q.offU;
            row[7] = q.offD >= 0 ? baseD + q.offD : -1;
            row[8] = q.offB >= 0 ? baseB + q.offB : -1;
            row[9] = q.offJ;
        }
        d2h(dbl_host, H->U.as<double>(), H->nU, s);
        d2h(dbl_host + baseD, H->D.as<double>(), H->nD, s);
        d2h(dbl_host + baseB, H->B.as<double>(), H->nB, s);
        std::vector<int32_t> j32(H->nJ);
        d2h(j32.data(), H->J.as<int32_t>(), H->nJ, s);
        sync(s);
        for (int64_t i = 0; i < H->nJ; ++i) int_host[i] = j32[i];
        return KRR_OK;
    });
}

int hss_ulv_factor(hss_t H, double lambda, void *stream, hss_ulv_t *out) {
    return guard([&] {
        KRR_REQUIRE(out != nullptr, "hss_ulv_factor: NULL out");
        *out = nullptr;
        KRR_REQUIRE(H != nullptr, "hss_ulv_factor: NULL handle");
        KRR_REQUIRE(lambda >= 0.0, "hss_ulv_factor: lambda must be >= 0");
        require_device();
        auto *F = new hss_ulv_s();
        try {
            const size_t np = H->hprob.size();
            ulv_factor(H, std::vector<double>(np, lambda), std::vector<double>(np, 0.0), S(stream), F);
        } catch (...) {
            delete F;
            throw;
        }
        *out = F;
        return KRR_OK;
    });
}

int hss_ulv_factor_spd(hss_t H, double lambda, double pivot_floor, void *stream, hss_ulv_t *out,
                       int64_t *clamped_host) {
    return guard([&] {
        KRR_REQUIRE(out != nullptr, "hss_ulv_factor_spd: NULL out");
        *out = nullptr;
        KRR_REQUIRE(H != nullptr, "hss_ulv_factor_spd: NULL handle");
        KRR_REQUIRE(lambda >= 0.0, "hss_ulv_factor_spd: lambda must be >= 0");
        KRR_REQUIRE(pivot_floor > 0.0, "hss_ulv_factor_spd: pivot_floor must be > 0");
        require_device();
        auto *F = new hss_ulv_s();
        try {
            const size_t np = H->hprob.size();
            int64_t clamped =
                ulv_factor(H, std::vector<double>(np, lambda), std::vector<double>(np, pivot_floor), S(stream), F);
            if (clamped_host) *clamped_host = clamped;
            if (verbose()) fprintf(stderr, "[krr] ulv factor: %lld pivots raised to %g\n", (long long)clamped, pivot_floor);
        } catch (...) {
            delete F;
            throw;
        }
        *out = F;
        return KRR_OK;
    });
}

int hss_ulv_factor_shifted(hss_t H, double lambda, void *stream, hss_ulv_t *out, double *shift_host) {
    return guard([&] {
        KRR_REQUIRE(out != nullptr, "hss_ulv_factor_shifted: NULL out");
        *out = nullptr;
        KRR_REQUIRE(H != nullptr, "hss_ulv_factor_shifted: NULL handle");
        KRR_REQUIRE(lambda > 0.0, "hss_ulv_factor_shifted: lambda must be > 0");
        require_device();
        std::vector<double> mult;
        *out = factor_shifted(H, std::vector<double>(H->hprob.size(), lambda), S(stream), mult);
        if (shift_host) *shift_host = *std::max_element(mult.begin(), mult.end()) * lambda;
        return KRR_OK;
    });
}

void hss_ulv_destroy(hss_ulv_t F) {
    if (!F) return;
    (void)hipDeviceSynchronize();
    delete F;
}

int hss_ulv_use_graph(hss_ulv_t F, int32_t enable) {
    return guard([&] {
        KRR_REQUIRE(F != nullptr, "hss_ulv_use_graph: NULL factor");
        F->use_graph = enable != 0;
        return KRR_OK;
    });
}

int hss_solve(hss_ulv_t F, const double *B, int32_t nrhs, double *Xout, void *stream) {
    return guard([&] {
        KRR_REQUIRE(F != nullptr && B && Xout, "hss_solve: NULL argument");
        KRR_REQUIRE(nrhs >= 1, "hss_solve: nrhs must be >= 1");
        require_device();
        ulv_solve(F, B, nrhs, Xout, S(stream));
        return KRR_OK;
    });
}

int krr_refine(hss_ulv_t F, const void *Xp, int64_t n, int32_t xprec, int32_t d, double h, double lambda,
               const double *Y, int32_t nrhs, double *alpha, double tol, int32_t max_iter, int32_t mv_prec,
               int32_t res_prec, void *stream, krr_refine_stats *stats_host) {
    return guard([&] {
        KRR_REQUIRE(Xp && Y && alpha, "krr_refine: NULL argument");
        KRR_REQUIRE(n >= 1 && (!F || F->n == n), "krr_refine: n must be >= 1 and match the factor");
        check_xprec(xprec);
        KRR_REQUIRE(nrhs >= 1 && nrhs <= 64, "krr_refine: nrhs must be in [1, 64]");
        KRR_REQUIRE(h > 0.0 && lambda >= 0.0 && tol > 0.0 && max_iter >= 0, "krr_refine: bad parameters");
        KRR_REQUIRE(mv_prec == KRR_F32 || mv_prec == KRR_F64, "krr_refine: mv_prec must be KRR_F32 or KRR_F64");
        KRR_REQUIRE(res_prec == KRR_F32 || res_prec == KRR_F64, "krr_refine: res_prec must be KRR_F32 or KRR_F64");
        require_device();
        int rc = refine(F, n, Xp, xprec, d, h, lambda, Y, nrhs, alpha, tol, max_iter, mv_prec, res_prec, S(stream),
                        stats_host);
        if (rc == KRR_E_NOT_CONVERGED) g_last_error = "krr_refine: tolerance not reached within max_iter";
        return rc;
    });
}

int krr_predict(const void *Xt, int64_t m, const void *Xp, int64_t n, int32_t d, int32_t xprec, double h,
                const double *alpha, int32_t nrhs, double *scores, int32_t *labels, int32_t prec, void *stream) {
    return guard([&] {
        check_xprec(xprec);
        KRR_REQUIRE(m >= 0 && n >= 1 && d >= 1 && nrhs >= 1 && nrhs <= 64, "krr_predict: bad sizes");
        KRR_REQUIRE(h > 0.0, "krr_predict: h must be positive");
        KRR_REQUIRE(prec == KRR_F32 || prec == KRR_F64, "krr_predict: prec must be KRR_F32 or KRR_F64");
        KRR_REQUIRE(m == 0 || (Xt && Xp && alpha && scores), "krr_predict: NULL pointer");
        require_device();
        kernel_matvec_impl(Xt, m, Xp, n, d, xprec, h, alpha, nrhs, 0.0, scores, prec, S(stream));
        if (labels) predict_labels(scores, m, nrhs, labels, S(stream));
        return KRR_OK;
    });
}

int krr_predict_noalloc(const void *Xt, int64_t m, const void *Xp, int64_t n, int32_t d, int32_t xprec, double h,
                        const double *alpha, int32_t nrhs, double *scores, int32_t *labels, int32_t prec,
                        void *stream) {
    return guard([&] {
        check_xprec(xprec);
        KRR_REQUIRE(m >= 0 && n >= 1 && d >= 1 && nrhs >= 1 && nrhs <= 64, "krr_predict_noalloc: bad sizes");
        KRR_REQUIRE(d <= 64, "krr_predict_noalloc: d = %d > 64 is not supported (use krr_predict)", d);
        KRR_REQUIRE(h > 0.0, "krr_predict_noalloc: h must be positive");
        KRR_REQUIRE(prec == KRR_F32 || prec == KRR_F64, "krr_predict_noalloc: prec must be KRR_F32 or KRR_F64");
        KRR_REQUIRE(m == 0 || (Xt && Xp && alpha && scores), "krr_predict_noalloc: NULL pointer");
        KRR_REQUIRE(Xt != Xp, "krr_predict_noalloc: Xt and Xp alias (use krr_predict)");
        require_device();
        if (m == 0) return KRR_OK;
        predict_noalloc(Xt, m, Xp, n, d, xprec, h, alpha, nrhs, scores, labels, prec, S(stream));
        return KRR_OK;
    });
}

int krr_set_tuning(int32_t knob, int32_t value) {
    return guard([&] {
        KRR_REQUIRE(knob >= 0 && knob < KRR_TUNE_COUNT, "krr_set_tuning: unknown knob %d", knob);
        switch (knob) {
            case KRR_TUNE_SYMMETRIC: KRR_REQUIRE(value >= 0 && value <= 4, "krr_set_tuning: symmetric is 0 to 4"); break;
            case KRR_TUNE_SAMPLE_RB:
                KRR_REQUIRE(value == 1 || value == 2 || value == 4 || value == 8, "krr_set_tuning: sample RB is 1, 2, 4 or 8");
                break;
            case KRR_TUNE_MV_BLOCKS: KRR_REQUIRE(value >= 64 && value <= 65536, "krr_set_tuning: blocks in [64, 65536]"); break;
            case KRR_TUNE_SAMPLE_SKIP: KRR_REQUIRE(value == 0 || value == 1, "krr_set_tuning: sample skip is 0 or 1"); break;
            case KRR_TUNE_SYM_SKIP: KRR_REQUIRE(value >= 0 && value <= 2, "krr_set_tuning: symmetric skip is 0, 1 or 2"); break;
            case KRR_TUNE_SYM_CHUNK:
                KRR_REQUIRE(value >= 64 && value % 64 == 0 && value <= (1 << 24), "krr_set_tuning: chunk multiple of 64");
                break;
        }
        g_tune[knob].store(value, std::memory_order_relaxed);
        return KRR_OK;
    });
}

int krr_get_tuning(int32_t knob, int32_t *value_host) {
    return guard([&] {
        KRR_REQUIRE(knob >= 0 && knob < KRR_TUNE_COUNT && value_host, "krr_get_tuning: bad arguments");
        *value_host = tune_get(knob);
        return KRR_OK;
    });
}

int krr_val_residual(const double *f, const double *yv, int64_t m, int32_t k, double *ge, double *loss,
                     void *stream) {
    return guard([&] {
        KRR_REQUIRE(f && yv && ge && loss, "krr_val_residual: NULL pointer");
        KRR_REQUIRE(m >= 1 && k >= 1, "krr_val_residual: need m >= 1 and k >= 1");
        require_device();
        val_residual(f, yv, m, k, ge, loss, S(stream));
        return KRR_OK;
    });
}

int krr_val_grad_finish(const double *bta, const double *dh_v, const double *dh_t, const double *gscale, double h,
                        double lambda, double *out, void *stream) {
    return guard([&] {
        KRR_REQUIRE(bta && dh_v && dh_t && out, "krr_val_grad_finish: NULL pointer");
        KRR_REQUIRE(h > 0.0 && lambda > 0.0, "krr_val_grad_finish: h and lambda must be positive");
        require_device();
        val_grad_finish(bta, dh_v, dh_t, gscale, h, lambda, out, S(stream));
        return KRR_OK;
    });
}

int krr_dot_columns(const double *a, const double *b, int64_t n, int32_t k, double *out, void *stream) {
    return guard([&] {
        KRR_REQUIRE(a && b && out && n >= 0 && k >= 1, "krr_dot_columns: bad arguments");
        require_device();
        DBuf scratch;
        dot_columns(a, b, n, k, out, scratch, S(stream));
        sync(S(stream));
        return KRR_OK;
    });
}

// ------------------------------------------------------------ batched form

int krr_cluster_2mn_batched(const void *X, int32_t xprec, const int64_t *offsets, int32_t np, int32_t d,
                            const krr_cluster_opts *opts, void *stream, int64_t *perm, krr_tree *out) {
    return guard([&] {
        KRR_REQUIRE(out != nullptr && opts != nullptr, "krr_cluster_2mn_batched: NULL opts or out");
        *out = nullptr;
        check_xprec(xprec);
        KRR_REQUIRE(np >= 1 && offsets != nullptr && d >= 1, "krr_cluster_2mn_batched: need np >= 1, offsets, d >= 1");
        KRR_REQUIRE(offsets[0] == 0, "krr_cluster_2mn_batched: offsets[0] must be 0");
        for (int k = 0; k < np; ++k)
            KRR_REQUIRE(offsets[k + 1] > offsets[k], "krr_cluster_2mn_batched: problem %d is empty", k);
        const int64_t n = offsets[np];
        KRR_REQUIRE(n <= INT32_MAX, "krr_cluster_2mn_batched: total size must fit in int32");
        KRR_REQUIRE(X != nullptr && perm != nullptr, "krr_cluster_2mn_batched: NULL X or perm");
        KRR_REQUIRE(opts->leaf_size >= 1 && opts->max_iter >= 1,
                    "krr_cluster_2mn_batched: leaf_size and max_iter must be >= 1");
        require_device();
        auto *t = new krr_tree_s();
        try {
            cluster_2mn(X, xprec, n, d, std::vector<int64_t>(offsets, offsets + np + 1), *opts, S(stream), perm, *t);
        } catch (...) {
            delete t;
            throw;
        }
        *out = t;
        return KRR_OK;
    });
}

int krr_tree_roots(krr_tree t, int64_t *roots_host, int32_t *count_host) {
    return guard([&] {
        KRR_REQUIRE(t != nullptr, "krr_tree_roots: NULL tree");
        if (count_host) *count_host = (int32_t)t->roots.size();
        if (roots_host) std::memcpy(roots_host, t->roots.data(), sizeof(int64_t) * t->roots.size());
        return KRR_OK;
    });
}

int hss_compress_batched(krr_tree t, const void *Xp, int32_t xprec, int32_t d, const double *h, const hss_opts *opts,
                         void *stream, hss_t *out, hss_stats *stats_host) {
    return guard([&] {
        KRR_REQUIRE(out != nullptr, "hss_compress_batched: NULL out");
        *out = nullptr;
        KRR_REQUIRE(t != nullptr && opts != nullptr && Xp != nullptr && h != nullptr,
                    "hss_compress_batched: NULL argument");
        check_xprec(xprec);
        KRR_REQUIRE(d >= 1, "hss_compress_batched: need d >= 1");
        check_hss_opts(*opts, "hss_compress_batched");
        validate_tree(t);
        const size_t np = t->roots.size();
        for (size_t k = 0; k < np; ++k) KRR_REQUIRE(h[k] > 0.0, "hss_compress_batched: h[%zu] must be > 0", k);
        require_device();
        auto *H = new hss_s();
        try {
            compress(t, Xp, xprec, d, std::vector<double>(h, h + np), *opts, S(stream), H, stats_host);
        } catch (...) {
            delete H;
            throw;
        }
        *out = H;
        return KRR_OK;
    });
}

int hss_num_problems(hss_t H, int32_t *np_host) {
    return guard([&] {
        KRR_REQUIRE(H != nullptr && np_host != nullptr, "hss_num_problems: NULL argument");
        *np_host = (int32_t)H->hprob.size();
        return KRR_OK;
    });
}

int hss_ulv_factor_batched(hss_t H, const double *lambda, int32_t shifted, void *stream, hss_ulv_t *out,
                           double *shift_mult_host) {
    return guard([&] {
        KRR_REQUIRE(out != nullptr, "hss_ulv_factor_batched: NULL out");
        *out = nullptr;
        KRR_REQUIRE(H != nullptr && lambda != nullptr, "hss_ulv_factor_batched: NULL argument");
        const size_t np = H->hprob.size();
        std::vector<double> lam(lambda, lambda + np);
        for (size_t k = 0; k < np; ++k)
            KRR_REQUIRE(shifted ? lam[k] > 0.0 : lam[k] >= 0.0, "hss_ulv_factor_batched: bad lambda[%zu]", k);
        require_device();
        if (shifted) {
            std::vector<double> mult;
            *out = factor_shifted(H, lam, S(stream), mult);
            if (shift_mult_host) std::copy(mult.begin(), mult.end(), shift_mult_host);
            return KRR_OK;
        }
        auto *F = new hss_ulv_s();
        try {
            ulv_factor(H, lam, std::vector<double>(np, 0.0), S(stream), F);
        } catch (...) {
            delete F;
            throw;
        }
        if (shift_mult_host) std::fill(shift_mult_host, shift_mult_host + np, 0.0);
        *out = F;
        return KRR_OK;
    });
}

int kernel_sample_batched(const void *X, int32_t xprec, const int64_t *offsets, int32_t np, int32_t d,
                          const double *h, const float *R, int32_t r, const int32_t *leaf_begin,
                          const int32_t *leaf_end, void *Sout, int32_t prec, int32_t split_terms, void *stream) {
    return guard([&] {
        check_xprec(xprec);
        Batch b = make_batch(offsets, np, h, nullptr, "kernel_sample_batched");
        KRR_REQUIRE(d >= 1, "kernel_sample_batched: need d >= 1");
        KRR_REQUIRE(r >= 32 && r % 32 == 0, "kernel_sample_batched: r must be a positive multiple of 32");
        KRR_REQUIRE(prec >= KRR_F64 && prec <= KRR_BF16_SPLIT, "kernel_sample_batched: bad prec %d", prec);
        KRR_REQUIRE(split_terms == 1 || split_terms == 2, "kernel_sample_batched: split_terms must be 1 or 2");
        KRR_REQUIRE((leaf_begin == nullptr) == (leaf_end == nullptr),
                    "kernel_sample_batched: give both leaf arrays or none");
        KRR_REQUIRE(X && R && Sout, "kernel_sample_batched: NULL pointer");
        require_device();
        sample_product(X, b.pbeg.back(), d, xprec, b.h[0], R, r, leaf_begin, leaf_end, Sout, prec, split_terms,
                       S(stream), &b);
        return KRR_OK;
    });
}

int kernel_matvec_batched(const void *X, int32_t xprec, const int64_t *offsets, int32_t np, int32_t d,
                          const double *h, const double *W, int32_t nrhs, double *Out, int32_t prec, void *stream) {
    return guard([&] {
        check_xprec(xprec);
        Batch b = make_batch(offsets, np, h, nullptr, "kernel_matvec_batched");
        KRR_REQUIRE(d >= 1 && nrhs >= 1 && nrhs <= 64, "kernel_matvec_batched: bad sizes");
        KRR_REQUIRE(prec == KRR_F32 || prec == KRR_F64, "kernel_matvec_batched: prec must be KRR_F32 or KRR_F64");
        KRR_REQUIRE(X && W && Out, "kernel_matvec_batched: NULL pointer");
        require_device();
        const int64_t n = b.pbeg.back();
        kernel_matvec_impl(X, n, X, n, d, xprec, b.h[0], W, nrhs, 0.0, Out, prec, S(stream), &b);
        return KRR_OK;
    });
}

int krr_refine_batched(hss_ulv_t F, const void *Xp, int32_t xprec, const int64_t *offsets, int32_t np, int32_t d,
                       const double *h, const double *lambda, const double *Y, int32_t nrhs, double *alpha,
                       double tol, int32_t max_iter, int32_t mv_prec, int32_t res_prec, void *stream,
                       krr_refine_stats *stats_host,
                       double *relres_host) {
    return guard([&] {
        check_xprec(xprec);
        KRR_REQUIRE(lambda != nullptr, "krr_refine_batched: NULL lambda");
        Batch b = make_batch(offsets, np, h, lambda, "krr_refine_batched");
        const int64_t n = b.pbeg.back();
        KRR_REQUIRE(Xp && Y && alpha, "krr_refine_batched: NULL argument");
        KRR_REQUIRE(!F || (F->n == n && F->lamprob.size() == (size_t)np),
                    "krr_refine_batched: the factor must cover the same problems");
        KRR_REQUIRE(d >= 1 && nrhs >= 1 && nrhs <= 64, "krr_refine_batched: bad sizes");
        KRR_REQUIRE(tol > 0.0 && max_iter >= 0, "krr_refine_batched: bad parameters");
        KRR_REQUIRE(mv_prec == KRR_F32 || mv_prec == KRR_F64, "krr_refine_batched: mv_prec must be KRR_F32 or KRR_F64");
        KRR_REQUIRE(res_prec == KRR_F32 || res_prec == KRR_F64,
                    "krr_refine_batched: res_prec must be KRR_F32 or KRR_F64");
        require_device();
        int rc = refine(F, n, Xp, xprec, d, b.h[0], b.lam[0], Y, nrhs, alpha, tol, max_iter, mv_prec, res_prec, S(stream),
                        stats_host, &b, relres_host);
        if (rc == KRR_E_NOT_CONVERGED) g_last_error = "krr_refine_batched: tolerance not reached within max_iter";
        return rc;
    });
}

}  // extern "C"
