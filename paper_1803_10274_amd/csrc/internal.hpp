// Internal types shared by the libkrr translation units.
#pragma once

#include <array>
#include <memory>
#include <vector>

#include "common.hpp"

struct krr_tree_s {
    int64_t n = 0;
    // n_nodes rows of (begin, end, left, right, parent), postorder, root last.
    // A forest (batched problems) lists its trees one after the other; roots
    // holds each tree's root (the last node of its run) and problem k spans
    // [nodes[roots[k]].begin, nodes[roots[k]].end).
    std::vector<int64_t> nodes;
    std::vector<int64_t> roots;
    std::array<int64_t, 4> stats{{0, 0, 0, 0}};
    int64_t n_nodes() const { return (int64_t)nodes.size() / 5; }
    int64_t b(int64_t i) const { return nodes[5 * i]; }
    int64_t e(int64_t i) const { return nodes[5 * i + 1]; }
    int64_t left(int64_t i) const { return nodes[5 * i + 2]; }
    int64_t right(int64_t i) const { return nodes[5 * i + 3]; }
    int64_t parent(int64_t i) const { return nodes[5 * i + 4]; }
    bool leaf(int64_t i) const { return nodes[5 * i + 2] < 0; }
    void set_single_root() { roots.assign(1, n_nodes() - 1); }
};

namespace krr {

// Per-node bookkeeping of a compressed HSS matrix (host side).
struct HNode {
    int64_t b, e, left, right, parent;
    int32_t height;   // 0 at leaves, 1 + max(children) above
    int32_t m;        // rows of U: leaf size, or k_left + k_right
    int32_t k;        // rank (columns of U); 0 at the root
    int64_t offU;     // into U pool (m * k doubles), -1 at the root
    int64_t offD;     // into D pool (leaf: m * m doubles), -1 otherwise
    int64_t offB;     // into B pool (k_left * k_right), -1 at leaves
    int64_t offJ;     // into J pool (k int32 positions), -1 at the root
};

// Nodes grouped by height: every node's children have smaller height, so a
// level is a batch of independent nodes for bottom-up sweeps.
std::vector<std::vector<int>> levels_by_height(std::vector<HNode> &nodes);

void validate_tree(const krr_tree_s *t);

// Independent problems of a batched (block-diagonal) operation: problem k
// owns the consecutive points [pbeg[k], pbeg[k + 1]) and has kernel width
// h[k] and ridge parameter lam[k] (lam may be empty where unused).
struct Batch {
    std::vector<int64_t> pbeg;
    std::vector<double> h, lam;
    // problems a kernel product may leave out (the refinement's converged
    // ones): their output rows are not computed (the plain paths write 0)
    std::vector<uint8_t> skip;
    int np() const { return (int)h.size(); }
    int64_t size(int k) const { return pbeg[k + 1] - pbeg[k]; }
    bool skipped(int k) const { return k < (int)skip.size() && skip[k]; }
    bool any_skipped() const {
        for (uint8_t v : skip)
            if (v) return true;
        return false;
    }
};

// One workgroup's share of a batched kernel product: rows [i0, iend) and
// columns [jlo, jhi) of one problem, whose kernel scale is inv = 1 / (2 h^2)
// (cs = inv log2(e) rounded to FP32 for the exp2 forms).  cps: columns per
// split-K slice where the product splits its columns.
struct SampBlock {
    int64_t i0, iend, jlo, jhi, cps;
    double inv, c2;
    float cs, pad_;
};

// Row blocks of `rows` rows over every problem, larger problems first (their
// blocks carry the most work, so they start before the short ones).
std::vector<SampBlock> row_blocks(const Batch &b, int rows);

// Negligible-tile map of the symmetric FP32-entry product, kept across the
// products of one refinement (same points, same kernel widths): the first
// product that takes the BF16 symmetric form records which of its waves'
// 16-point tiles hold an entry of at least 2^-32, the later ones evaluate
// only those.  key identifies the item layout the map was recorded for; a
// product with another layout records again.
struct SymSkip {
    DBuf bits;
    std::vector<double> key;
    bool ready = false;
    int64_t tiles = 0;          // wave tiles the map covers
    int64_t entries_per_tile = 0;
};
// Number of tiles a recorded map marks for evaluation (synchronizes s).
int64_t sym_skip_kept(const SymSkip &m, hipStream_t s);

// Diagnostic logging to stderr when the environment sets KRR_VERBOSE.
bool verbose();

// Current value of a KRR_TUNE_* knob.
int tune_get(int knob);

}  // namespace krr

struct hss_s {
    int64_t n = 0;
    int32_t d = 0;
    double h = 0;                  // kernel width (problem 0; see hprob)
    std::vector<double> hprob;     // kernel width per problem (forest)
    std::vector<int64_t> pbeg;     // problem k spans [pbeg[k], pbeg[k + 1])
    std::vector<int32_t> nprob;    // problem of each node
    std::vector<krr::HNode> node;
    std::vector<std::vector<int>> levels;
    krr::DBuf U, D, B, J;     // generator pools (FP64, FP64, FP64, int32)
    int64_t nU = 0, nD = 0, nB = 0, nJ = 0;
    int32_t r_final = 0, regrowths = 0, max_rank = 0, truncated = 0;
};

namespace krr {
struct UlvSolvePlan;
}

struct hss_ulv_s {
    // solve plans (one per number of right-hand sides), built on first use
    std::vector<std::shared_ptr<krr::UlvSolvePlan>> plans;
    bool use_graph = true;             // replay each plan's launches as a HIP graph
    int64_t n = 0;
    double lambda = 0;
    std::vector<double> lamprob;        // lambda per problem (forest)
    std::vector<krr::HNode> node;       // copy of the HSS node table
    std::vector<std::vector<int>> levels;
    // Per node: Householder vectors of U's QR (m x k, column j = reflector j),
    // tau (k), the compact WY factor Y of Q = I - V Y V^T (k x k, upper
    // triangular), the inverse L^{-1} of the eliminated block's Cholesky factor
    // ((m-k)^2, lower triangular), and W = A_ce L^{-T} (k x (m-k)).  The root
    // holds the inverse Cholesky factor of its whole reduced block in L.
    std::vector<int64_t> offV, offT, offL, offW, offY;
    krr::DBuf V, T, L, W, Y;
    int64_t nV = 0, nT = 0, nL = 0, nW = 0, nY = 0;
    // The QR of a node's basis (V, tau, Y and the triangular factor Rh passed
    // to the parent, k x k at offY) depends only on the HSS bases, not on
    // lambda or a shift: passes over the same compression (the shift search's
    // tries) reuse it.  qr_ok marks the nodes whose QR is in place.
    krr::DBuf R;
    std::vector<uint8_t> qr_ok;
};

// ------------------------------------------------ entry points across units
namespace krr {

// method: KRR_ORDER_2MN (recursive two-means), _NP, _KD or _PCA
void cluster_2mn(const void *X, int32_t xprec, int64_t n, int32_t d, const std::vector<int64_t> &roots,
                 const krr_cluster_opts &o, hipStream_t s, int64_t *perm, krr_tree_s &tree,
                 int32_t method = KRR_ORDER_2MN);
// skip (optional): the negligible-tile map of a sequence of products with the
// same X = Y and widths (recorded by the first that can use it).
void kernel_matvec_impl(const void *X, int64_t m, const void *Y, int64_t n, int d, int xprec, double h,
                        const double *W, int nrhs, double beta, double *Out, int prec, hipStream_t s,
                        const Batch *batch = nullptr, SymSkip *skip = nullptr);
// FP32-entry K(X, Y; h) W + beta Out for points wider than 64 on the matrix cores.
void kmv_wide_mfma(const float *X, int64_t m, const float *Y, int64_t n, int d, double h, const double *W, int nrhs,
                   double beta, double *Out, hipStream_t s, const Batch *batch);
template <class T>
void kmv_wide_mfma64(const T *X, int64_t m, const T *Y, int64_t n, int d, double h, const double *W, int nrhs,
                     double beta, double *Out, hipStream_t s, const Batch *batch);
void kernel_matvec_bwd_impl(const void *X, int64_t m, const void *Y, int64_t n, int d, int xprec, double h,
                            const double *W, const double *G, int nrhs, double *dX, double *dY, double *dW,
                            double *dh, int prec, hipStream_t s);
void sample_product(const void *X, int64_t n, int d, int xprec, double h, const float *R, int r, const int32_t *lb,
                    const int32_t *le, void *S, int prec, int split, hipStream_t s, const Batch *batch = nullptr);
void random_block(uint64_t seed, int64_t n, int r, int c0, float *R, int ldr, hipStream_t s);
void gather_rows(const void *src, int prec, int64_t n, int cols, const int64_t *perm, void *dst, bool scatter,
                 hipStream_t s);
// hprob: kernel width of each tree of the forest (one entry per root)
void compress(const krr_tree_s *t, const void *Xp, int xprec, int d, const std::vector<double> &hprob,
              const hss_opts &o, hipStream_t s, hss_s *H, hss_stats *st);
// lam / floor: diagonal shift and pivot floor of each problem (per root).
// Returns the number of pivots raised to the floor; deficit (if given)
// receives each problem's largest floor - pivot over the raised pivots.  With
// stop_at_floor, a problem whose pivot falls below its floor stops at that
// level.  active (if given): in, the problems to factor (a factor F already
// holding the others is completed in place); out (with stop_at_floor), the
// problems that stopped.
int64_t ulv_factor(const hss_s *H, const std::vector<double> &lam, const std::vector<double> &floor, hipStream_t s,
                   hss_ulv_s *F, std::vector<double> *deficit = nullptr, bool stop_at_floor = false,
                   std::vector<uint8_t> *active = nullptr);
void ulv_solve(const hss_ulv_s *F, const double *Bin, int nrhs, double *Xout, hipStream_t s);
void hss_matvec_impl(const hss_s *H, const double *x, int nrhs, double *y, hipStream_t s);
// mv_prec: the iterations' kernel products; res_prec: the recomputed true
// residual that confirms convergence and restarts the iteration (KRR_F64 with
// mv_prec KRR_F32 is mixed-precision iterative refinement).
// batch == nullptr: one problem (h, lambda); otherwise per-problem h and lam
// (relres_all, if given, receives np x nrhs relative residuals)
int refine(const hss_ulv_s *F, int64_t n, const void *Xp, int xprec, int d, double h, double lambda, const double *Y,
           int nrhs, double *alpha, double tol, int max_iter, int mv_prec, int res_prec, hipStream_t s,
           krr_refine_stats *st,
           const Batch *batch = nullptr, double *relres_all = nullptr);
void predict_labels(const double *scores, int64_t m, int k, int32_t *labels, hipStream_t s);
void predict_noalloc(const void *Xt, int64_t m, const void *Xp, int64_t n, int d, int xprec, double h,
                     const double *alpha, int nrhs, double *scores, int32_t *labels, int prec, hipStream_t s);
// The plain product Out = K(X, Y) W (d <= 64, no symmetric form) with
// caller-given scratch: its size, and the product (no allocation, no sync).
size_t kernel_matvec_ws_bytes(int64_t m, int64_t n, int d, int nrhs, int prec);
void kernel_matvec_ws(const void *X, int64_t m, const void *Y, int64_t n, int d, int xprec, double h,
                      const double *W, int nrhs, double *Out, int prec, void *ws, size_t ws_bytes, hipStream_t s);
// Out = sum_j exp2(t_ij) t_ij W_j, t_ij = -|x_i - y_j|^2 log2(e) / (2 h^2):
// the product with K o T (FP32 entries, one right-hand side, d <= 64).
void kernel_matvec_q(const void *X, int64_t m, const void *Y, int64_t n, int d, int xprec, double h,
                     const double *W, double *Out, hipStream_t s);
void val_residual(const double *f, const double *yv, int64_t m, int k, double *ge, double *loss, hipStream_t s);
void val_grad_finish(const double *bta, const double *dh_v, const double *dh_t, const double *gscale, double h,
                     double lam, double *out, hipStream_t s);
void dot_columns(const double *a, const double *b, int64_t n, int k, double *out, DBuf &scratch, hipStream_t s);

}  // namespace krr
