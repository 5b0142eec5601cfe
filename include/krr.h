/*
 * krr.h -- C ABI of the MI355X (gfx950) Gaussian-kernel ridge regression
 * library: recursive two-means ordering, HSS compression by randomized
 * sampling, ULV factorization and solve, refinement, prediction, gradients.
 *
 * The system solved is (K + lambda I) alpha = y with the Gaussian kernel
 * K_ij = exp(-||x_i - x_j||^2 / (2 h^2)) (eq. (1.1); Algorithm 1 steps 1-2),
 * then test labels are the signs of K(X', X) alpha (Algorithm 1 steps 3-4).
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE pointers unless the parameter name ends in _host.
 *     Device buffers belong to the caller and must stay alive until the work
 *     enqueued on `stream` has completed.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it; calls that must read results back to plan the
 *     next launch (noted per call) synchronize that stream.
 *   - Matrices are row-major and densely packed (leading dimension = columns).
 *   - Point arrays have dtype KRR_F32 or KRR_F64 (argument `xprec`).
 *   - Return value: KRR_OK (0) or a negative KRR_E_* code.  On error no
 *     handle is created, and krr_last_error() returns a message for the
 *     calling thread.  Nothing throws across this boundary.
 *   - After clustering every quantity is in the PERMUTED order:
 *     perm[i] is the original index of position i.
 *   - A handle must not be used from two host threads at once.
 */
#ifndef KRR_H
#define KRR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    KRR_OK = 0,
    KRR_E_INVAL = -1,         /* invalid argument (sizes, NULL pointers, h <= 0, lambda < 0) */
    KRR_E_NOMEM = -2,         /* device allocation failed */
    KRR_E_HIP = -3,           /* a HIP runtime call or kernel launch failed */
    KRR_E_RANK_CAP = -4,      /* adaptive sampling reached r_max before ranks were revealed */
    KRR_E_NUMERIC = -5,       /* non-finite sample, or a non-positive pivot in a Cholesky factor */
    KRR_E_NOT_CONVERGED = -6, /* refinement stopped at max_iter above the requested tolerance */
    KRR_E_NODEVICE = -7       /* no HIP device is available */
};

/* Arithmetic of the kernel products. */
enum {
    KRR_F64 = 0,        /* all FP64 */
    KRR_F32 = 1,        /* FP32 entries and products, FP32 matrix cores for samples */
    KRR_F16_SPLIT = 2,  /* samples: kernel entries split into FP16 hi (+ lo) terms, FP32 accumulation */
    KRR_BF16_SPLIT = 3  /* samples: as above with BF16 terms */
};

typedef struct krr_tree_s *krr_tree;
typedef struct hss_s *hss_t;
typedef struct hss_ulv_s *hss_ulv_t;

/* ---------------------------------------------------------------- errors */

/* Message for the last failed call on this thread ("" if none). */
const char *krr_last_error(void);

/* Device memory (ownership convention, Algorithm 1's data stay the caller's).
 * Registers the caller's stream-ordered device allocator for every buffer the
 * library allocates from now on: temporaries of a call and the storage of
 * the handles (trees, HSS generators, factors, solve plans).  alloc(bytes,
 * stream, ctx) returns device memory usable in stream order on `stream` (the
 * stream of the call that asks, NULL for the legacy default stream) or NULL
 * on failure (the call then fails with KRR_E_NOMEM); dealloc(ptr, stream, ctx)
 * receives every such buffer back with the stream it was allocated on, when
 * the call or the handle is done with it.  A buffer is always returned to
 * the allocator that made it, also after another one has been registered.
 * alloc = dealloc = NULL restores hipMalloc / hipFree for new buffers.  Not
 * to be called while another thread is inside the library.  Errors:
 * KRR_E_INVAL when only one of the two functions is given. */
int krr_set_allocator(void *(*alloc)(size_t, void *, void *), void (*dealloc)(void *, void *, void *),
                      void *ctx);

/* Device allocations made so far by the library: with hipMalloc (direct) and
 * with a registered allocator (by_caller); host outputs.  Errors: KRR_E_INVAL
 * for NULL. */
int krr_alloc_counts(int64_t *direct, int64_t *by_caller);

/* Number of usable HIP devices (0 when none); never fails. */
int krr_device_count(void);

/* ---------------------------------------------------- clustering (A1, A2) */

typedef struct {
    int32_t leaf_size; /* nodes larger than this are split (> 0) */
    int32_t max_iter;  /* Lloyd iteration cap per split (>= 1; 100 recommended) */
    uint64_t seed;     /* key of the counter-based seeding draws */
} krr_cluster_opts;

/*
 * Recursive two-means ordering and cluster tree (Section 4.2 steps 1-3;
 * Section 4.3 "Recursive two-means"; leaf-size rule of Section 4.3; postorder
 * tree of Fig. 3).  Per node [b, e) larger than the leaf size: first seed
 * uniform over the node, second seed with probability proportional to the
 * distance from the first, Lloyd iterations until no label changes (ties to
 * the first cluster, at most max_iter), stable split with first-cluster points
 * first; an empty cluster or all-equal points split the node in halves by
 * position.  The result is bit-for-bit deterministic for a given seed.
 *
 *   X      n x d points (xprec), not modified
 *   perm   (out, n int64) perm[new position] = original index
 *   out    (out) tree handle; free with krr_tree_destroy
 * Synchronizes `stream` once per tree level and once per Lloyd iteration.
 */
int krr_cluster_2mn(const void *X, int32_t xprec, int64_t n, int32_t d,
                    const krr_cluster_opts *opts, void *stream, int64_t *perm,
                    krr_tree *out);

/* The orderings the paper compares with recursive two-means (Section 4.3,
 * "Selected Preprocessing Methods"), each a recursive split of [b, e) while
 * its size exceeds the leaf size, stable, left part first, tree in postorder:
 *   KRR_ORDER_NP   no reordering; halves by position (left floor(size / 2)).
 *   KRR_ORDER_KD   coordinate of maximum spread (max - min; lowest index on
 *                  ties), split at its mean (left: coordinate <= mean).  If
 *                  100 min(left, right) < max(left, right), the median split:
 *                  the floor(size / 2) points first in (coordinate, position)
 *                  order go left.  Zero spread: halves.
 *   KRR_ORDER_PCA  first principal direction of the node by 32 power steps
 *                  v <- C v / max|C v| from v = (1, ..., 1), C the scatter
 *                  matrix about the node's mean point; left: projection <= the
 *                  mean projection.  An empty side or C v = 0: halves.
 * Means and scatter products are FP64 sums in chunks of 256 positions (in
 * order, then over chunks in order) with no fused multiply-add, so the result
 * is bit-for-bit deterministic.  KRR_ORDER_2MN runs krr_cluster_2mn. */
enum { KRR_ORDER_2MN = 0, KRR_ORDER_NP = 1, KRR_ORDER_KD = 2, KRR_ORDER_PCA = 3 };

/*
 * Ordering and cluster tree of X by `method` (KRR_ORDER_*); a forest when
 * offsets (host, np + 1 int64, offsets[0] = 0, increasing) is given, one tree
 * per problem, each equal to ordering that problem alone shifted by its
 * offset (offsets = NULL: one problem of n points, np ignored).
 *   X      n x d points (xprec), not modified
 *   opts   leaf_size as krr_cluster_2mn (max_iter, seed: 2MN only)
 *   perm   (out, n int64) perm[new position] = original index
 *   out    (out) tree handle; statistics (krr_tree_export): halves splits
 *          (NP not counted), KD median splits, 0, levels
 * Errors: KRR_E_INVAL for a bad method, sizes or NULL pointers.
 * Synchronizes `stream` once per tree level.
 */
int krr_cluster_order(const void *X, int32_t xprec, int64_t n, int32_t d, int32_t method,
                      const int64_t *offsets, int32_t np, const krr_cluster_opts *opts, void *stream,
                      int64_t *perm, krr_tree *out);

/* Builds a tree handle from a host node table (n_nodes rows of begin, end,
 * left, right, parent; postorder, children before parents, root last; leaves
 * have left = right = -1).  Lets any ordering (or a test) drive compression.
 * A forest (the batched form) lists its trees one after the other, each
 * ending at its root (parent = -1), the roots covering [0, n) in order. */
int krr_tree_from_host(const int64_t *nodes_host, int64_t n_nodes, krr_tree *out);

/* Number of points and of nodes of a tree. */
int krr_tree_size(krr_tree t, int64_t *n_host, int64_t *n_nodes_host);

/* Copies the node table (n_nodes x 5 int64, layout of krr_tree_from_host)
 * and the clustering statistics (4 int64: fallback splits, splits that hit
 * max_iter, Lloyd iterations, levels; zeros for a tree built from a table). */
int krr_tree_export(krr_tree t, int64_t *nodes_host, int64_t *stats_host);

void krr_tree_destroy(krr_tree t);

/* Roots of the trees of a forest (count_host: their number; roots_host, if
 * not NULL, receives that many node indices in order).  A single tree has
 * one root, its last node. */
int krr_tree_roots(krr_tree t, int64_t *roots_host, int32_t *count_host);

/* dst[i, :] = src[perm[i], :]  (rows of `cols` elements of dtype prec). */
int krr_gather_rows(const void *src, int32_t prec, int64_t n, int32_t cols,
                    const int64_t *perm, void *dst, void *stream);

/* dst[perm[i], :] = src[i, :]  (inverse of krr_gather_rows). */
int krr_scatter_rows(const void *src, int32_t prec, int64_t n, int32_t cols,
                     const int64_t *perm, void *dst, void *stream);

/* ----------------------------------------------------- kernel products */

/*
 * Out = K(X, Y; h) W + beta * Out  with the Gaussian kernel of eq. (1.1)
 * (Algorithm 1 step 3 for prediction; the residual of refinement).  K is
 * never stored.
 *   X    m x d points, Y  n x d points (both xprec)
 *   W    n x nrhs FP64,  Out  m x nrhs FP64 (read only if beta != 0)
 *   prec KRR_F64: FP64 throughout (exponents from exact coordinate
 *        differences for d <= 64; for d > 64 an FP64 matrix-core GEMM of the
 *        norm expansion on coordinates centred on the mean of Y).
 *        KRR_F32: kernel entries and products in FP32, sums over each column
 *        tile in FP32 and across tiles in FP64.  Exponents: for d <= 64 the
 *        FP64 norm expansion; for K(X, X) with one right-hand side (the
 *        symmetric form, KRR_TUNE_SYMMETRIC) FP32-accurate matrix-core
 *        exponents on coordinates re-centred per row block; for d > 64 a
 *        matrix-core GEMM of three-term BF16 splits (six cross products,
 *        FP32 accumulation: FP32-accurate) on coordinates centred on the
 *        mean of Y.
 *   1 <= nrhs <= 64.
 */
int kernel_matvec(const void *X, int64_t m, const void *Y, int64_t n, int32_t d,
                  int32_t xprec, double h, const double *W, int32_t nrhs, double beta,
                  double *Out, int32_t prec, void *stream);

/*
 * Negligible-tile map of the symmetric FP32 product (the products of the
 * refinement of Section 6, kept across a sequence of products with the same
 * points and width).  The first product through a map evaluates every entry
 * and records which 16-point tiles of the product's waves hold an entry of
 * at least 2^-32; later products evaluate only those tiles and leave out the
 * rest (every entry left out is below 2^-32).  A map is recorded again when
 * the address of X, n, d or h differs from its recording; the caller makes
 * a new map (or destroys this one) when the contents of X change at the same
 * address.  Applies to K(X, X) with FP32 points, d <= 31, one right-hand
 * side and the BF16 symmetric form (KRR_TUNE_SYMMETRIC 4); other products
 * evaluate every entry, and so do all products when KRR_TUNE_SYM_SKIP is 0.
 * The map's device memory belongs to the handle (4 bytes per 64 x 256
 * entries of K's upper triangle at d <= 9: 136 MB at n = 2^20).  Errors:
 * KRR_E_INVAL for NULL handles.
 */
typedef struct krr_tile_map_s *krr_tile_map_t;
int krr_tile_map_create(krr_tile_map_t *map_out);
int krr_tile_map_destroy(krr_tile_map_t map);

/* Out = K(X, X; h) W + beta * Out as kernel_matvec (X = Y, prec KRR_F32)
 * through a tile map (recording it when it does not match).  X n x d
 * (xprec), W and Out n x nrhs FP64.  Calls that share a map run one after
 * the other on one stream. */
int kernel_matvec_mapped(const void *X, int64_t n, int32_t d, int32_t xprec, double h,
                         const double *W, int32_t nrhs, double beta, double *Out,
                         krr_tile_map_t map, void *stream);

/* counts_host[0] = tiles the map marks for evaluation, [1] = tiles it covers,
 * [2] = kernel entries per tile (rows of a wave x 16 points); all 0 before a
 * recording.  The diagonal blocks of the symmetric form (all of their
 * entries) are not part of the map.  Synchronizes `stream`. */
int krr_tile_map_counts(krr_tile_map_t map, int64_t *counts_host, void *stream);

/*
 * Off-diagonal sampling product of the randomized HSS construction
 * (Section 3.1): S = K(X, X; h) R where row i skips the columns of its own
 * leaf [leaf_begin[i], leaf_end[i]) (pass both NULL for no masking).
 *   X  n x d points (xprec);  R  n x r FP32 random block (values exactly
 *   representable in the chosen precision, e.g. +-1);  S  n x r FP32 out
 *   (FP64 when prec == KRR_F64).  r must be a multiple of 32.
 *   prec: KRR_F64, KRR_F32, KRR_F16_SPLIT, KRR_BF16_SPLIT;
 *   split_terms: 1 or 2 terms of the kernel entries for the split modes.
 */
int kernel_sample(const void *X, int64_t n, int32_t d, int32_t xprec, double h,
                  const float *R, int32_t r, const int32_t *leaf_begin,
                  const int32_t *leaf_end, void *S, int32_t prec, int32_t split_terms,
                  void *stream);

/* The random block hss_compress draws: R[i, c] = +-1 from a counter-based
 * generator keyed by (seed, i, c0 + c); n x r FP32 out. */
int krr_random_block(uint64_t seed, int64_t n, int32_t r, int32_t c0, float *R,
                     void *stream);

/*
 * Backward of Out = K(X, Y; h) W for the upstream gradient G (m x nrhs):
 *   dW = K(X, Y)^T G                 (n x nrhs FP64)
 *   P  = K o (G W^T)  (formed on the fly, never stored)
 *   dX_i = -(1/h^2) [ (sum_j P_ij) x_i - (P Y)_i ]      (m x d FP64)
 *   dY_j =  (1/h^2) [ (P^T X)_j - (sum_i P_ij) y_j ]    (n x d FP64)
 *   dh   = sum_ij P_ij ||x_i - y_j||^2 / h^3            (1 FP64, device)
 * Any of dX, dY, dW, dh may be NULL.  W, G FP64; prec as for kernel_matvec.
 */
int kernel_matvec_bwd(const void *X, int64_t m, const void *Y, int64_t n, int32_t d,
                      int32_t xprec, double h, const double *W, const double *G,
                      int32_t nrhs, double *dX, double *dY, double *dW, double *dh,
                      int32_t prec, void *stream);

/* ------------------------------------------------- HSS compression (A3-A5) */

typedef struct {
    double rtol;         /* relative ID tolerance on the pivoted-QR diagonal */
    double atol;         /* absolute tolerance on |R_jj| / sqrt(r) (0 = off) */
    int32_t r0;          /* initial sample width (multiple of 32) */
    int32_t dr;          /* growth step of the sample width (multiple of 32) */
    int32_t r_max;       /* cap of the sample width */
    int32_t oversample;  /* p: ranks must stay <= r - p, else the sample grows */
    int32_t prec;        /* sampling arithmetic (KRR_F64 .. KRR_BF16_SPLIT) */
    int32_t split_terms; /* 1 or 2 for the split modes */
    int32_t cap_policy;  /* at r_max: 0 = fail with KRR_E_RANK_CAP, 1 = truncate ranks to r_max - p */
    uint64_t seed;       /* random block key */
} hss_opts;

typedef struct {
    int64_t n, n_nodes, levels;
    int32_t r_final;          /* sample width that revealed every rank */
    int32_t regrowths;        /* times the sample was widened */
    int32_t max_rank;
    int32_t truncated;        /* 1 if ranks were cut at r_max - oversample */
    int64_t bytes_paper;      /* memory metric: D, U, V, B_ij, B_ji as stored separately */
    int64_t bytes_stored;     /* generators actually stored (symmetric: U = V) */
    double t_sample_ms;       /* phase times (HIP events) */
    double t_id_ms;
    double t_total_ms;
} hss_stats;

/*
 * Randomized HSS compression of K(Xp, Xp; h) on the tree `t`
 * (Section 3.1; the randomized construction with adaptive sampling of
 * Section 1.1): S = K R with each leaf's own block removed; per tree level,
 * leaves take the interpolative decomposition (ID) of their sample rows,
 * parents of their children's skeleton rows minus the coupling B times the
 * sibling's reduced random block; D = K(I, I) at leaves and
 * B = K(J_left, J_right) at parents are extracted in FP64.  IDs, D and B are
 * FP64.  If some rank exceeds r - oversample the sample is widened by dr
 * (only the new columns are sampled) and the IDs are redone, up to r_max;
 * there, cap_policy 1 truncates every rank to r_max - oversample (recorded in
 * the statistics) instead of failing.
 *   Xp     n x d points in tree order (xprec)
 *   stats_host  optional (may be NULL)
 * Synchronizes `stream` once per level (ranks size the next level).
 */
int hss_compress(krr_tree t, const void *Xp, int32_t xprec, int32_t d, double h,
                 const hss_opts *opts, void *stream, hss_t *out, hss_stats *stats_host);

/* Frees the generators (waits for the device first: the storage may come
 * from a stream-ordered allocator). */
void hss_destroy(hss_t H);

/* y = K_hss x for n x nrhs FP64 blocks in the permuted order (the matrix the
 * generators represent, without lambda): upward pass through the nested
 * bases, coupling blocks, downward pass, dense leaf blocks. */
int hss_matvec(hss_t H, const double *x, int32_t nrhs, double *y, void *stream);

/* Sizes of the generator export: node count, FP64 values, int64 values. */
int hss_export_sizes(hss_t H, int64_t *n_nodes_host, int64_t *n_dbl_host,
                     int64_t *n_int_host);

/*
 * Copies the generators to the host.  table_host: n_nodes rows of 10 int64 =
 * (begin, end, left, right, m, k, off_U, off_D, off_B, off_J), offsets into
 * dbl_host / int_host, -1 where absent.  U is m x k (leaf: basis over the
 * leaf's points; non-leaf: transfer matrix over the children's skeletons),
 * D is (end-begin)^2 at leaves, B = K(J_left, J_right) at non-leaves, J the
 * k skeleton positions.  Synchronizes `stream`.
 */
int hss_export(hss_t H, int64_t *table_host, double *dbl_host, int64_t *int_host,
               void *stream);

/* ------------------------------------------------ ULV factor / solve (A6, A7) */

/*
 * ULV factorization of K_hss + lambda I (Section 3.1; lambda changes only the
 * leaf diagonal blocks, Section 5.3, so a new lambda needs no new compression).
 * Bottom-up per level: an orthogonal Q with Q^T U = [R; 0], D' = Q^T D Q,
 * Cholesky elimination of the rows outside U's range, the Schur complement on
 * the remaining k rows merged with the coupling blocks into the parent; dense
 * Cholesky at the root.  FP64.  Fails with KRR_E_NUMERIC on a non-positive
 * pivot.  Synchronizes `stream` once at the end (pivot check).
 */
int hss_ulv_factor(hss_t H, double lambda, void *stream, hss_ulv_t *out);

/*
 * As hss_ulv_factor, for use as a preconditioner.  In exact arithmetic every
 * Cholesky pivot of a Schur complement of K + lambda I is at least lambda; a
 * truncated compression can drive pivots of K_hss + lambda I below that (or
 * negative).  Here any pivot below pivot_floor (> 0; lambda / 2 is a good
 * choice) is raised to pivot_floor, which factors exactly the symmetric
 * positive definite matrix K_hss + lambda I + (node-local diagonal terms) in a
 * single pass.  clamped_host (optional) receives the number of raised pivots.
 */
int hss_ulv_factor_spd(hss_t H, double lambda, double pivot_floor, void *stream, hss_ulv_t *out,
                       int64_t *clamped_host);

/*
 * As hss_ulv_factor, for use as a preconditioner: factors K_hss + (lambda +
 * delta) I with every Cholesky pivot at least lambda / 2 (in exact arithmetic
 * every pivot of K + lambda I is at least lambda; truncated compression can
 * make K_hss + lambda I indefinite).  delta is found by a bracketed search:
 * 0; then the first of lambda, 4 lambda, 16 lambda, ... that covers the
 * largest deficit (lambda / 2 - pivot) seen, repeated until a try succeeds at
 * delta = hi; then hi / 8 and hi / 2 are tried and the first that succeeds
 * kept (a smaller shift is a better preconditioner; pivots of the Schur
 * complements grow faster than the shift, so hi overshoots).  A try stops at
 * the first level with a failing pivot.  The refinement still applies the
 * exact operator K + lambda I.  shift_host (optional) receives delta.
 * KRR_E_NUMERIC if no try succeeds (20 tries).
 */
int hss_ulv_factor_shifted(hss_t H, double lambda, void *stream, hss_ulv_t *out, double *shift_host);

/* Frees the factor and its solve plans (waits for the device first). */
void hss_ulv_destroy(hss_ulv_t F);

/* Graph replay of solves (default on): the first hss_solve with a given
 * nrhs builds a plan (sweep workspace and per-level descriptors on the
 * device) and captures its launches into a HIP graph; later solves copy B in,
 * replay the graph and copy the solution out, with no allocation, upload or
 * synchronization.  enable = 0 issues the same launches directly instead.
 * Either way a factor must not be used by two host threads at once. */
int hss_ulv_use_graph(hss_ulv_t F, int32_t enable);

/* Xout = (K_hss + lambda I)^{-1} B for n x nrhs FP64 B (permuted order).
 * B and Xout may alias.  The factor is symmetric, so it also solves the
 * transposed system. */
int hss_solve(hss_ulv_t F, const double *B, int32_t nrhs, double *Xout, void *stream);

/* --------------------------------------------------- refinement (A8) */

typedef struct {
    int32_t iterations;
    int32_t matvecs;
    double relres[64];   /* final true relative residual per right-hand side */
    double t_ms;
} krr_refine_stats;

/*
 * Preconditioned conjugate gradients on (K + lambda I) alpha = Y with the ULV
 * factor as preconditioner (F = NULL: no preconditioner) and kernel_matvec
 * (prec mv_prec) for the products;
 * the stopping test uses the recomputed true residual ||Y - (K + lambda I)
 * alpha|| / ||Y|| <= tol per column, formed with products of precision
 * res_prec; when the iteration's own residual has converged but the true one
 * has not, the iteration restarts from the true residual (res_prec = KRR_F64
 * with mv_prec = KRR_F32 is mixed-precision iterative refinement: FP32-entry
 * products inside, FP64 residuals outside).  alpha: in = start, out = solution
 * (n x nrhs FP64, permuted order).  Returns KRR_E_NOT_CONVERGED if max_iter
 * is reached first (alpha then holds the last iterate).  Synchronizes
 * `stream` once per iteration.
 */
int krr_refine(hss_ulv_t F, const void *Xp, int64_t n, int32_t xprec, int32_t d, double h,
               double lambda, const double *Y, int32_t nrhs, double *alpha, double tol,
               int32_t max_iter, int32_t mv_prec, int32_t res_prec, void *stream,
               krr_refine_stats *stats_host);

/* --------------------------------------------------- prediction (A9) */

/*
 * scores = K(Xt, Xp; h) alpha (m x nrhs FP64) and labels (m int32):
 * nrhs == 1: sign, zero counts as +1 (Algorithm 1 step 4);
 * nrhs > 1: index of the largest signed score, ties to the lowest (one-vs-all,
 * Section 2).  labels may be NULL.
 */
int krr_predict(const void *Xt, int64_t m, const void *Xp, int64_t n, int32_t d,
                int32_t xprec, double h, const double *alpha, int32_t nrhs,
                double *scores, int32_t *labels, int32_t prec, void *stream);

/* Scratch of krr_predict_noalloc per device: 128 MiB. */
#define KRR_NOALLOC_SCRATCH_BYTES (128u * 1024u * 1024u)

/*
 * krr_predict without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments and results as krr_predict (the same
 * kernels; identical scores) for d <= 64 and Xt != Xp; the split-K partial
 * sums and column data live in a static device array of
 * KRR_NOALLOC_SCRATCH_BYTES per device, held until the process ends.  It
 * needs 8 nsplit m nrhs bytes (nsplit, the column splits of the product, is
 * at most ceil(2048 / ceil(m / rows per workgroup)) with the default launch
 * knobs) plus, for prec = KRR_F32, n (8 LD + 4 nrhs) bytes, LD = D + 2 with D
 * the kernel width d is rounded up to (a multiple of 4 up to 24, then 32, 48,
 * 56 or 64), each part rounded up to 256 bytes; larger sizes fail with
 * KRR_E_INVAL (use krr_predict).  No hipMalloc, hipFree, memset or
 * stream synchronization.  Every call on a device shares its array: calls that
 * overlap on one device (two streams, two threads) race and must be ordered by
 * the caller.  Errors as krr_predict, plus KRR_E_INVAL for d > 64, Xt == Xp,
 * or a size over the limit.
 */
int krr_predict_noalloc(const void *Xt, int64_t m, const void *Xp, int64_t n, int32_t d, int32_t xprec,
                        double h, const double *alpha, int32_t nrhs, double *scores, int32_t *labels,
                        int32_t prec, void *stream);

/* ---------------------------------------------- batched form (A1-A8) */

/*
 * A batch is np independent KRR problems of equal dimension d stored one
 * after the other: problem k owns the points [offsets[k], offsets[k+1]) of a
 * single n x d array (offsets: host, np + 1 int64, offsets[0] = 0, every
 * problem non-empty, n = offsets[np]) and has its own kernel width h[k] and
 * ridge parameter lambda[k] (host arrays of np doubles).  The kernel matrix of
 * a batch is block diagonal; every batched call runs all problems together
 * (one launch per phase and tree level over every problem's nodes).  Problems
 * of different d form separate batches.
 */

/* 2MN clustering of every problem (the steps of krr_cluster_2mn, each
 * problem's tree started from its own range; each tree's result is identical
 * to clustering that problem alone, shifted by its offset).  perm (out, n
 * int64) keeps each problem within its range; out: a forest whose k-th tree
 * is problem k.  Synchronizes once per level and Lloyd iteration of the
 * whole forest. */
int krr_cluster_2mn_batched(const void *X, int32_t xprec, const int64_t *offsets, int32_t np,
                            int32_t d, const krr_cluster_opts *opts, void *stream, int64_t *perm,
                            krr_tree *out);

/* HSS compression of every problem of a forest (as hss_compress; h: host,
 * one width per tree).  One sampling launch covers every problem (each row
 * sums over its own problem's columns only); sample width, growth and rank
 * rule are shared.  Each tree's generators equal those of compressing that
 * problem alone with the same final sample width and random block rows. */
int hss_compress_batched(krr_tree t, const void *Xp, int32_t xprec, int32_t d, const double *h,
                         const hss_opts *opts, void *stream, hss_t *out, hss_stats *stats_host);

/* Number of problems (trees) of a compressed batch. */
int hss_num_problems(hss_t H, int32_t *np_host);

/* ULV factorization of every problem of a compressed batch with its own
 * lambda[k] (host, np doubles).  shifted = 0: as hss_ulv_factor.  shifted = 1:
 * as hss_ulv_factor_shifted, each problem with its own shift lambda[k] s_k
 * from its own search (a retry refactors only the problems still searching;
 * shift_mult_host, optional, host np doubles, receives every s_k, zeros when
 * shifted = 0).  Solve with
 * hss_solve (the factor is block diagonal over the problems). */
int hss_ulv_factor_batched(hss_t H, const double *lambda, int32_t shifted, void *stream,
                           hss_ulv_t *out, double *shift_mult_host);

/* kernel_sample on every problem of a batch in one launch: row i of
 * problem k gets sum over problem k's columns j outside [leaf_begin[i],
 * leaf_end[i]) of K(x_i, x_j; h[k]) R[j, :] (arguments as kernel_sample;
 * leaf ranges in global positions). */
int kernel_sample_batched(const void *X, int32_t xprec, const int64_t *offsets, int32_t np,
                          int32_t d, const double *h, const float *R, int32_t r,
                          const int32_t *leaf_begin, const int32_t *leaf_end, void *S,
                          int32_t prec, int32_t split_terms, void *stream);

/* Out = blockdiag_k K(X_k, X_k; h[k]) W (kernel_matvec on each problem's
 * own points; W, Out n x nrhs FP64; prec KRR_F32 or KRR_F64). */
int kernel_matvec_batched(const void *X, int32_t xprec, const int64_t *offsets, int32_t np,
                          int32_t d, const double *h, const double *W, int32_t nrhs, double *Out,
                          int32_t prec, void *stream);

/* krr_refine on every problem at once (one conjugate-gradient recurrence
 * per problem and right-hand side, sharing each launch).  F: a factor of the
 * same batch or NULL.  stats_host->relres holds, per right-hand side, the
 * largest over the problems; relres_host (optional, host np x nrhs) each
 * problem's own.  Converged when every problem meets tol. */
int krr_refine_batched(hss_ulv_t F, const void *Xp, int32_t xprec, const int64_t *offsets,
                       int32_t np, int32_t d, const double *h, const double *lambda,
                       const double *Y, int32_t nrhs, double *alpha, double tol,
                       int32_t max_iter, int32_t mv_prec, int32_t res_prec, void *stream,
                       krr_refine_stats *stats_host, double *relres_host);

/* ------------------------------------------------------------ tuning */

/* Launch-shape knobs of the hot kernels (process-wide; the autotuner in the
 * Python package sets them from its cache).  Values are validated; results
 * do not depend on them beyond floating-point summation order. */
enum {
    KRR_TUNE_SYMMETRIC = 0,  /* K(X, X) W evaluates each off-diagonal entry once (FP32 points, one
                                right-hand side; otherwise the vector form 2). Exponent engine:
                                4 (default) FP32-accurate exponents from three-term BF16 splits on the
                                matrix cores, re-centred per row block (d <= 31; else as 3);
                                3 FP32 exponents on the matrix cores, re-centred per row block;
                                1 FP64 exponents on the matrix cores; 2 FP64 exponents on the vector
                                ALUs; 0 off */
    KRR_TUNE_SAMPLE_RB = 1,  /* max 32-column blocks per sampling pass: 1, 2, 4 or 8 (default 8) */
    KRR_TUNE_MV_BLOCKS = 2,  /* workgroups the split-K kernel product aims for, 64..65536 (default 2048) */
    KRR_TUNE_SYM_CHUNK = 3,  /* columns per item of the symmetric product, multiple of 64 (default 16384;
                                halved for products too small to fill the chip) */
    KRR_TUNE_SAMPLE_SKIP = 4, /* 1: the matrix-core sampler skips 32 x 32 tiles whose entries are all below
                                 2^-32 (default); 0: every tile is evaluated */
    KRR_TUNE_SYM_SKIP = 5,    /* negligible tiles of the BF16 symmetric product (a wave's 16-point tile with
                                 every entry below 2^-32): 1 (default) the refinement's first product
                                 records them and its later products skip them; 2 as 1, and every other
                                 such product records, then skips them, in two passes; 0 every tile is
                                 evaluated */
    KRR_TUNE_COUNT = 6
};
int krr_set_tuning(int32_t knob, int32_t value);
int krr_get_tuning(int32_t knob, int32_t *value_host);

/* ------------------------------------------------ small vector kernels */

/* The validation mean squared error of a fit (the objective of the tuning of
 * h and lambda, Section 5.3) and the source of its adjoint system: for scores
 * f (m x k, K(X_v, X) alpha) and targets y_v (m x k), all FP64 device arrays,
 *   ge[i, c] = (2 / m) (f[i, c] - y_v[i, c])      (out, m x k)
 *   loss[c]  = sum_i (f[i, c] - y_v[i, c])^2 / m  (out, k, device)
 * summed in a fixed order (deterministic).  Errors: KRR_E_INVAL for m < 1,
 * k < 1 or NULL pointers. */
int krr_val_residual(const double *f, const double *yv, int64_t m, int32_t k, double *ge, double *loss,
                     void *stream);

/* The gradient of the validation loss in (log h, log lambda) from the adjoint
 * method's pieces, all device scalars: bta = beta^T alpha (beta the adjoint
 * solution), dh_v = (2 / m) e^T (dK_v/dh) alpha and dh_t = beta^T (dK/dh)
 * alpha (the dh outputs of kernel_matvec_bwd), gscale an optional upstream
 * factor (NULL: 1):
 *   out[0] = gscale h (dh_v - dh_t),   out[1] = -gscale lambda bta
 * (out: 2 FP64, device).  Errors: KRR_E_INVAL for NULL pointers or h, lambda
 * not positive. */
int krr_val_grad_finish(const double *bta, const double *dh_v, const double *dh_t, const double *gscale,
                        double h, double lambda, double *out, void *stream);

/* out[c] = sum_i a[i, c] * b[i, c] (n x k FP64, deterministic order; device out). */
int krr_dot_columns(const double *a, const double *b, int64_t n, int32_t k, double *out,
                    void *stream);

#ifdef __cplusplus
}
#endif

#endif /* KRR_H */
