/*
 * CPU FP64 oracle, C part.  TEST INFRASTRUCTURE ONLY: nothing in the product
 * library links, includes or calls this file.  It is built with plain gcc,
 * -O2 -ffp-contract=off, so every floating-point operation below is rounded
 * exactly as written (no fused multiply-add, no reassociation).
 *
 *   oracle_cluster2mn   recursive two-means ordering and cluster tree
 *                       (Section 4.2 steps 1-3, Section 4.3 "Recursive
 *                       two-means", tree numbered in postorder as in Fig. 3)
 *   oracle_order        the NP, KD and PCA orderings of Section 4.3 with
 *                       their cluster trees (readings at the function)
 *   oracle_seeds        the two seeds (and integer weights) the clustering
 *                       draws for one node, for the tests' distribution pins
 *   oracle_kmv          Out = K(X, Y; h) W, Gaussian kernel of eq. (1.1) formed
 *                       entry by entry from the difference x_i - y_j
 *   oracle_sample_masked  S = K(X, X; h) R with each row's own leaf block
 *                       removed, on a subset of rows: the off-diagonal sample a
 *                       leaf of the HSS tree needs (Section 3.1, randomized
 *                       construction)
 *
 * Readings where the paper is silent (all documented in the design notes):
 *   - a node is split while its size exceeds the leaf size;
 *   - first seed uniform over the node, second seed with probability
 *     proportional to the (Euclidean, not squared) distance from the first;
 *     both draws come from a counter-based generator keyed by
 *     (seed, node begin, node end, draw index) built from the SplitMix64
 *     finalizer (Steele, Lea, Flood, OOPSLA 2014);
 *   - the distance weights are made exact integers so that the draw does not
 *     depend on summation order: w_j = isqrt(floor(q_j * 2^(62 - e))) where
 *     q_j is the squared distance and 2^e bounds the node's largest q;
 *   - Lloyd iterations stop when no label changes, at most max_iter times;
 *     ties go to the first cluster;
 *   - centroids are summed in a fixed two-level order: consecutive chunks of
 *     256 node positions left to right, then the chunk partials left to right;
 *   - an empty cluster or all-equal points fall back to splitting the node
 *     into two halves by position (left half = floor(size / 2));
 *   - the split is stable: first-cluster points first, relative order kept.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ull
#define CHUNK 256

/* SplitMix64 output function applied to state x + golden gamma. */
static uint64_t sm_step(uint64_t x) {
    uint64_t z = x + GOLDEN;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t oracle_sm_step(uint64_t x) { return sm_step(x); }

uint64_t oracle_node_draw(uint64_t seed, int64_t b, int64_t e, uint64_t k) {
    uint64_t hsh = sm_step(seed);
    hsh = sm_step(hsh ^ (uint64_t)b);
    hsh = sm_step(hsh ^ (uint64_t)e);
    hsh = sm_step(hsh ^ k);
    return hsh;
}

static uint64_t mulhi64(uint64_t a, uint64_t b) {
    return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
}

/* floor(sqrt(v)) by the binary digit-by-digit method. */
uint64_t oracle_isqrt64(uint64_t v) {
    uint64_t res = 0, bit = 1ull << 62;
    while (bit > v) bit >>= 2;
    while (bit) {
        if (v >= res + bit) {
            v -= res + bit;
            res = (res >> 1) + bit;
        } else {
            res >>= 1;
        }
        bit >>= 2;
    }
    return res;
}

typedef struct {
    double *X;        /* n x d working copy, reordered as the recursion proceeds */
    int64_t *perm;    /* perm[pos] = original index */
    uint8_t *lab, *lab_new;
    double *tmp_row;  /* n x d scratch for the stable partition */
    int64_t *tmp_idx;
    double *q;
    uint64_t *w;
    int64_t n;
    int32_t d, leaf, max_iter;
    uint64_t seed;
    int64_t *nodes;   /* out: n_nodes x 5 (begin, end, left, right, parent) */
    int64_t n_nodes;
    int64_t fallbacks, capped, iterations;
    double *c0, *c1, *s0, *s1, *p0, *p1;
} ctx_t;

static double sqdist(const double *x, const double *c, int32_t d) {
    double acc = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        double t = x[k] - c[k];
        acc = acc + t * t;
    }
    return acc;
}

/* label 1 iff strictly closer to c1; returns number of label-1 points. */
static int64_t assign(ctx_t *C, int64_t b, int64_t e, uint8_t *out) {
    int64_t n1 = 0;
    for (int64_t p = b; p < e; ++p) {
        const double *x = C->X + p * C->d;
        double d0 = sqdist(x, C->c0, C->d);
        double d1 = sqdist(x, C->c1, C->d);
        out[p] = (d1 < d0) ? 1 : 0;
        n1 += out[p];
    }
    return n1;
}

static void centroids(ctx_t *C, int64_t b, int64_t e) {
    int32_t d = C->d;
    int64_t n0 = 0, n1 = 0;
    for (int32_t k = 0; k < d; ++k) { C->s0[k] = 0.0; C->s1[k] = 0.0; }
    for (int64_t cs = b; cs < e; cs += CHUNK) {
        int64_t ce = cs + CHUNK < e ? cs + CHUNK : e;
        for (int32_t k = 0; k < d; ++k) { C->p0[k] = 0.0; C->p1[k] = 0.0; }
        for (int64_t p = cs; p < ce; ++p) {
            const double *x = C->X + p * d;
            if (C->lab[p] == 0) {
                for (int32_t k = 0; k < d; ++k) C->p0[k] = C->p0[k] + x[k];
                ++n0;
            } else {
                for (int32_t k = 0; k < d; ++k) C->p1[k] = C->p1[k] + x[k];
                ++n1;
            }
        }
        for (int32_t k = 0; k < d; ++k) {
            C->s0[k] = C->s0[k] + C->p0[k];
            C->s1[k] = C->s1[k] + C->p1[k];
        }
    }
    for (int32_t k = 0; k < d; ++k) {
        C->c0[k] = C->s0[k] / (double)n0;
        C->c1[k] = C->s1[k] / (double)n1;
    }
}

/* The two seeds of a node [b, e) (Section 4.3 "Recursive two-means"): the
 * first uniform over the node, the second drawn with probability proportional
 * to its distance (not squared) from the first.  The integer weights
 * w_j = isqrt(floor(q_j 2^(62 - e))) are, up to the floor, the distances
 * |x_j - x_i1| scaled by 2^(31 - e/2), so the draw is exact and independent of
 * summation order.  Returns 0 with *i1, *i2 set, or -1 when every point of the
 * node equals the first seed (the fallback split applies). */
static int pick_seeds(ctx_t *C, int64_t b, int64_t e, int64_t *i1_out, int64_t *i2_out) {
    int32_t d = C->d;
    int64_t s = e - b;
    int64_t i1 = b + (int64_t)mulhi64(oracle_node_draw(C->seed, b, e, 0), (uint64_t)s);
    const double *x1 = C->X + i1 * d;
    double qmax = 0.0;
    for (int64_t p = b; p < e; ++p) {
        C->q[p] = sqdist(C->X + p * d, x1, d);
        if (C->q[p] > qmax) qmax = C->q[p];
    }
    *i1_out = i1;
    if (qmax == 0.0) return -1;
    int ex;
    frexp(qmax, &ex);
    int shift = 62 - ex;
    uint64_t W = 0;
    for (int64_t p = b; p < e; ++p) {
        double v = floor(ldexp(C->q[p], shift));
        C->w[p] = oracle_isqrt64((uint64_t)v);
        W += C->w[p];
    }
    if (W == 0) return -1;
    uint64_t u = mulhi64(oracle_node_draw(C->seed, b, e, 1), W);
    uint64_t acc = 0;
    int64_t i2 = e - 1;
    for (int64_t p = b; p < e; ++p) {
        acc += C->w[p];
        if (acc > u) { i2 = p; break; }
    }
    *i2_out = i2;
    return 0;
}

/* Returns the size of the left part, or -1 when the fallback split applies. */
static int64_t two_means(ctx_t *C, int64_t b, int64_t e) {
    int32_t d = C->d;
    int64_t s = e - b;
    int64_t i1, i2;
    if (pick_seeds(C, b, e, &i1, &i2) < 0) return -1;
    memcpy(C->c0, C->X + i1 * d, sizeof(double) * d);
    memcpy(C->c1, C->X + i2 * d, sizeof(double) * d);
    int64_t n1 = assign(C, b, e, C->lab);
    if (n1 == 0 || n1 == s) return -1;
    int it = 0;
    for (; it < C->max_iter; ++it) {
        centroids(C, b, e);
        n1 = assign(C, b, e, C->lab_new);
        C->iterations++;
        int changed = 0;
        for (int64_t p = b; p < e; ++p) changed |= (C->lab_new[p] != C->lab[p]);
        memcpy(C->lab + b, C->lab_new + b, (size_t)s);
        if (n1 == 0 || n1 == s) return -1;
        if (!changed) break;
    }
    if (it == C->max_iter) C->capped++;
    return s - n1;
}

static void stable_partition(ctx_t *C, int64_t b, int64_t e) {
    int32_t d = C->d;
    int64_t o = b;
    for (int pass = 0; pass < 2; ++pass)
        for (int64_t p = b; p < e; ++p)
            if (C->lab[p] == pass) {
                memcpy(C->tmp_row + o * d, C->X + p * d, sizeof(double) * d);
                C->tmp_idx[o] = C->perm[p];
                ++o;
            }
    memcpy(C->X + b * d, C->tmp_row + b * d, sizeof(double) * d * (e - b));
    memcpy(C->perm + b, C->tmp_idx + b, sizeof(int64_t) * (e - b));
}

static int64_t build(ctx_t *C, int64_t b, int64_t e) {
    int64_t s = e - b, left = -1, right = -1;
    if (s > C->leaf) {
        int64_t nl = two_means(C, b, e);
        if (nl < 0) {
            C->fallbacks++;
            nl = s / 2;
        } else {
            stable_partition(C, b, e);
        }
        left = build(C, b, b + nl);
        right = build(C, b + nl, e);
    }
    int64_t id = C->n_nodes++;
    int64_t *row = C->nodes + 5 * id;
    row[0] = b; row[1] = e; row[2] = left; row[3] = right; row[4] = -1;
    if (left >= 0) { C->nodes[5 * left + 4] = id; C->nodes[5 * right + 4] = id; }
    return id;
}

/*
 * X: n x d FP64 points (exact promotions of the caller's data), not modified.
 * perm (out, n): perm[new position] = original index.
 * nodes (out, capacity >= 2n - 1 rows of 5): postorder node table.
 * stats (out, 3): fallback splits, nodes that hit max_iter, Lloyd iterations.
 * Returns the node count, or -1 on allocation failure.
 */
int64_t oracle_cluster2mn(const double *X, int64_t n, int32_t d, int32_t leaf,
                          int32_t max_iter, uint64_t seed, int64_t *perm,
                          int64_t *nodes, int64_t *stats) {
    ctx_t C;
    memset(&C, 0, sizeof C);
    C.n = n; C.d = d; C.leaf = leaf < 1 ? 1 : leaf; C.max_iter = max_iter; C.seed = seed;
    C.X = malloc(sizeof(double) * n * d);
    C.tmp_row = malloc(sizeof(double) * n * d);
    C.tmp_idx = malloc(sizeof(int64_t) * n);
    C.lab = malloc(n); C.lab_new = malloc(n);
    C.q = malloc(sizeof(double) * n);
    C.w = malloc(sizeof(uint64_t) * n);
    double *cbuf = malloc(sizeof(double) * 6 * d);
    if (!C.X || !C.tmp_row || !C.tmp_idx || !C.lab || !C.lab_new || !C.q || !C.w || !cbuf) {
        free(C.X); free(C.tmp_row); free(C.tmp_idx); free(C.lab); free(C.lab_new);
        free(C.q); free(C.w); free(cbuf);
        return -1;
    }
    C.c0 = cbuf; C.c1 = cbuf + d; C.s0 = cbuf + 2 * d; C.s1 = cbuf + 3 * d;
    C.p0 = cbuf + 4 * d; C.p1 = cbuf + 5 * d;
    memcpy(C.X, X, sizeof(double) * n * d);
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    C.perm = perm;
    C.nodes = nodes;
    if (n > 0) build(&C, 0, n);
    stats[0] = C.fallbacks; stats[1] = C.capped; stats[2] = C.iterations;
    free(C.X); free(C.tmp_row); free(C.tmp_idx); free(C.lab); free(C.lab_new);
    free(C.q); free(C.w); free(cbuf);
    return C.n_nodes;
}

/* ------------------------------------------------------------------------
 * The other orderings of Section 4.3 ("Selected Preprocessing Methods"),
 * each a recursive split of [b, e) while its size exceeds the leaf size, the
 * left part first, the split stable (relative order kept), the tree numbered
 * in postorder.  Readings where the paper is silent:
 *   NP   no reordering: the left part is the first floor(size / 2) positions.
 *   KD   the coordinate of maximum spread (max - min over the node, lowest
 *        index on ties); its mean (chunked sum as the 2MN centroids, divided
 *        by the size); left = points with coordinate <= mean.  When
 *        100 * min(left, right) < max(left, right) (the paper's imbalance
 *        test, applied to either side) the split falls back to the median:
 *        the left part is the floor(size / 2) points first in the order of
 *        (coordinate, position).  Zero spread splits into halves.
 *   PCA  mean point mu (chunked sums); the first principal direction v by
 *        PCA_ITERS power iterations v <- C v / |C v| with C the (unscaled)
 *        scatter matrix of the node, applied as sum_j (x_j - mu) t_j with
 *        t_j = (x_j - mu) . v, from v0 = (1, ..., 1), each step scaled by
 *        its largest |component| (max norm, so no square root); projections
 *        p_j = (x_j - mu) . v and their chunked mean m; left = p_j <= m.
 *        An empty side or C v = 0 splits into halves.
 * Every sum runs in the written order with no fused multiply-add.
 * ---------------------------------------------------------------------- */
#define PCA_ITERS 32
enum { ORDER_NP = 1, ORDER_KD = 2, ORDER_PCA = 3 };

typedef struct {
    ctx_t *C;
    int method;
    double *mu, *v, *wv, *acc, *key;
    int64_t median_splits;
} octx_t;

/* sum over positions [b, e) of f(p) in the fixed chunked order */
static double chunked_sum(const double *val, int64_t b, int64_t e) {
    double s = 0.0;
    for (int64_t cs = b; cs < e; cs += CHUNK) {
        int64_t ce = cs + CHUNK < e ? cs + CHUNK : e;
        double part = 0.0;
        for (int64_t p = cs; p < ce; ++p) part = part + val[p];
        s = s + part;
    }
    return s;
}

static int cmp_key_pos(const void *a, const void *b, const double *key) {
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    if (key[i] < key[j]) return -1;
    if (key[i] > key[j]) return 1;
    return (i > j) - (i < j);
}

static const double *g_sort_key;
static int cmp_idx(const void *a, const void *b) { return cmp_key_pos(a, b, g_sort_key); }

/* Labels for a KD split of [b, e): 0 = left.  Returns the left size, or -1
 * for the halves fallback. */
static int64_t kd_labels(octx_t *O, int64_t b, int64_t e) {
    ctx_t *C = O->C;
    int32_t d = C->d;
    int64_t s = e - b;
    int32_t kbest = 0;
    double best = -1.0;
    for (int32_t k = 0; k < d; ++k) {
        double lo = C->X[b * d + k], hi = lo;
        for (int64_t p = b; p < e; ++p) {
            double v = C->X[p * d + k];
            if (v < lo) lo = v;
            if (v > hi) hi = v;
        }
        double spread = hi - lo;
        if (spread > best) { best = spread; kbest = k; }
    }
    if (!(best > 0.0)) return -1;
    for (int64_t p = b; p < e; ++p) O->key[p] = C->X[p * d + kbest] + 0.0;  /* -0 becomes +0 */
    double mean = chunked_sum(O->key, b, e) / (double)s;
    int64_t n0 = 0;
    for (int64_t p = b; p < e; ++p) {
        C->lab[p] = O->key[p] <= mean ? 0 : 1;
        n0 += C->lab[p] == 0;
    }
    int64_t n1 = s - n0;
    int64_t mn = n0 < n1 ? n0 : n1, mx = n0 < n1 ? n1 : n0;
    if (100 * mn < mx) {
        /* median: the floor(s / 2) first points in (key, position) order */
        int64_t *idx = C->tmp_idx + b;  /* scratch, restored by the partition */
        for (int64_t p = b; p < e; ++p) idx[p - b] = p;
        g_sort_key = O->key;
        qsort(idx, (size_t)s, sizeof(int64_t), cmp_idx);
        for (int64_t r = 0; r < s; ++r) C->lab[idx[r]] = r < s / 2 ? 0 : 1;
        n0 = s / 2;
        O->median_splits++;
    }
    return n0;
}

/* Labels for a PCA split of [b, e); returns the left size or -1. */
static int64_t pca_labels(octx_t *O, int64_t b, int64_t e) {
    ctx_t *C = O->C;
    int32_t d = C->d;
    int64_t s = e - b;
    double *col = O->key;
    for (int32_t k = 0; k < d; ++k) {
        for (int64_t p = b; p < e; ++p) col[p] = C->X[p * d + k];
        O->mu[k] = chunked_sum(col, b, e) / (double)s;
    }
    for (int32_t k = 0; k < d; ++k) O->v[k] = 1.0;
    for (int it = 0; it < PCA_ITERS; ++it) {
        for (int64_t p = b; p < e; ++p) {
            double t = 0.0;
            for (int32_t k = 0; k < d; ++k) t = t + (C->X[p * d + k] - O->mu[k]) * O->v[k];
            C->q[p] = t;
        }
        for (int32_t k = 0; k < d; ++k) {
            for (int64_t p = b; p < e; ++p) col[p] = (C->X[p * d + k] - O->mu[k]) * C->q[p];
            O->wv[k] = chunked_sum(col, b, e);
        }
        double nrm = 0.0;
        for (int32_t k = 0; k < d; ++k)
            if (fabs(O->wv[k]) > nrm) nrm = fabs(O->wv[k]);
        if (!(nrm > 0.0)) return -1;
        for (int32_t k = 0; k < d; ++k) O->v[k] = O->wv[k] / nrm;
    }
    for (int64_t p = b; p < e; ++p) {
        double t = 0.0;
        for (int32_t k = 0; k < d; ++k) t = t + (C->X[p * d + k] - O->mu[k]) * O->v[k];
        C->q[p] = t;
    }
    double m = chunked_sum(C->q, b, e) / (double)s;
    int64_t n0 = 0;
    for (int64_t p = b; p < e; ++p) {
        C->lab[p] = C->q[p] <= m ? 0 : 1;
        n0 += C->lab[p] == 0;
    }
    if (n0 == 0 || n0 == s) return -1;
    return n0;
}

static int64_t build_order(octx_t *O, int64_t b, int64_t e) {
    ctx_t *C = O->C;
    int64_t s = e - b, left = -1, right = -1;
    if (s > C->leaf) {
        int64_t nl = -1;
        if (O->method == ORDER_KD) nl = kd_labels(O, b, e);
        else if (O->method == ORDER_PCA) nl = pca_labels(O, b, e);
        if (nl < 0) {
            if (O->method != ORDER_NP) C->fallbacks++;
            nl = s / 2;
        } else {
            stable_partition(C, b, e);
        }
        left = build_order(O, b, b + nl);
        right = build_order(O, b + nl, e);
    }
    int64_t id = C->n_nodes++;
    int64_t *row = C->nodes + 5 * id;
    row[0] = b; row[1] = e; row[2] = left; row[3] = right; row[4] = -1;
    if (left >= 0) { C->nodes[5 * left + 4] = id; C->nodes[5 * right + 4] = id; }
    return id;
}

/*
 * NP / KD / PCA ordering of X (n x d FP64) with the tree in postorder.
 * method: 1 NP, 2 KD, 3 PCA.  perm, nodes as oracle_cluster2mn.
 * stats (out, 2): fallback (halves) splits, median splits (KD).
 * Returns the node count, -1 on allocation failure, -2 on a bad method.
 */
int64_t oracle_order(const double *X, int64_t n, int32_t d, int32_t leaf, int32_t method,
                     int64_t *perm, int64_t *nodes, int64_t *stats) {
    if (method < ORDER_NP || method > ORDER_PCA) return -2;
    ctx_t C;
    octx_t O;
    memset(&C, 0, sizeof C);
    memset(&O, 0, sizeof O);
    C.n = n; C.d = d; C.leaf = leaf < 1 ? 1 : leaf;
    C.X = malloc(sizeof(double) * n * d);
    C.tmp_row = malloc(sizeof(double) * n * d);
    C.tmp_idx = malloc(sizeof(int64_t) * n);
    C.lab = malloc(n);
    C.q = malloc(sizeof(double) * n);
    O.key = malloc(sizeof(double) * n);
    double *dbuf = malloc(sizeof(double) * 4 * d);
    if (!C.X || !C.tmp_row || !C.tmp_idx || !C.lab || !C.q || !O.key || !dbuf) {
        free(C.X); free(C.tmp_row); free(C.tmp_idx); free(C.lab); free(C.q); free(O.key); free(dbuf);
        return -1;
    }
    O.C = &C; O.method = method;
    O.mu = dbuf; O.v = dbuf + d; O.wv = dbuf + 2 * d; O.acc = dbuf + 3 * d;
    memcpy(C.X, X, sizeof(double) * n * d);
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    C.perm = perm;
    C.nodes = nodes;
    if (n > 0) build_order(&O, 0, n);
    stats[0] = C.fallbacks; stats[1] = O.median_splits;
    free(C.X); free(C.tmp_row); free(C.tmp_idx); free(C.lab); free(C.q); free(O.key); free(dbuf);
    return C.n_nodes;
}

/*
 * The seed pick of one node [b, e) of X (n x d FP64) under `seed`, exposed so
 * that tests observe the draw the clustering actually makes.
 * seeds (out, 2): i1, i2 (i2 = -1 when the fallback split applies).
 * weights (out, optional, n): the integer weights w_j at positions [b, e).
 * Returns 0, -1 on invalid arguments, -2 on allocation failure.
 */
int oracle_seeds(const double *X, int64_t n, int32_t d, int64_t b, int64_t e,
                 uint64_t seed, int64_t *seeds, uint64_t *weights) {
    if (b < 0 || e > n || e - b < 1 || d < 1) return -1;
    ctx_t C;
    memset(&C, 0, sizeof C);
    C.n = n; C.d = d; C.seed = seed;
    C.X = (double *)X;
    C.q = malloc(sizeof(double) * n);
    C.w = calloc((size_t)n, sizeof(uint64_t));
    if (!C.q || !C.w) { free(C.q); free(C.w); return -2; }
    int64_t i1 = -1, i2 = -1;
    if (pick_seeds(&C, b, e, &i1, &i2) < 0) i2 = -1;
    seeds[0] = i1; seeds[1] = i2;
    if (weights) memcpy(weights + b, C.w + b, sizeof(uint64_t) * (size_t)(e - b));
    free(C.q); free(C.w);
    return 0;
}

/* Out[i, c] = sum_j exp(-||x_i - y_j||^2 / (2 h^2)) W[j, c], all FP64.
 * rows (optional, length m_sel): compute only these rows of X; Out is then
 * m_sel x nrhs.  Pass rows = NULL and m_sel = m for all rows. */
void oracle_kmv(const double *X, const double *Y, int64_t n, int32_t d, double h,
                const double *W, int32_t nrhs, const int64_t *rows, int64_t m_sel,
                double *Out) {
    double inv = 1.0 / (2.0 * h * h);
#pragma omp parallel
    {
        double *acc = malloc(sizeof(double) * (size_t)nrhs);
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < m_sel; ++t) {
            int64_t i = rows ? rows[t] : t;
            const double *x = X + i * d;
            for (int32_t c = 0; c < nrhs; ++c) acc[c] = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                double q = sqdist(x, Y + j * d, d);
                double kij = exp(-q * inv);
                const double *w = W + j * nrhs;
                for (int32_t c = 0; c < nrhs; ++c) acc[c] = acc[c] + kij * w[c];
            }
            for (int32_t c = 0; c < nrhs; ++c) Out[t * nrhs + c] = acc[c];
        }
        free(acc);
    }
}

/* Off-diagonal sample rows: S[t, c] = sum_{j outside [lb[i], le[i])} K(x_i, x_j) R[j, c]
 * for i = rows[t].  lb / le give, per point, the range of its own leaf. */
void oracle_sample_masked(const double *X, int64_t n, int32_t d, double h,
                          const double *R, int32_t r, const int64_t *lb,
                          const int64_t *le, const int64_t *rows, int64_t m_sel,
                          double *Out) {
    double inv = 1.0 / (2.0 * h * h);
#pragma omp parallel
    {
        double *acc = malloc(sizeof(double) * (size_t)r);
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < m_sel; ++t) {
            int64_t i = rows[t];
            const double *x = X + i * d;
            for (int32_t c = 0; c < r; ++c) acc[c] = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                if (j >= lb[i] && j < le[i]) continue;
                double q = sqdist(x, X + j * d, d);
                double kij = exp(-q * inv);
                const double *w = R + j * r;
                for (int32_t c = 0; c < r; ++c) acc[c] = acc[c] + kij * w[c];
            }
            for (int32_t c = 0; c < r; ++c) Out[t * r + c] = acc[c];
        }
        free(acc);
    }
}
