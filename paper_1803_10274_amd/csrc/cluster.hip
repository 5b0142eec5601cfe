// Recursive two-means (2MN) ordering on the GPU (Section 4.2 steps 1-3,
// Section 4.3 "Recursive two-means"), level-synchronous: every node of a tree
// level that is larger than the leaf size is split by the same launches.
//
// The split is specified down to the last bit so that it does not depend on
// how the work is scheduled:
//   * first seed  i1 = b + mulhi(draw(seed, b, e, 0), size);
//   * second seed drawn with probability proportional to the Euclidean
//     distance from the first seed, with exact integer weights
//     w_j = isqrt(floor(q_j * 2^(62 - ex))), q_j the FP64 squared distance and
//     2^ex > max q; u = mulhi(draw(seed, b, e, 1), sum w); i2 = first position
//     whose inclusive prefix sum of w exceeds u;
//   * Lloyd iterations: label 1 iff strictly closer to the second center
//     (FP64, coordinates summed in order, no fused multiply-add); centers are
//     sums over consecutive 256-position chunks (in order), then over chunks
//     (in order), divided by the count; stop when no label changes, at most
//     max_iter iterations;
//   * empty cluster / all-equal points: split in halves by position;
//   * stable partition, first cluster first.
// draw() chains four SplitMix64 output steps over (seed, b, e, k).
//
// The same driver builds the other orderings the paper compares (Section 4.3,
// "Selected Preprocessing Methods"), with the same stable partition and tree:
//   * NP: no reordering, halves by position;
//   * KD: coordinate of maximum spread (max - min, lowest index on ties), split
//     at its mean (chunked sum as the centroids), left = coordinate <= mean;
//     if 100 min(left, right) < max(left, right), the floor(size / 2) points
//     first in (coordinate, position) order go left (median), found by an
//     8-pass radix select on the order-preserving bit pattern of the key;
//     zero spread splits in halves;
//   * PCA: mean point mu, 32 power steps v <- C v / max|C v| from v = 1 with
//     C v = sum_j (x_j - mu) ((x_j - mu) . v) (chunked sums), projections
//     p_j = (x_j - mu) . v, left = p_j <= their chunked mean; an empty side or
//     C v = 0 splits in halves.
#include "internal.hpp"

// This file is compiled with -ffp-contract=off; the pragma keeps it so even if
// the flag is dropped.
#pragma clang fp contract(off)

namespace krr {
namespace {

constexpr int CH = 256;  // positions per chunk (also the block size of point kernels)
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
enum : int32_t { ACTIVE = 0, CONVERGED = 1, FALLBACK = 2, MEDIAN = 3 };
constexpr int PCA_ITERS = 32;

uint64_t sm_out(uint64_t x) {
    uint64_t z = x + kGamma;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t node_draw(uint64_t seed, int64_t b, int64_t e, uint64_t k) {
    uint64_t v = sm_out(seed);
    v = sm_out(v ^ (uint64_t)b);
    v = sm_out(v ^ (uint64_t)e);
    return sm_out(v ^ k);
}

uint64_t mulhi_u64(uint64_t a, uint64_t b) {
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
}

__device__ __forceinline__ uint64_t isqrt_u64(uint64_t v) {
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

template <class T>
__device__ __forceinline__ double sqdist_c(const T *x, const double *c, int d) {
    double acc = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = (double)x[k] - c[k];
        acc = acc + t * t;
    }
    return acc;
}

template <class T>
__device__ __forceinline__ double sqdist_p(const T *x, const T *y, int d) {
    double acc = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = (double)x[k] - (double)y[k];
        acc = acc + t * t;
    }
    return acc;
}

struct Level {
    // per active node
    const int64_t *nb, *ne, *i1;
    const uint64_t *draw1;
    const int32_t *ch0, *nch;
    int64_t *i2, *n1;
    uint64_t *qmax, *W;
    int32_t *status, *changed, *iters;
    double *c0, *c1;
    int64_t *off0, *off1;
    // per chunk
    const int32_t *cnode;
    const int64_t *cb, *ce;
    uint64_t *cw;
    int32_t *cn1;
    double *cps;
    int32_t *n_active;
    // orderings
    int32_t *kstar;
    double *nmean, *c2;
    uint64_t *pfx;
    int64_t *krem, *cless;
    int32_t *hist;
};

template <class T>
__global__ void k_q(const T *__restrict__ X, int d, Level L, double *__restrict__ q) {
    int c = blockIdx.x;
    int node = L.cnode[c];
    int64_t p = L.cb[c] + threadIdx.x;
    uint64_t bits = 0;
    if (p < L.ce[c]) {
        double v = sqdist_p(X + p * d, X + L.i1[node] * d, d);
        q[p] = v;
        bits = (uint64_t)__double_as_longlong(v);
    }
    bits = wave_max(bits);
    if ((threadIdx.x & 63) == 0 && bits) atomicMax((unsigned long long *)&L.qmax[node], (unsigned long long)bits);
}

__global__ void k_w(Level L, const double *__restrict__ q, uint64_t *__restrict__ w) {
    __shared__ uint64_t part[CH / 64];
    int c = blockIdx.x;
    int node = L.cnode[c];
    int64_t p = L.cb[c] + threadIdx.x;
    double qm = __longlong_as_double((long long)L.qmax[node]);
    uint64_t wv = 0;
    if (p < L.ce[c] && qm > 0.0) {
        int ex;
        frexp(qm, &ex);
        double v = floor(ldexp(q[p], 62 - ex));
        wv = isqrt_u64((uint64_t)v);
    }
    if (p < L.ce[c]) w[p] = wv;
    uint64_t s = wave_sum(wv);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int i = 0; i < CH / 64; ++i) t += part[i];
        L.cw[c] = t;
        if (t) atomicAdd((unsigned long long *)&L.W[node], (unsigned long long)t);
    }
}

__global__ void k_pick(Level L, int na, const uint64_t *__restrict__ w) {
    int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= na) return;
    uint64_t W = L.W[node];
    if (W == 0) {
        L.status[node] = FALLBACK;
        return;
    }
    uint64_t u = __umul64hi(L.draw1[node], W);
    uint64_t acc = 0;
    int c = L.ch0[node], cend = L.ch0[node] + L.nch[node];
    for (; c < cend - 1; ++c) {
        if (acc + L.cw[c] > u) break;
        acc += L.cw[c];
    }
    int64_t i2 = L.ce[c] - 1;
    for (int64_t p = L.cb[c]; p < L.ce[c]; ++p) {
        acc += w[p];
        if (acc > u) {
            i2 = p;
            break;
        }
    }
    L.i2[node] = i2;
}

template <class T>
__global__ void k_seed_centers(const T *__restrict__ X, int d, int na, Level L) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)na * d) return;
    int node = (int)(t / d), k = (int)(t % d);
    if (L.status[node] != ACTIVE) return;
    L.c0[t] = (double)X[L.i1[node] * d + k];
    L.c1[t] = (double)X[L.i2[node] * d + k];
}

template <class T>
__global__ void k_assign(const T *__restrict__ X, int d, Level L, uint8_t *__restrict__ lab, int first) {
    __shared__ int part[CH / 64];
    __shared__ int chg[CH / 64];
    int c = blockIdx.x;
    int node = L.cnode[c];
    if (L.status[node] != ACTIVE) return;
    int64_t p = L.cb[c] + threadIdx.x;
    int one = 0, changed = 0;
    if (p < L.ce[c]) {
        const T *x = X + p * d;
        double d0 = sqdist_c(x, L.c0 + (int64_t)node * d, d);
        double d1 = sqdist_c(x, L.c1 + (int64_t)node * d, d);
        uint8_t lb = (d1 < d0) ? 1 : 0;
        if (!first) changed = (lab[p] != lb);
        lab[p] = lb;
        one = lb;
    }
    int s = wave_sum(one);
    int ch = wave_sum(changed);
    if ((threadIdx.x & 63) == 0) {
        part[threadIdx.x >> 6] = s;
        chg[threadIdx.x >> 6] = ch;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0, u = 0;
        for (int i = 0; i < CH / 64; ++i) {
            t += part[i];
            u += chg[i];
        }
        L.cn1[c] = t;
        if (u) atomicOr(&L.changed[node], 1);
    }
}

__global__ void k_node_update(Level L, int na, int first) {
    int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= na || L.status[node] != ACTIVE) return;
    int64_t n1 = 0;
    const int ce = L.ch0[node] + L.nch[node];
    int c = L.ch0[node];
    for (; c + 8 <= ce; c += 8) {  // eight loads in flight
        int32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = L.cn1[c + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) n1 += v[u];
    }
    for (; c < ce; ++c) n1 += L.cn1[c];
    int64_t s = L.ne[node] - L.nb[node];
    L.n1[node] = n1;
    if (!first) L.iters[node] += 1;
    if (n1 == 0 || n1 == s) {
        L.status[node] = FALLBACK;
    } else if (!first && !L.changed[node]) {
        L.status[node] = CONVERGED;
    } else {
        atomicAdd(L.n_active, 1);
    }
    L.changed[node] = 0;
}

template <class T>
__global__ void k_centroid_partial(const T *__restrict__ X, int d, int nc, Level L,
                                   const uint8_t *__restrict__ lab) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nc * d) return;
    int c = (int)(t / d), k = (int)(t % d);
    if (L.status[L.cnode[c]] != ACTIVE) return;
    double p0 = 0.0, p1 = 0.0;
    // the loads of eight points are issued together, the sums still run
    // point by point in order (the result is the sequential sum)
    const int64_t pe = L.ce[c];
    int64_t p = L.cb[c];
    for (; p + 8 <= pe; p += 8) {
        double v[8];
        uint8_t lb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            v[u] = (double)X[(p + u) * d + k];
            lb[u] = lab[p + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (lb[u] == 0)
                p0 = p0 + v[u];
            else
                p1 = p1 + v[u];
        }
    }
    for (; p < pe; ++p) {
        double v = (double)X[p * d + k];
        if (lab[p] == 0)
            p0 = p0 + v;
        else
            p1 = p1 + v;
    }
    L.cps[2 * t] = p0;
    L.cps[2 * t + 1] = p1;
}

__global__ void k_centroid_final(int d, int na, Level L) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)na * d) return;
    int node = (int)(t / d), k = (int)(t % d);
    if (L.status[node] != ACTIVE) return;
    double s0 = 0.0, s1 = 0.0;
    // chunks in order, their loads eight at a time
    const int ce = L.ch0[node] + L.nch[node];
    int c = L.ch0[node];
    for (; c + 8 <= ce; c += 8) {
        double a0[8], a1[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            a0[u] = L.cps[2 * ((int64_t)(c + u) * d + k)];
            a1[u] = L.cps[2 * ((int64_t)(c + u) * d + k) + 1];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            s0 = s0 + a0[u];
            s1 = s1 + a1[u];
        }
    }
    for (; c < ce; ++c) {
        s0 = s0 + L.cps[2 * ((int64_t)c * d + k)];
        s1 = s1 + L.cps[2 * ((int64_t)c * d + k) + 1];
    }
    int64_t n1 = L.n1[node];
    int64_t n0 = (L.ne[node] - L.nb[node]) - n1;
    L.c0[t] = s0 / (double)n0;
    L.c1[t] = s1 / (double)n1;
}

__global__ void k_part_prefix(Level L, int na) {
    int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= na || L.status[node] == FALLBACK) return;
    int64_t o0 = 0, o1 = 0;
    for (int c = L.ch0[node]; c < L.ch0[node] + L.nch[node]; ++c) {
        L.off0[c] = o0;
        L.off1[c] = o1;
        int64_t sz = L.ce[c] - L.cb[c];
        o0 += sz - L.cn1[c];
        o1 += L.cn1[c];
    }
}

__global__ void k_iota(int64_t n, int64_t *__restrict__ dest) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) dest[p] = p;
}

__global__ void k_part_dest(Level L, const uint8_t *__restrict__ lab, int64_t *__restrict__ dest) {
    __shared__ int wz[CH / 64];
    int c = blockIdx.x;
    int node = L.cnode[c];
    if (L.status[node] == FALLBACK) return;
    int64_t p = L.cb[c] + threadIdx.x;
    bool valid = p < L.ce[c];
    int isz = valid && lab[p] == 0;
    uint64_t mask = __ballot(isz);
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    int before_in_wave = __popcll(mask & lt);
    if (lane == 0) wz[wv] = __popcll(mask);
    __syncthreads();
    int before = before_in_wave;
    for (int i = 0; i < wv; ++i) before += wz[i];
    if (!valid) return;
    int64_t nb = L.nb[node];
    int64_t n0 = (L.ne[node] - nb) - L.n1[node];
    int64_t pos_in_chunk = threadIdx.x;
    if (isz)
        dest[p] = nb + L.off0[c] + before;
    else
        dest[p] = nb + n0 + L.off1[c] + (pos_in_chunk - before);
}

template <class T>
__global__ void k_move(const T *__restrict__ X, const int64_t *__restrict__ perm, int64_t n, int d,
                       const int64_t *__restrict__ dest, T *__restrict__ Xo, int64_t *__restrict__ permo) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * d) return;
    int64_t p = t / d;
    int k = (int)(t % d);
    int64_t q = dest[p];
    Xo[q * d + k] = X[t];
    if (k == 0) permo[q] = perm[p];
}

__global__ void k_perm_init(int64_t n, int64_t *perm) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) perm[p] = p;
}

// ------------------------------------------------------------- orderings

// KD: min and max of each coordinate over each chunk (exact, first occurrence
// kept on equal values, as a scan from the node's first point would).
template <class T>
__global__ void k_kd_minmax(const T *__restrict__ X, int d, int nc, Level L) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nc * d) return;
    int c = (int)(t / d), k = (int)(t % d);
    if (L.status[L.cnode[c]] != ACTIVE) return;
    double lo = (double)X[L.cb[c] * d + k], hi = lo;
    for (int64_t p = L.cb[c] + 1; p < L.ce[c]; ++p) {
        double v = (double)X[p * d + k];
        if (v < lo) lo = v;
        if (v > hi) hi = v;
    }
    L.cps[2 * t] = lo;
    L.cps[2 * t + 1] = hi;
}

// KD: coordinate of maximum spread per node (lowest index on ties).
__global__ void k_kd_pick(int d, int na, Level L) {
    int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= na || L.status[node] != ACTIVE) return;
    double best = -1.0;
    int kb = 0;
    const int c0 = L.ch0[node], c1 = L.ch0[node] + L.nch[node];
    for (int k = 0; k < d; ++k) {
        double lo = L.cps[2 * ((int64_t)c0 * d + k)], hi = L.cps[2 * ((int64_t)c0 * d + k) + 1];
        for (int c = c0 + 1; c < c1; ++c) {
            double a = L.cps[2 * ((int64_t)c * d + k)], b = L.cps[2 * ((int64_t)c * d + k) + 1];
            if (a < lo) lo = a;
            if (b > hi) hi = b;
        }
        double spread = hi - lo;
        if (spread > best) {
            best = spread;
            kb = k;
        }
    }
    if (!(best > 0.0))
        L.status[node] = FALLBACK;
    else
        L.kstar[node] = kb;
}

// KD: the key of each point (the chosen coordinate, -0 made +0) and its
// chunk sum in position order.
template <class T>
__global__ void k_kd_key(const T *__restrict__ X, int d, int nc, Level L, double *__restrict__ key) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    int node = L.cnode[c];
    if (L.status[node] != ACTIVE) return;
    const int k = L.kstar[node];
    double part = 0.0;
    for (int64_t p = L.cb[c]; p < L.ce[c]; ++p) {
        double v = (double)X[p * d + k] + 0.0;
        key[p] = v;
        part = part + v;
    }
    L.cps[c] = part;
}

// Chunk sums of a node added in chunk order, divided by the node size.
__global__ void k_node_mean(int na, Level L) {
    int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= na || L.status[node] != ACTIVE) return;
    double s = 0.0;
    for (int c = L.ch0[node]; c < L.ch0[node] + L.nch[node]; ++c) s = s + L.cps[c];
    L.nmean[node] = s / (double)(L.ne[node] - L.nb[node]);
}

// label 1 iff key > the node's threshold; label-1 count per chunk
__global__ void k_thresh_assign(Level L, const double *__restrict__ key, uint8_t *__restrict__ lab) {
    __shared__ int part[CH / 64];
    int c = blockIdx.x;
    int node = L.cnode[c];
    if (L.status[node] != ACTIVE) return;
    int64_t p = L.cb[c] + threadIdx.x;
    int one = 0;
    if (p < L.ce[c]) {
        one = key[p] <= L.nmean[node] ? 0 : 1;
        lab[p] = (uint8_t)one;
    }
    int s = wave_sum(one);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int i = 0; i < CH / 64; ++i) t += part[i];
        L.cn1[c] = t;
    }
}

// KD: left size from the mean split, or the median fallback when one side
// is more than 100 times the other.
__global__ void k_kd_update(int na, Level L) {
    int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= na || L.status[node] != ACTIVE) return;
    int64_t n1 = 0;
    for (int c = L.ch0[node]; c < L.ch0[node] + L.nch[node]; ++c) n1 += L.cn1[c];
    const int64_t s = L.ne[node] - L.nb[node], n0 = s - n1;
    const int64_t mn = n0 < n1 ? n0 : n1, mx = n0 < n1 ? n1 : n0;
    if (100 * mn < mx) {
        L.status[node] = MEDIAN;
        L.pfx[node] = 0;
        L.krem[node] = s / 2 - 1;  // 0-based rank of the last left point
        L.cless[node] = 0;
    } else {
        L.n1[node] = n1;
    }
}

// order-preserving map of an FP64 value (no -0, no NaN) to uint64
__device__ __forceinline__ uint64_t ordered_bits(double v) {
    uint64_t u = (uint64_t)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | (1ull << 63));
}

// Radix-select pass: histogram of the 8-bit digit at `shift` among the keys
// whose higher digits equal the node's prefix.
__global__ void k_kd_hist(Level L, const double *__restrict__ key, int shift) {
    int c = blockIdx.x;
    int node = L.cnode[c];
    if (L.status[node] != MEDIAN) return;
    int64_t p = L.cb[c] + threadIdx.x;
    if (p >= L.ce[c]) return;
    const uint64_t o = ordered_bits(key[p]);
    const int hs = shift + 8;
    const bool match = hs >= 64 || (o >> hs) == (L.pfx[node] >> hs);
    if (match) atomicAdd(&L.hist[(int64_t)node * 256 + ((o >> shift) & 255)], 1);
}

__global__ void k_kd_select(int na, Level L, int shift) {
    int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= na || L.status[node] != MEDIAN) return;
    int64_t cum = 0;
    const int32_t *h = L.hist + (int64_t)node * 256;
    for (int b = 0; b < 256; ++b) {
        if (L.krem[node] < cum + h[b]) {
            L.pfx[node] |= (uint64_t)b << shift;
            L.krem[node] -= cum;
            L.cless[node] += cum;
            return;
        }
        cum += h[b];
    }
}

// Median split: ties with the selected key per chunk, then their prefix over
// the node's chunks in order.
__global__ void k_kd_ties(Level L, const double *__restrict__ key) {
    __shared__ int part[CH / 64];
    int c = blockIdx.x;
    int node = L.cnode[c];
    if (L.status[node] != MEDIAN) return;
    int64_t p = L.cb[c] + threadIdx.x;
    int tie = p < L.ce[c] && ordered_bits(key[p]) == L.pfx[node];
    int s = wave_sum(tie);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int i = 0; i < CH / 64; ++i) t += part[i];
        L.cn1[c] = t;
    }
}

__global__ void k_kd_tie_prefix(int na, Level L) {
    int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= na || L.status[node] != MEDIAN) return;
    int64_t o = 0;
    for (int c = L.ch0[node]; c < L.ch0[node] + L.nch[node]; ++c) {
        L.off0[c] = o;
        o += L.cn1[c];
    }
    const int64_t s = L.ne[node] - L.nb[node];
    L.n1[node] = s - s / 2;
}

// Median labels: keys below the selected one go left, above go right, and
// the first krem + 1 ties in position order go left.
__global__ void k_kd_median_label(Level L, const double *__restrict__ key, uint8_t *__restrict__ lab) {
    __shared__ int wz[CH / 64];
    __shared__ int part[CH / 64];
    int c = blockIdx.x;
    int node = L.cnode[c];
    if (L.status[node] != MEDIAN) return;
    int64_t p = L.cb[c] + threadIdx.x;
    const bool valid = p < L.ce[c];
    const uint64_t o = valid ? ordered_bits(key[p]) : 0;
    const uint64_t T = L.pfx[node];
    const int tie = valid && o == T;
    uint64_t mask = __ballot(tie);
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    if (lane == 0) wz[wv] = __popcll(mask);
    __syncthreads();
    int before = __popcll(mask & lt);
    for (int i = 0; i < wv; ++i) before += wz[i];
    int one = 0;
    if (valid) {
        if (tie)
            one = (L.off0[c] + before <= L.krem[node]) ? 0 : 1;
        else
            one = o < T ? 0 : 1;
        lab[p] = (uint8_t)one;
    }
    int s = wave_sum(one);
    if (lane == 0) part[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int i = 0; i < CH / 64; ++i) t += part[i];
        L.cn1[c] = t;
    }
}

// PCA: per (chunk, coordinate) sums of the coordinate in position order.
template <class T>
__global__ void k_col_partial(const T *__restrict__ X, int d, int nc, Level L) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nc * d) return;
    int c = (int)(t / d), k = (int)(t % d);
    if (L.status[L.cnode[c]] != ACTIVE) return;
    double part = 0.0;
    for (int64_t p = L.cb[c]; p < L.ce[c]; ++p) part = part + (double)X[p * d + k];
    L.cps[t] = part;
}

// PCA: mean point (c0) and the start vector v = 1 (c1).
__global__ void k_pca_mean(int d, int na, Level L) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)na * d) return;
    int node = (int)(t / d), k = (int)(t % d);
    if (L.status[node] != ACTIVE) return;
    double s = 0.0;
    for (int c = L.ch0[node]; c < L.ch0[node] + L.nch[node]; ++c) s = s + L.cps[(int64_t)c * d + k];
    L.c0[t] = s / (double)(L.ne[node] - L.nb[node]);
    L.c1[t] = 1.0;
}

// PCA: t_p = (x_p - mu) . v, coordinates in order.
template <class T>
__global__ void k_pca_proj(const T *__restrict__ X, int d, Level L, double *__restrict__ q) {
    int c = blockIdx.x;
    int node = L.cnode[c];
    if (L.status[node] != ACTIVE) return;
    int64_t p = L.cb[c] + threadIdx.x;
    if (p >= L.ce[c]) return;
    const double *mu = L.c0 + (int64_t)node * d, *v = L.c1 + (int64_t)node * d;
    double t = 0.0;
    for (int k = 0; k < d; ++k) t = t + ((double)X[p * d + k] - mu[k]) * v[k];
    q[p] = t;
}

// PCA: per (chunk, coordinate) sums of (x_pk - mu_k) t_p in position order.
template <class T>
__global__ void k_pca_wpart(const T *__restrict__ X, int d, int nc, Level L, const double *__restrict__ q) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nc * d) return;
    int c = (int)(t / d), k = (int)(t % d);
    int node = L.cnode[c];
    if (L.status[node] != ACTIVE) return;
    const double mu = L.c0[(int64_t)node * d + k];
    double part = 0.0;
    for (int64_t p = L.cb[c]; p < L.ce[c]; ++p) part = part + ((double)X[p * d + k] - mu) * q[p];
    L.cps[t] = part;
}

// PCA: w = C v (chunk sums in order), v <- w / max|w_k|.
__global__ void k_pca_step(int d, int na, Level L) {
    int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= na || L.status[node] != ACTIVE) return;
    double *w = L.c2 + (int64_t)node * d, *v = L.c1 + (int64_t)node * d;
    double nrm = 0.0;
    for (int k = 0; k < d; ++k) {
        double s = 0.0;
        for (int c = L.ch0[node]; c < L.ch0[node] + L.nch[node]; ++c) s = s + L.cps[(int64_t)c * d + k];
        w[k] = s;
        if (fabs(s) > nrm) nrm = fabs(s);
    }
    if (!(nrm > 0.0)) {
        L.status[node] = FALLBACK;
        return;
    }
    for (int k = 0; k < d; ++k) v[k] = w[k] / nrm;
}

// PCA: chunk sums of the projections in position order.
__global__ void k_chunk_sum(int nc, Level L, const double *__restrict__ q) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc || L.status[L.cnode[c]] != ACTIVE) return;
    double part = 0.0;
    for (int64_t p = L.cb[c]; p < L.ce[c]; ++p) part = part + q[p];
    L.cps[c] = part;
}

// PCA: left size, or the halves fallback for an empty side.
__global__ void k_pca_update(int na, Level L) {
    int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= na || L.status[node] != ACTIVE) return;
    int64_t n1 = 0;
    for (int c = L.ch0[node]; c < L.ch0[node] + L.nch[node]; ++c) n1 += L.cn1[c];
    const int64_t s = L.ne[node] - L.nb[node];
    if (n1 == 0 || n1 == s)
        L.status[node] = FALLBACK;
    else
        L.n1[node] = n1;
}

struct TmpNode {
    int64_t b, e;
    int64_t base;                   // first position of the node's problem
    int64_t left = -1, right = -1;  // indices into the TmpNode list
};

// Labels, left sizes and statuses of one level's nodes by one of the other
// orderings (NP needs no launch: every node splits in halves).
template <class T>
void order_level(int method, const T *Xc, int d, int na, int nc, Level &L, double *key, uint8_t *lab, hipStream_t s) {
    const unsigned gn = ceil_div(na, 64), gnd = ceil_div((int64_t)na * d, 256);
    const unsigned gcd = ceil_div((int64_t)nc * d, 256), gc = ceil_div(nc, 64);
    if (method == KRR_ORDER_KD) {
        k_kd_minmax<T><<<gcd, 256, 0, s>>>(Xc, d, nc, L);
        check_launch("k_kd_minmax");
        k_kd_pick<<<gn, 64, 0, s>>>(d, na, L);
        check_launch("k_kd_pick");
        k_kd_key<T><<<gc, 64, 0, s>>>(Xc, d, nc, L, key);
        check_launch("k_kd_key");
        k_node_mean<<<gn, 64, 0, s>>>(na, L);
        check_launch("k_node_mean");
        k_thresh_assign<<<nc, CH, 0, s>>>(L, key, lab);
        check_launch("k_thresh_assign");
        k_kd_update<<<gn, 64, 0, s>>>(na, L);
        check_launch("k_kd_update");
        for (int shift = 56; shift >= 0; shift -= 8) {
            KRR_HIP(hipMemsetAsync(L.hist, 0, sizeof(int32_t) * 256 * (size_t)na, s));
            k_kd_hist<<<nc, CH, 0, s>>>(L, key, shift);
            check_launch("k_kd_hist");
            k_kd_select<<<gn, 64, 0, s>>>(na, L, shift);
            check_launch("k_kd_select");
        }
        k_kd_ties<<<nc, CH, 0, s>>>(L, key);
        check_launch("k_kd_ties");
        k_kd_tie_prefix<<<gn, 64, 0, s>>>(na, L);
        check_launch("k_kd_tie_prefix");
        k_kd_median_label<<<nc, CH, 0, s>>>(L, key, lab);
        check_launch("k_kd_median_label");
    } else if (method == KRR_ORDER_PCA) {
        k_col_partial<T><<<gcd, 256, 0, s>>>(Xc, d, nc, L);
        check_launch("k_col_partial");
        k_pca_mean<<<gnd, 256, 0, s>>>(d, na, L);
        check_launch("k_pca_mean");
        for (int it = 0; it < PCA_ITERS; ++it) {
            k_pca_proj<T><<<nc, CH, 0, s>>>(Xc, d, L, key);
            check_launch("k_pca_proj");
            k_pca_wpart<T><<<gcd, 256, 0, s>>>(Xc, d, nc, L, key);
            check_launch("k_pca_wpart");
            k_pca_step<<<gn, 64, 0, s>>>(d, na, L);
            check_launch("k_pca_step");
        }
        k_pca_proj<T><<<nc, CH, 0, s>>>(Xc, d, L, key);
        check_launch("k_pca_proj");
        k_chunk_sum<<<gc, 64, 0, s>>>(nc, L, key);
        check_launch("k_chunk_sum");
        k_node_mean<<<gn, 64, 0, s>>>(na, L);
        check_launch("k_node_mean");
        k_thresh_assign<<<nc, CH, 0, s>>>(L, key, lab);
        check_launch("k_thresh_assign");
        k_pca_update<<<gn, 64, 0, s>>>(na, L);
        check_launch("k_pca_update");
    }
}

template <class T>
void cluster_impl(const T *X, int64_t n, int d, const std::vector<int64_t> &roots, const krr_cluster_opts &o,
                  int method, hipStream_t s, int64_t *perm_out, krr_tree_s &tree) {
    const int leaf = o.leaf_size;
    DBuf xa = dalloc<T>(n * d), xb = dalloc<T>(n * d);
    DBuf pa = dalloc<int64_t>(n), pb = dalloc<int64_t>(n);
    DBuf q = dalloc<double>(n), w = dalloc<uint64_t>(n), lab = dalloc<uint8_t>(n), dest = dalloc<int64_t>(n);
    KRR_HIP(hipMemcpyAsync(xa.get(), X, sizeof(T) * n * d, hipMemcpyDeviceToDevice, s));
    k_perm_init<<<ceil_div(n, 256), 256, 0, s>>>(n, pa.as<int64_t>());
    check_launch("k_perm_init");

    // one tree per range [roots[k], roots[k + 1]) (a forest for batched problems)
    std::vector<TmpNode> tn;
    std::vector<int64_t> active;
    const int nroots = (int)roots.size() - 1;
    for (int k = 0; k < nroots; ++k) {
        tn.push_back({roots[k], roots[k + 1], roots[k]});
        if (roots[k + 1] - roots[k] > leaf) active.push_back(k);
    }
    DBuf counter = dalloc<int32_t>(1);
    int64_t levels = 0, fallbacks = 0, capped = 0, iterations = 0;

    while (!active.empty()) {
        ++levels;
        const int na = (int)active.size();
        std::vector<int64_t> nb(na), ne(na), i1(na);
        std::vector<uint64_t> draw1(na);
        std::vector<int32_t> ch0(na), nch(na);
        std::vector<int32_t> cnode;
        std::vector<int64_t> cb, ce;
        for (int a = 0; a < na; ++a) {
            const TmpNode &t = tn[active[a]];
            nb[a] = t.b;
            ne[a] = t.e;
            uint64_t sz = (uint64_t)(t.e - t.b);
            // draws keyed by positions within the problem: each tree of a
            // forest is the tree of its problem clustered alone
            i1[a] = t.b + (int64_t)mulhi_u64(node_draw(o.seed, t.b - t.base, t.e - t.base, 0), sz);
            draw1[a] = node_draw(o.seed, t.b - t.base, t.e - t.base, 1);
            ch0[a] = (int32_t)cnode.size();
            for (int64_t p = t.b; p < t.e; p += CH) {
                cnode.push_back(a);
                cb.push_back(p);
                ce.push_back(std::min<int64_t>(p + CH, t.e));
            }
            nch[a] = (int32_t)cnode.size() - ch0[a];
        }
        const int nc = (int)cnode.size();
        DBuf d_nb = upload(nb, s), d_ne = upload(ne, s), d_i1 = upload(i1, s), d_draw1 = upload(draw1, s);
        DBuf d_ch0 = upload(ch0, s), d_nch = upload(nch, s), d_cnode = upload(cnode, s);
        DBuf d_cb = upload(cb, s), d_ce = upload(ce, s);
        DBuf d_i2 = dalloc<int64_t>(na), d_n1 = dalloc<int64_t>(na), d_qmax = dalloc<uint64_t>(na),
             d_W = dalloc<uint64_t>(na), d_status = dalloc<int32_t>(na), d_changed = dalloc<int32_t>(na),
             d_iters = dalloc<int32_t>(na), d_c0 = dalloc<double>((size_t)na * d),
             d_c1 = dalloc<double>((size_t)na * d), d_off0 = dalloc<int64_t>(nc), d_off1 = dalloc<int64_t>(nc),
             d_cw = dalloc<uint64_t>(nc), d_cn1 = dalloc<int32_t>(nc), d_cps = dalloc<double>((size_t)nc * d * 2),
             d_kstar = dalloc<int32_t>(na), d_nmean = dalloc<double>(na), d_c2 = dalloc<double>((size_t)na * d),
             d_pfx = dalloc<uint64_t>(na), d_krem = dalloc<int64_t>(na), d_cless = dalloc<int64_t>(na),
             d_hist = dalloc<int32_t>(method == KRR_ORDER_KD ? (size_t)na * 256 : 1);
        KRR_HIP(hipMemsetAsync(d_qmax.get(), 0, sizeof(uint64_t) * na, s));
        KRR_HIP(hipMemsetAsync(d_W.get(), 0, sizeof(uint64_t) * na, s));
        KRR_HIP(hipMemsetAsync(d_status.get(), 0, sizeof(int32_t) * na, s));
        KRR_HIP(hipMemsetAsync(d_changed.get(), 0, sizeof(int32_t) * na, s));
        KRR_HIP(hipMemsetAsync(d_iters.get(), 0, sizeof(int32_t) * na, s));
        Level L{d_nb.as<int64_t>(), d_ne.as<int64_t>(), d_i1.as<int64_t>(), d_draw1.as<uint64_t>(),
                d_ch0.as<int32_t>(), d_nch.as<int32_t>(), d_i2.as<int64_t>(), d_n1.as<int64_t>(),
                d_qmax.as<uint64_t>(), d_W.as<uint64_t>(), d_status.as<int32_t>(),
                d_changed.as<int32_t>(), d_iters.as<int32_t>(), d_c0.as<double>(), d_c1.as<double>(),
                d_off0.as<int64_t>(), d_off1.as<int64_t>(), d_cnode.as<int32_t>(), d_cb.as<int64_t>(),
                d_ce.as<int64_t>(), d_cw.as<uint64_t>(), d_cn1.as<int32_t>(), d_cps.as<double>(),
                counter.as<int32_t>(), d_kstar.as<int32_t>(), d_nmean.as<double>(), d_c2.as<double>(),
                d_pfx.as<uint64_t>(), d_krem.as<int64_t>(), d_cless.as<int64_t>(), d_hist.as<int32_t>()};
        const T *Xc = xa.as<T>();
        unsigned gn = ceil_div(na, 64);
        unsigned gnd = ceil_div((int64_t)na * d, 256);
        std::vector<int64_t> n1(na);
        std::vector<int32_t> status(na), iters(na);
        if (method == KRR_ORDER_NP) {
            // no reordering: every node splits in halves, nothing moves
            std::fill(status.begin(), status.end(), (int32_t)FALLBACK);
        } else if (method != KRR_ORDER_2MN) {
            order_level<T>(method, Xc, d, na, nc, L, q.as<double>(), lab.as<uint8_t>(), s);
        }
        if (method == KRR_ORDER_2MN) {
            k_q<T><<<nc, CH, 0, s>>>(Xc, d, L, q.as<double>());
            check_launch("k_q");
            k_w<<<nc, CH, 0, s>>>(L, q.as<double>(), w.as<uint64_t>());
            check_launch("k_w");
            k_pick<<<gn, 64, 0, s>>>(L, na, w.as<uint64_t>());
            check_launch("k_pick");
            k_seed_centers<T><<<gnd, 256, 0, s>>>(Xc, d, na, L);
            check_launch("k_seed_centers");
            k_assign<T><<<nc, CH, 0, s>>>(Xc, d, L, lab.as<uint8_t>(), 1);
            check_launch("k_assign");
            KRR_HIP(hipMemsetAsync(counter.get(), 0, sizeof(int32_t), s));
            k_node_update<<<gn, 64, 0, s>>>(L, na, 1);
            check_launch("k_node_update");
            // Lloyd iterations in groups of four between checks of the
            // active count: the kernels skip nodes that are no longer active,
            // so an iteration after the last node settles changes nothing
            // (each node still runs at most max_iter iterations)
            constexpr int kLloydGroup = 4;
            for (int it = 0; it < o.max_iter; it += kLloydGroup) {
                int32_t nact = 0;
                d2h(&nact, counter.as<int32_t>(), 1, s);
                sync(s);
                if (nact == 0) break;
                for (int j = 0; j < kLloydGroup && it + j < o.max_iter; ++j) {
                    k_centroid_partial<T><<<ceil_div((int64_t)nc * d, 256), 256, 0, s>>>(Xc, d, nc, L,
                                                                                         lab.as<uint8_t>());
                    check_launch("k_centroid_partial");
                    k_centroid_final<<<gnd, 256, 0, s>>>(d, na, L);
                    check_launch("k_centroid_final");
                    k_assign<T><<<nc, CH, 0, s>>>(Xc, d, L, lab.as<uint8_t>(), 0);
                    check_launch("k_assign");
                    KRR_HIP(hipMemsetAsync(counter.get(), 0, sizeof(int32_t), s));
                    k_node_update<<<gn, 64, 0, s>>>(L, na, 0);
                    check_launch("k_node_update");
                }
            }
        }
        if (method != KRR_ORDER_NP) {
            k_part_prefix<<<gn, 64, 0, s>>>(L, na);
            check_launch("k_part_prefix");
            k_iota<<<ceil_div(n, 256), 256, 0, s>>>(n, dest.as<int64_t>());
            check_launch("k_iota");
            k_part_dest<<<nc, CH, 0, s>>>(L, lab.as<uint8_t>(), dest.as<int64_t>());
            check_launch("k_part_dest");
            k_move<T><<<ceil_div(n * d, 256), 256, 0, s>>>(xa.as<T>(), pa.as<int64_t>(), n, d, dest.as<int64_t>(),
                                                            xb.as<T>(), pb.as<int64_t>());
            check_launch("k_move");
            std::swap(xa, xb);
            std::swap(pa, pb);
            d2h(n1.data(), d_n1.as<int64_t>(), na, s);
            d2h(status.data(), d_status.as<int32_t>(), na, s);
            d2h(iters.data(), d_iters.as<int32_t>(), na, s);
            sync(s);
        }
        std::vector<int64_t> next;
        for (int a = 0; a < na; ++a) {
            int64_t id = active[a];
            int64_t b = tn[id].b, e = tn[id].e, sz = e - b;
            int64_t nl;
            if (method == KRR_ORDER_2MN) iterations += iters[a];
            if (status[a] == FALLBACK) {
                if (method != KRR_ORDER_NP) ++fallbacks;
                nl = sz / 2;
            } else {
                // 2MN: a split still active after max_iter hit the cap; KD: a
                // median split
                if ((method == KRR_ORDER_2MN && status[a] == ACTIVE) || status[a] == MEDIAN) ++capped;
                nl = sz - n1[a];
            }
            int64_t li = (int64_t)tn.size();
            tn.push_back({b, b + nl, tn[id].base});
            tn.push_back({b + nl, e, tn[id].base});
            tn[id].left = li;
            tn[id].right = li + 1;
            if (nl > leaf) next.push_back(li);
            if (sz - nl > leaf) next.push_back(li + 1);
        }
        active.swap(next);
    }
    KRR_HIP(hipMemcpyAsync(perm_out, pa.get(), sizeof(int64_t) * n, hipMemcpyDeviceToDevice, s));

    // postorder numbering of the discovered trees, one after the other
    tree.n = n;
    tree.nodes.assign(tn.size() * 5, -1);
    tree.roots.clear();
    std::vector<int64_t> id_of(tn.size(), -1);
    int64_t next_id = 0;
    for (int k = 0; k < nroots; ++k) {
        std::vector<std::pair<int64_t, int>> stack{{(int64_t)k, 0}};
        while (!stack.empty()) {
            auto &top = stack.back();
            const TmpNode &t = tn[top.first];
            if (t.left >= 0 && top.second == 0) {
                top.second = 1;
                stack.push_back({t.left, 0});
            } else if (t.left >= 0 && top.second == 1) {
                top.second = 2;
                stack.push_back({t.right, 0});
            } else {
                int64_t id = next_id++;
                id_of[top.first] = id;
                int64_t *row = &tree.nodes[5 * id];
                row[0] = t.b;
                row[1] = t.e;
                row[2] = t.left >= 0 ? id_of[t.left] : -1;
                row[3] = t.right >= 0 ? id_of[t.right] : -1;
                row[4] = -1;
                if (t.left >= 0) {
                    tree.nodes[5 * row[2] + 4] = id;
                    tree.nodes[5 * row[3] + 4] = id;
                }
                stack.pop_back();
            }
        }
        tree.roots.push_back(next_id - 1);
    }
    tree.stats = {fallbacks, capped, iterations, levels};
    sync(s);  // keep the temporaries alive until the last copy is done
}

}  // namespace

void cluster_2mn(const void *X, int32_t xprec, int64_t n, int32_t d, const std::vector<int64_t> &roots,
                 const krr_cluster_opts &o, hipStream_t s, int64_t *perm, krr_tree_s &tree, int32_t method) {
    if (xprec == KRR_F64)
        cluster_impl<double>(static_cast<const double *>(X), n, d, roots, o, method, s, perm, tree);
    else
        cluster_impl<float>(static_cast<const float *>(X), n, d, roots, o, method, s, perm, tree);
}

}  // namespace krr
