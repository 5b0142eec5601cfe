// HSS compression by randomized sampling (Section 3.1, the randomized
// construction that needs only a kernel product with a random block and
// selected kernel entries -- the "partially matrix-free" interface of
// Section 1.1 -- with adaptive sample growth).
//
// K is symmetric, so U = V and B_right,left = B_left,right^T.  Bottom-up over
// the tree levels (nodes grouped by height), one workgroup per node:
//   leaf    Y = rows I of the off-diagonal sample S = K R (own leaf block
//           excluded), D = K(I, I)
//   parent  Y = [Ysk_a - B_ab Om_b ; Ysk_b - B_ab^T Om_a], B_ab = K(J_a, J_b)
//   ID      pivoted Cholesky of the Gram matrix Y Y^T (the same pivots and
//           |R_jj| as column-pivoted QR of Y^T): rank k = leading pivots with
//           |R_jj| > max(rtol |R_00|, atol sqrt(r)); U = P [I; (R11^{-1} R12)^T]
//   then    Ysk = Y(J), Om = U^T R(I) (leaf) or U^T [Om_a; Om_b] (parent).
// If some node whose sample could hide rank (m > r - p) reaches k > r - p,
// the block R is widened by dr columns (only the new columns are sampled)
// and the levels are redone.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "dense.hpp"
#include "internal.hpp"

namespace krr {


std::vector<std::vector<int>> levels_by_height(std::vector<HNode> &nodes) {
    int maxh = 0;
    for (size_t i = 0; i < nodes.size(); ++i) {
        HNode &nd = nodes[i];
        nd.height = nd.left < 0 ? 0 : 1 + std::max(nodes[nd.left].height, nodes[nd.right].height);
        maxh = std::max(maxh, nd.height);
    }
    std::vector<std::vector<int>> lv(maxh + 1);
    for (size_t i = 0; i < nodes.size(); ++i) lv[nodes[i].height].push_back((int)i);
    return lv;
}

void validate_tree(const krr_tree_s *t) {
    const int64_t nn = t->n_nodes();
    KRR_REQUIRE(nn >= 1, "tree has no nodes");
    KRR_REQUIRE(!t->roots.empty(), "tree has no roots");
    for (int64_t i = 0; i < nn; ++i) {
        KRR_REQUIRE(t->e(i) > t->b(i), "node %lld is empty", (long long)i);
        if (!t->leaf(i)) {
            int64_t l = t->left(i), r = t->right(i);
            KRR_REQUIRE(l >= 0 && r >= 0 && l < i && r < i, "node %lld: children must precede it", (long long)i);
            KRR_REQUIRE(t->b(l) == t->b(i) && t->e(l) == t->b(r) && t->e(r) == t->e(i),
                        "node %lld: children must split its range", (long long)i);
            KRR_REQUIRE(t->parent(l) == i && t->parent(r) == i, "node %lld: children's parent link", (long long)i);
        } else {
            KRR_REQUIRE(t->right(i) < 0, "leaf %lld has a right child", (long long)i);
        }
        const int64_t p = t->parent(i);
        KRR_REQUIRE(p < 0 || (p > i && p < nn && (t->left(p) == i || t->right(p) == i)),
                    "node %lld: parent link", (long long)i);
    }
    int64_t pos = 0, prev = -1;
    for (int64_t r : t->roots) {
        KRR_REQUIRE(r > prev && r < nn && t->parent(r) < 0, "root %lld is not a root", (long long)r);
        KRR_REQUIRE(t->b(r) == pos, "roots must cover [0, n) in order");
        // each tree's nodes are stored together, ending at its root
        for (int64_t i = prev + 1; i <= r; ++i)
            KRR_REQUIRE(t->b(i) >= t->b(r) && t->e(i) <= t->e(r), "node %lld lies outside its tree", (long long)i);
        pos = t->e(r);
        prev = r;
    }
    KRR_REQUIRE(pos == t->n && prev == nn - 1, "roots must cover [0, n) and end the node list");
}

namespace {

struct NodeDesc {
    int32_t m, kl, kr, leaf;
    int32_t k, pad_;
    int64_t b;
    double inv;  // 1 / (2 h^2) of the node's problem
    double *Y, *G, *Lf;
    int32_t *piv;
    double *D, *B;
    const double *Ysk_l, *Ysk_r, *Om_l, *Om_r;
    const int32_t *J_l, *J_r;
    double *U;
    int32_t *J;
    double *Ysk, *Om;
};

template <class T>
__device__ __forceinline__ double pair_kernel(const T *__restrict__ X, int d, int64_t i, int64_t j, double inv) {
    double q = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = (double)X[i * d + k] - (double)X[j * d + k];
        q = fma(t, t, q);
    }
    return exp(-q * inv);
}

template <class T>
__global__ __launch_bounds__(BG_T) void k_extract(const T *__restrict__ X, int d, const NodeDesc *nds) {
    const NodeDesc nd = nds[blockIdx.x];
    const double inv = nd.inv;
    if (nd.leaf) {
        const int m = nd.m;
        for (int t = threadIdx.x; t < m * m; t += BG_T) {
            int a = t / m, c = t % m;
            nd.D[t] = (a == c) ? 1.0 : pair_kernel(X, d, nd.b + a, nd.b + c, inv);
        }
    } else {
        for (int t = threadIdx.x; t < nd.kl * nd.kr; t += BG_T) {
            int a = t / nd.kr, c = t % nd.kr;
            nd.B[t] = pair_kernel(X, d, nd.J_l[a], nd.J_r[c], inv);
        }
    }
}

template <class ST>
__global__ __launch_bounds__(BG_T) void k_build_y(const NodeDesc *nds, const ST *__restrict__ S, int r) {
    __shared__ double smem[2 * 16 * 65];
    const NodeDesc nd = nds[blockIdx.x];
    if (nd.leaf) {
        for (int64_t t = threadIdx.x; t < (int64_t)nd.m * r; t += BG_T) nd.Y[t] = (double)S[nd.b * r + t];
        return;
    }
    for (int64_t t = threadIdx.x; t < (int64_t)nd.kl * r; t += BG_T) nd.Y[t] = nd.Ysk_l[t];
    for (int64_t t = threadIdx.x; t < (int64_t)nd.kr * r; t += BG_T) nd.Y[(int64_t)nd.kl * r + t] = nd.Ysk_r[t];
    __syncthreads();
    // Y_top -= B Om_r ; Y_bottom -= B^T Om_l
    block_gemm(nd.kl, r, nd.kr, -1.0, nd.B, nd.kr, 1, nd.Om_r, r, 1, 1.0, nd.Y, r, smem);
    block_gemm(nd.kr, r, nd.kl, -1.0, nd.B, 1, nd.kr, nd.Om_l, r, 1, 1.0, nd.Y + (int64_t)nd.kl * r, r, smem);
}

__global__ __launch_bounds__(BG_T) void k_gram(const NodeDesc *nds, int r) {
    __shared__ double smem[2 * 16 * 65];
    const NodeDesc nd = nds[blockIdx.x];
    block_gemm(nd.m, nd.m, r, 1.0, nd.Y, r, 1, nd.Y, 1, r, 0.0, nd.G, nd.m, smem);
}

// Pivoted Cholesky of G = Y Y^T with the ID stopping rule.  Dynamic LDS:
// m doubles (residual diagonal) + m ints (pivoted flags).
__global__ __launch_bounds__(BG_T) void k_pivchol(const NodeDesc *nds, int r, int kmax, double rtol, double atol_abs,
                                                  int32_t *kout, int32_t *flag) {
    extern __shared__ double dyn[];
    __shared__ double redv[BG_T / 64];
    __shared__ int redi[BG_T / 64];
    const NodeDesc nd = nds[blockIdx.x];
    const int m = nd.m;
    double *dres = dyn;
    int *done = reinterpret_cast<int *>(dyn + m);
    for (int i = threadIdx.x; i < m; i += BG_T) {
        dres[i] = nd.G[(int64_t)i * m + i];
        done[i] = 0;
    }
    __syncthreads();
    const int kcap = min(m, min(r, kmax));
    double r00 = 0.0;
    int j = 0;
    bool bad = false;
    for (; j < kcap; ++j) {
        double bv = -1.0;
        int bi = -1;
        for (int i = threadIdx.x; i < m; i += BG_T) {
            if (done[i]) continue;
            double v = dres[i];
            if (bi < 0 || v > bv) {
                bv = v;
                bi = i;
            }
        }
        double best;
        int p;
        block_argmax(bv, bi, redv, redi, best, p);
        if (p < 0) break;
        if (!(best == best) || isinf(best)) {
            bad = true;
            break;
        }
        if (j == 0) r00 = sqrt(fmax(best, 0.0));
        double thr = fmax(rtol * r00, atol_abs);
        if (best <= 0.0 || sqrt(best) <= thr) break;
        const double sp = sqrt(best);
        for (int i = threadIdx.x; i < m; i += BG_T) {
            if (done[i] || i == p) continue;
            double v = nd.G[(int64_t)i * m + p];
            const double *li = nd.Lf + (int64_t)i * m;
            const double *lp = nd.Lf + (int64_t)p * m;
            for (int l = 0; l < j; ++l) v -= li[l] * lp[l];
            v /= sp;
            nd.Lf[(int64_t)i * m + j] = v;
            dres[i] -= v * v;
        }
        if (threadIdx.x == 0) {
            nd.Lf[(int64_t)p * m + j] = sp;
            nd.piv[j] = p;
            done[p] = 1;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int o = j;
        for (int i = 0; i < m; ++i)
            if (!done[i]) nd.piv[o++] = i;
        kout[blockIdx.x] = j;
        if (bad) atomicOr(flag, 1);
    }
}

template <class RT>
__global__ __launch_bounds__(BG_T) void k_id_finish(const NodeDesc *nds, int r, const RT *__restrict__ R) {
    __shared__ double smem[2 * 16 * 65];
    const NodeDesc nd = nds[blockIdx.x];
    const int m = nd.m, k = nd.k, ne = m - k;
    // T = R11^{-1} R12, written straight into the rows of U it belongs to
    for (int c = threadIdx.x; c < ne; c += BG_T) {
        const int rowc = nd.piv[k + c];
        double *urow = nd.U + (int64_t)rowc * k;
        for (int l = k - 1; l >= 0; --l) {
            double t = nd.Lf[(int64_t)rowc * m + l];
            for (int l2 = l + 1; l2 < k; ++l2) t -= nd.Lf[(int64_t)nd.piv[l2] * m + l] * urow[l2];
            urow[l] = t / nd.Lf[(int64_t)nd.piv[l] * m + l];
        }
    }
    for (int t = threadIdx.x; t < k * k; t += BG_T) {
        int l = t / k, c = t % k;
        nd.U[(int64_t)nd.piv[l] * k + c] = (l == c) ? 1.0 : 0.0;
    }
    for (int l = threadIdx.x; l < k; l += BG_T) {
        int p = nd.piv[l];
        nd.J[l] = nd.leaf ? (int32_t)(nd.b + p) : (p < nd.kl ? nd.J_l[p] : nd.J_r[p - nd.kl]);
    }
    for (int64_t t = threadIdx.x; t < (int64_t)k * r; t += BG_T) {
        int64_t l = t / r, c = t % r;
        nd.Ysk[t] = nd.Y[(int64_t)nd.piv[l] * r + c];
    }
    __syncthreads();
    if (k == 0) return;
    if (nd.leaf) {
        block_gemm(k, r, m, 1.0, nd.U, 1, k, R + nd.b * r, r, 1, 0.0, nd.Om, r, smem);
    } else {
        block_gemm(k, r, nd.kl, 1.0, nd.U, 1, k, nd.Om_l, r, 1, 0.0, nd.Om, r, smem);
        block_gemm(k, r, nd.kr, 1.0, nd.U + (int64_t)nd.kl * k, 1, k, nd.Om_r, r, 1, 1.0, nd.Om, r, smem);
    }
}

__global__ void k_leaf_ranges(const int64_t *lb64, const int64_t *le64, int nleaves, int32_t *lb, int32_t *le) {
    int t = blockIdx.x;
    int64_t b = lb64[t], e = le64[t];
    for (int64_t p = b + threadIdx.x; p < e; p += blockDim.x) {
        lb[p] = (int32_t)b;
        le[p] = (int32_t)e;
    }
}

// Per-node device storage produced by one level.
// Gather of the per-level node outputs into the generator pools: one
// workgroup per (source, destination, 4-byte words) segment, so the pools are
// filled by a single launch instead of a copy per node and pool.
struct CopySeg {
    const uint32_t *src;
    uint32_t *dst;
    int64_t words;
};

__global__ __launch_bounds__(256) void k_copy_segments(const CopySeg *__restrict__ segs) {
    const CopySeg c = segs[blockIdx.x];
    for (int64_t w = threadIdx.x; w < c.words; w += blockDim.x) c.dst[w] = c.src[w];
}

struct NodeOut {
    double *U = nullptr, *Ysk = nullptr, *Om = nullptr, *B = nullptr, *D = nullptr;
    int32_t *J = nullptr;
    int32_t k = 0, m = 0;
};

struct Attempt {
    std::vector<NodeOut> out;
    std::vector<DBuf> keep;        // per-level U, J, Ysk, Om, B buffers
    std::vector<int64_t> lvl_uoff; // unused placeholder for symmetry
};

// Runs every level with sample width r.  Returns false when some rank
// reached r - p while its sample could have hidden more.
bool run_levels(hss_s *H, const void *Xp, int xprec, int d, const hss_opts &o, int r, bool truncate,
                const float *R, const void *S, bool s64, double *Dpool, const std::vector<int64_t> &doff,
                Attempt &A, hipStream_t s, double &t_id) {
    EventTimer timer(s);
    const int nn = (int)H->node.size();
    A.out.assign(nn, NodeOut());
    A.keep.clear();
    const double atol_abs = o.atol * std::sqrt((double)r);
    DBuf flag = dalloc<int32_t>(1);
    KRR_HIP(hipMemsetAsync(flag.get(), 0, sizeof(int32_t), s));
    for (const auto &lv : H->levels) {
        const int cnt = (int)lv.size();
        std::vector<NodeDesc> nd(cnt);
        int64_t ysz = 0, gsz = 0, psz = 0, bsz = 0;
        int mmax = 0;
        std::vector<int> ids(cnt);
        for (int a = 0; a < cnt; ++a) {
            const HNode &hn = H->node[lv[a]];
            NodeDesc &q = nd[a];
            std::memset(&q, 0, sizeof q);
            ids[a] = lv[a];
            q.leaf = hn.left < 0;
            q.b = hn.b;
            {
                const double hk = H->hprob[H->nprob[lv[a]]];
                q.inv = 1.0 / (2.0 * hk * hk);
            }
            if (q.leaf) {
                q.m = (int32_t)(hn.e - hn.b);
            } else {
                q.kl = A.out[hn.left].k;
                q.kr = A.out[hn.right].k;
                q.m = q.kl + q.kr;
                bsz += (int64_t)q.kl * q.kr;
            }
            ysz += (int64_t)q.m * r;
            gsz += (int64_t)q.m * q.m;
            psz += q.m;
            mmax = std::max(mmax, q.m);
        }
        DBuf Yb = dalloc<double>(ysz), Gb = dalloc<double>(gsz), Lb = dalloc<double>(gsz), Pb = dalloc<int32_t>(psz);
        DBuf Bb = dalloc<double>(bsz);
        {
            int64_t oy = 0, og = 0, op = 0, ob = 0;
            for (int a = 0; a < cnt; ++a) {
                NodeDesc &q = nd[a];
                const HNode &hn = H->node[ids[a]];
                q.Y = Yb.as<double>() + oy;
                q.G = Gb.as<double>() + og;
                q.Lf = Lb.as<double>() + og;
                q.piv = Pb.as<int32_t>() + op;
                oy += (int64_t)q.m * r;
                og += (int64_t)q.m * q.m;
                op += q.m;
                if (q.leaf) {
                    q.D = Dpool + doff[ids[a]];
                    A.out[ids[a]].D = q.D;
                } else {
                    q.B = Bb.as<double>() + ob;
                    ob += (int64_t)q.kl * q.kr;
                    A.out[ids[a]].B = q.B;
                    const NodeOut &L = A.out[hn.left], &Rr = A.out[hn.right];
                    q.Ysk_l = L.Ysk; q.Ysk_r = Rr.Ysk; q.Om_l = L.Om; q.Om_r = Rr.Om;
                    q.J_l = L.J; q.J_r = Rr.J;
                }
                A.out[ids[a]].m = q.m;
            }
        }
        DBuf dnd = upload(nd, s);
        auto *dq = dnd.as<NodeDesc>();
        if (xprec == KRR_F64)
            k_extract<double><<<cnt, BG_T, 0, s>>>(static_cast<const double *>(Xp), d, dq);
        else
            k_extract<float><<<cnt, BG_T, 0, s>>>(static_cast<const float *>(Xp), d, dq);
        check_launch("k_extract");
        A.keep.push_back(std::move(Bb));
        // roots have no basis: the rest of the level works on the other nodes
        {
            std::vector<NodeDesc> keep_nd;
            std::vector<int> keep_ids;
            for (int a = 0; a < cnt; ++a)
                if (H->node[ids[a]].parent >= 0) {
                    keep_nd.push_back(nd[a]);
                    keep_ids.push_back(ids[a]);
                }
            if (keep_nd.empty()) {
                sync(s);
                continue;
            }
            if ((int)keep_nd.size() != cnt) {
                sync(s);  // the uploaded descriptors are replaced below
                nd.swap(keep_nd);
                ids.swap(keep_ids);
                dnd = upload(nd, s);
                dq = dnd.as<NodeDesc>();
            }
        }
        const int cnt2 = (int)nd.size();
        if (s64)
            k_build_y<double><<<cnt2, BG_T, 0, s>>>(dq, static_cast<const double *>(S), r);
        else
            k_build_y<float><<<cnt2, BG_T, 0, s>>>(dq, static_cast<const float *>(S), r);
        check_launch("k_build_y");
        k_gram<<<cnt2, BG_T, 0, s>>>(dq, r);
        check_launch("k_gram");
        DBuf kout = dalloc<int32_t>(cnt2);
        size_t dyn = (size_t)mmax * (sizeof(double) + sizeof(int));
        KRR_REQUIRE(dyn <= 150 * 1024, "node sample of %d rows exceeds the LDS budget", mmax);
        const int kmax = truncate ? std::max(0, r - o.oversample) : r;
        k_pivchol<<<cnt2, BG_T, dyn, s>>>(dq, r, kmax, o.rtol, atol_abs, kout.as<int32_t>(), flag.as<int32_t>());
        check_launch("k_pivchol");
        std::vector<int32_t> ks(cnt2);
        int32_t bad = 0;
        d2h(ks.data(), kout.as<int32_t>(), cnt2, s);
        d2h(&bad, flag.as<int32_t>(), 1, s);
        sync(s);
        if (bad) fail(KRR_E_NUMERIC, "non-finite values in the sampled block rows");
        bool grow = false;
        int64_t usz = 0, ksz = 0;
        for (int a = 0; a < cnt2; ++a) {
            nd[a].k = ks[a];
            if (nd[a].m > r - o.oversample && ks[a] > r - o.oversample) grow = true;
            usz += (int64_t)nd[a].m * ks[a];
            ksz += ks[a];
        }
        if (verbose()) {
            int mk = 0, mm = 0;
            for (int a = 0; a < cnt2; ++a) {
                mk = std::max(mk, (int)ks[a]);
                mm = std::max(mm, (int)nd[a].m);
            }
            fprintf(stderr, "[krr] compress r=%d level h=%d nodes=%d max m=%d max k=%d%s\n", r,
                    H->node[ids[0]].height, cnt2, mm, mk, grow ? " -> grow" : "");
        }
        if (grow && !truncate) return false;
        DBuf Ub = dalloc<double>(usz), Jb = dalloc<int32_t>(ksz), Sk = dalloc<double>(ksz * r),
             Om = dalloc<double>(ksz * r);
        {
            int64_t ou = 0, ok = 0;
            for (int a = 0; a < cnt2; ++a) {
                NodeDesc &q = nd[a];
                q.U = Ub.as<double>() + ou;
                q.J = Jb.as<int32_t>() + ok;
                q.Ysk = Sk.as<double>() + ok * r;
                q.Om = Om.as<double>() + ok * r;
                ou += (int64_t)q.m * q.k;
                ok += q.k;
                NodeOut &no = A.out[ids[a]];
                no.U = q.U; no.J = q.J; no.Ysk = q.Ysk; no.Om = q.Om; no.k = q.k;
            }
        }
        h2d(dq, nd.data(), cnt2, s);
        k_id_finish<float><<<cnt2, BG_T, 0, s>>>(dq, r, R);
        check_launch("k_id_finish");
        A.keep.push_back(std::move(Ub));
        A.keep.push_back(std::move(Jb));
        A.keep.push_back(std::move(Sk));
        A.keep.push_back(std::move(Om));
        sync(s);  // level temporaries (Y, G, L, piv, descriptors) are released next
    }
    t_id += timer.stop_ms();
    return true;
}

}  // namespace

void compress(const krr_tree_s *t, const void *Xp, int xprec, int d, const std::vector<double> &hprob,
              const hss_opts &o, hipStream_t s, hss_s *H, hss_stats *st) {
    EventTimer total(s);
    const int64_t n = t->n;
    const int64_t nn = t->n_nodes();
    const int np = (int)t->roots.size();
    KRR_REQUIRE((int)hprob.size() == np, "one kernel width per tree is required (%d trees, %d widths)", np,
                (int)hprob.size());
    H->n = n;
    H->d = d;
    H->h = hprob[0];
    H->hprob = hprob;
    H->node.resize(nn);
    H->nprob.assign(nn, 0);
    H->pbeg.assign(1, 0);
    {
        int64_t first = 0;  // trees are stored one after the other, each ending at its root
        for (int k = 0; k < np; ++k) {
            const int64_t rt = t->roots[k];
            for (int64_t i = first; i <= rt; ++i) H->nprob[i] = k;
            first = rt + 1;
            H->pbeg.push_back(t->e(rt));
        }
    }
    Batch batch;
    batch.pbeg = H->pbeg;
    batch.h = hprob;
    const Batch *bp = np > 1 ? &batch : nullptr;
    const double h = hprob[0];
    for (int64_t i = 0; i < nn; ++i) {
        HNode &q = H->node[i];
        q = HNode{t->b(i), t->e(i), t->left(i), t->right(i), t->parent(i), 0, 0, 0, -1, -1, -1, -1};
    }
    H->levels = levels_by_height(H->node);
    // leaf ranges per point (for the sample mask) and the D pool
    std::vector<int64_t> lb64, le64, doff(nn, -1);
    int64_t dsz = 0;
    for (int64_t i = 0; i < nn; ++i)
        if (H->node[i].left < 0) {
            lb64.push_back(H->node[i].b);
            le64.push_back(H->node[i].e);
            doff[i] = dsz;
            int64_t m = H->node[i].e - H->node[i].b;
            dsz += m * m;
        }
    DBuf dlb = upload(lb64, s), dle = upload(le64, s);
    DBuf plb = dalloc<int32_t>(n), ple = dalloc<int32_t>(n);
    k_leaf_ranges<<<(unsigned)lb64.size(), 256, 0, s>>>(dlb.as<int64_t>(), dle.as<int64_t>(), (int)lb64.size(),
                                                        plb.as<int32_t>(), ple.as<int32_t>());
    check_launch("k_leaf_ranges");
    H->D.alloc(sizeof(double) * dsz);
    H->nD = dsz;

    const bool s64 = (o.prec == KRR_F64);
    const size_t sel = s64 ? sizeof(double) : sizeof(float);
    int r = o.r0;
    DBuf R = dalloc<float>((size_t)n * r);
    DBuf S((size_t)n * r * sel);
    double t_sample = 0, t_id = 0;
    {
        EventTimer ts(s);
        random_block(o.seed, n, r, 0, R.as<float>(), r, s);
        sample_product(Xp, n, d, xprec, h, R.as<float>(), r, plb.as<int32_t>(), ple.as<int32_t>(), S.get(),
                       o.prec, o.split_terms, s, bp);
        t_sample += ts.stop_ms();
    }
    Attempt A;
    int regrowths = 0;
    bool truncated = false;
    while (!run_levels(H, Xp, xprec, d, o, r, truncated, R.as<float>(), S.get(), s64, H->D.as<double>(), doff, A,
                       s, t_id)) {
        if (r >= o.r_max) {
            if (o.cap_policy == 0)
                fail(KRR_E_RANK_CAP, "ranks not revealed with the sample width cap r_max = %d", o.r_max);
            truncated = true;  // redo the levels once more, cutting ranks at r_max - p
            continue;
        }
        int r2 = std::min(o.r_max, r + o.dr);
        int dr = r2 - r;
        EventTimer ts(s);
        DBuf Rn = dalloc<float>((size_t)n * dr), Sn((size_t)n * dr * sel);
        random_block(o.seed, n, dr, r, Rn.as<float>(), dr, s);
        sample_product(Xp, n, d, xprec, h, Rn.as<float>(), dr, plb.as<int32_t>(), ple.as<int32_t>(), Sn.get(),
                       o.prec, o.split_terms, s, bp);
        DBuf R2 = dalloc<float>((size_t)n * r2), S2((size_t)n * r2 * sel);
        KRR_HIP(hipMemcpy2DAsync(R2.get(), r2 * sizeof(float), R.get(), r * sizeof(float), r * sizeof(float), n,
                                 hipMemcpyDeviceToDevice, s));
        KRR_HIP(hipMemcpy2DAsync(R2.as<float>() + r, r2 * sizeof(float), Rn.get(), dr * sizeof(float),
                                 dr * sizeof(float), n, hipMemcpyDeviceToDevice, s));
        KRR_HIP(hipMemcpy2DAsync(S2.get(), r2 * sel, S.get(), r * sel, r * sel, n, hipMemcpyDeviceToDevice, s));
        KRR_HIP(hipMemcpy2DAsync(static_cast<char *>(S2.get()) + r * sel, r2 * sel, Sn.get(), dr * sel, dr * sel, n,
                                 hipMemcpyDeviceToDevice, s));
        t_sample += ts.stop_ms();
        R = std::move(R2);
        S = std::move(S2);
        r = r2;
        ++regrowths;
    }
    // consolidate the per-level generator buffers into single pools
    int64_t usz = 0, jsz = 0, bsz = 0;
    int maxk = 0;
    for (int64_t i = 0; i < nn; ++i) {
        HNode &q = H->node[i];
        const NodeOut &no = A.out[i];
        q.m = no.m;
        q.k = no.k;
        maxk = std::max(maxk, (int)no.k);
        q.offD = doff[i];
        if (q.parent >= 0) {
            q.offU = usz;
            usz += (int64_t)no.m * no.k;
            q.offJ = jsz;
            jsz += no.k;
        } else {
            q.k = 0;
        }
        if (q.left >= 0) {
            q.offB = bsz;
            bsz += (int64_t)A.out[q.left].k * A.out[q.right].k;
        }
    }
    H->U.alloc(sizeof(double) * std::max<int64_t>(usz, 1));
    H->J.alloc(sizeof(int32_t) * std::max<int64_t>(jsz, 1));
    H->B.alloc(sizeof(double) * std::max<int64_t>(bsz, 1));
    H->nU = usz;
    H->nJ = jsz;
    H->nB = bsz;
    std::vector<CopySeg> segs;
    segs.reserve(3 * nn);
    auto seg = [&](const void *src, void *dst, int64_t bytes) {
        segs.push_back({static_cast<const uint32_t *>(src), static_cast<uint32_t *>(dst), bytes / 4});
    };
    for (int64_t i = 0; i < nn; ++i) {
        const HNode &q = H->node[i];
        const NodeOut &no = A.out[i];
        if (q.offU >= 0 && q.m * (int64_t)q.k > 0) seg(no.U, H->U.as<double>() + q.offU, sizeof(double) * q.m * q.k);
        if (q.offJ >= 0 && q.k > 0) seg(no.J, H->J.as<int32_t>() + q.offJ, sizeof(int32_t) * q.k);
        if (q.offB >= 0) {
            const int64_t kb = (int64_t)A.out[q.left].k * A.out[q.right].k;
            if (kb) seg(no.B, H->B.as<double>() + q.offB, sizeof(double) * kb);
        }
    }
    if (!segs.empty()) {
        DBuf dseg = upload(segs, s);
        k_copy_segments<<<(unsigned)segs.size(), 256, 0, s>>>(dseg.as<CopySeg>());
        check_launch("k_copy_segments");
        sync(s);  // the segment table and the per-level outputs are released after this
    }
    sync(s);
    H->r_final = r;
    H->regrowths = regrowths;
    H->max_rank = maxk;
    H->truncated = truncated ? 1 : 0;
    if (st) {
        st->truncated = H->truncated;
        st->n = n;
        st->n_nodes = nn;
        st->levels = (int64_t)H->levels.size();
        st->r_final = r;
        st->regrowths = regrowths;
        st->max_rank = maxk;
        int64_t paper = H->nD + 2 * H->nU + 2 * H->nB;
        st->bytes_paper = 8 * paper;
        st->bytes_stored = 8 * (H->nD + H->nU + H->nB) + 4 * H->nJ;
        st->t_sample_ms = t_sample;
        st->t_id_ms = t_id;
        st->t_total_ms = total.stop_ms();
    }
}

}  // namespace krr
