// Product of a compressed HSS matrix with a block of vectors (Section 3.1
// representation, symmetric with U = V): upward pass x^_t = U_t^T x(I_t) at
// leaves and x^_p = U_p^T [x^_a; x^_b] above; downward pass
// y^_a = B_ab x^_b + (U_p y^_p)_a, y^_b = B_ab^T x^_a + (U_p y^_p)_b;
// leaves y(I_t) = D_t x(I_t) + U_t y^_t.  One workgroup per node per level.
#include <cstring>

#include "dense.hpp"
#include "internal.hpp"

namespace krr {
namespace {

struct MvDesc {
    int32_t m, k, kl, kr, leaf, root;
    int64_t b;
    const double *U, *D, *B;
    double *xh, *yh;                 // this node's k x nrhs
    const double *xh_l, *xh_r;       // children (upward)
    double *yh_l, *yh_r;             // children (downward)
};

__global__ __launch_bounds__(BG_T) void k_mv_up(const MvDesc *dsc, const double *__restrict__ x, int nrhs) {
    __shared__ double smem[2 * 16 * 65];
    const MvDesc q = dsc[blockIdx.x];
    if (q.root || q.k == 0) return;
    if (q.leaf) {
        block_gemm(q.k, nrhs, q.m, 1.0, q.U, 1, q.k, x + q.b * nrhs, nrhs, 1, 0.0, q.xh, nrhs, smem);
    } else {
        block_gemm(q.k, nrhs, q.kl, 1.0, q.U, 1, q.k, q.xh_l, nrhs, 1, 0.0, q.xh, nrhs, smem);
        block_gemm(q.k, nrhs, q.kr, 1.0, q.U + (int64_t)q.kl * q.k, 1, q.k, q.xh_r, nrhs, 1, 1.0, q.xh, nrhs, smem);
    }
}

// Non-leaf p: children's y^ from the coupling and from p's own y^.
__global__ __launch_bounds__(BG_T) void k_mv_down(const MvDesc *dsc, int nrhs) {
    __shared__ double smem[2 * 16 * 65];
    const MvDesc q = dsc[blockIdx.x];
    if (q.leaf) return;
    const double beta = q.root ? 0.0 : 1.0;
    if (!q.root) {
        // y^_children = U_p y^_p (written first), then the coupling terms are added
        block_gemm(q.kl, nrhs, q.k, 1.0, q.U, q.k, 1, q.yh, nrhs, 1, 0.0, q.yh_l, nrhs, smem);
        block_gemm(q.kr, nrhs, q.k, 1.0, q.U + (int64_t)q.kl * q.k, q.k, 1, q.yh, nrhs, 1, 0.0, q.yh_r, nrhs, smem);
    }
    block_gemm(q.kl, nrhs, q.kr, 1.0, q.B, q.kr, 1, q.xh_r, nrhs, 1, beta, q.yh_l, nrhs, smem);
    block_gemm(q.kr, nrhs, q.kl, 1.0, q.B, 1, q.kr, q.xh_l, nrhs, 1, beta, q.yh_r, nrhs, smem);
}

__global__ __launch_bounds__(BG_T) void k_mv_leaf(const MvDesc *dsc, const double *__restrict__ x, int nrhs,
                                                  double *__restrict__ y) {
    __shared__ double smem[2 * 16 * 65];
    const MvDesc q = dsc[blockIdx.x];
    if (!q.leaf) return;
    block_gemm(q.m, nrhs, q.m, 1.0, q.D, q.m, 1, x + q.b * nrhs, nrhs, 1, 0.0, y + q.b * nrhs, nrhs, smem);
    if (!q.root && q.k > 0)
        block_gemm(q.m, nrhs, q.k, 1.0, q.U, q.k, 1, q.yh, nrhs, 1, 1.0, y + q.b * nrhs, nrhs, smem);
}

}  // namespace

void hss_matvec_impl(const hss_s *H, const double *x, int nrhs, double *y, hipStream_t s) {
    const int nn = (int)H->node.size();
    std::vector<int64_t> off(nn);
    int64_t tot = 0;
    for (int i = 0; i < nn; ++i) {
        off[i] = tot;
        tot += (int64_t)(H->node[i].parent < 0 ? 0 : H->node[i].k) * nrhs;
    }
    DBuf xh = dalloc<double>(std::max<int64_t>(tot, 1)), yh = dalloc<double>(std::max<int64_t>(tot, 1));
    std::vector<MvDesc> all(nn);
    for (int i = 0; i < nn; ++i) {
        const HNode &q = H->node[i];
        MvDesc &d = all[i];
        std::memset(&d, 0, sizeof d);
        d.leaf = q.left < 0;
        d.root = q.parent < 0;
        d.m = q.m;
        d.k = d.root ? 0 : q.k;
        d.b = q.b;
        d.U = q.offU >= 0 ? H->U.as<double>() + q.offU : nullptr;
        d.D = q.offD >= 0 ? H->D.as<double>() + q.offD : nullptr;
        d.B = q.offB >= 0 ? H->B.as<double>() + q.offB : nullptr;
        d.xh = xh.as<double>() + off[i];
        d.yh = yh.as<double>() + off[i];
        if (!d.leaf) {
            d.kl = H->node[q.left].k;
            d.kr = H->node[q.right].k;
            d.xh_l = xh.as<double>() + off[q.left];
            d.xh_r = xh.as<double>() + off[q.right];
            d.yh_l = yh.as<double>() + off[q.left];
            d.yh_r = yh.as<double>() + off[q.right];
        }
        if (d.leaf) d.m = (int32_t)(q.e - q.b);
    }
    std::vector<std::vector<MvDesc>> hold;
    std::vector<DBuf> keep;
    for (const auto &lv : H->levels) {
        hold.emplace_back();
        for (int id : lv) hold.back().push_back(all[id]);
        keep.push_back(upload(hold.back(), s));
        k_mv_up<<<(unsigned)lv.size(), BG_T, 0, s>>>(keep.back().as<MvDesc>(), x, nrhs);
        check_launch("k_mv_up");
    }
    for (int h = (int)H->levels.size() - 1; h >= 0; --h) {
        k_mv_down<<<(unsigned)H->levels[h].size(), BG_T, 0, s>>>(keep[h].as<MvDesc>(), nrhs);
        check_launch("k_mv_down");
    }
    if (!H->levels.empty()) {
        k_mv_leaf<<<(unsigned)H->levels[0].size(), BG_T, 0, s>>>(keep[0].as<MvDesc>(), x, nrhs, y);
        check_launch("k_mv_leaf");
    }
    sync(s);
}

}  // namespace krr
