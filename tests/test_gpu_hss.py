"""GPU HSS compression, ULV factorization / solve, refinement and fit.

Compression is compared with the oracle's randomized construction run on the
very same random block (read back from the device) and with the plain
definition K; the ULV solve is compared with a dense Cholesky solve of the
exported GPU HSS (independent of the compression's randomness)."""
import numpy as np
import pytest
import torch

import synthdata as sd
from oracle import cluster as oc, cmath, hss as oh, kernel as ok

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _as_oracle(ex, nodes):
    H = oh.HSS(nodes=nodes[:, :4])
    H.U, H.D, H.B, H.J = ex["U"], ex["D"], ex["B"], ex["J"]
    return H


def _compress(krr, X, leaf, h, rtol, prec="f64", r0=256, seed=3, tree_seed=1, **kw):
    t = oc.cluster2mn(X, leaf, tree_seed)
    Xp = np.ascontiguousarray(X[t.perm])
    tree = krr.tree_from_nodes(t.nodes)
    opts = krr.HssOptions(rtol=rtol, r0=r0, dr=kw.pop("dr", 64), r_max=kw.pop("r_max", 2048),
                          oversample=kw.pop("oversample", 10), prec=prec, seed=seed, **kw)
    H = krr.HSS(tree, _t(Xp), h, opts)
    return t, Xp, H


@pytest.mark.parametrize("rtol", [1e-6, 1e-3])
def test_compress_matches_oracle_randomized(gpu_lib, rtol):
    p = sd.c1_two_gaussians()
    t, Xp, H = _compress(gpu_lib, p.X, p.leaf, p.h, rtol)
    ex = H.export()
    G = _as_oracle(ex, t.nodes)
    K = ok.kernel_dense(Xp, Xp, p.h)
    err_gpu = np.linalg.norm(K - oh.assemble(G)) / np.linalg.norm(K)
    r = H.stats.r_final
    R = gpu_lib.random_block(3, p.n, r).cpu().numpy().astype(np.float64)
    Ho = oh.randomized(Xp, t.nodes, p.h, rtol, R, K=K)
    err_or = np.linalg.norm(K - oh.assemble(Ho)) / np.linalg.norm(K)
    ranks_gpu = np.array([ex["U"][i].shape[1] for i in sorted(ex["U"])])
    ranks_or = np.array([Ho.U[i].shape[1] for i in sorted(Ho.U)])
    assert err_gpu <= 2 * err_or + 1e-14
    assert err_gpu <= 20 * rtol
    assert np.max(np.abs(ranks_gpu - ranks_or)) <= 2
    # generators: D and B are kernel entries, J are positions inside the node
    for i, D in ex["D"].items():
        b, e = t.nodes[i, :2]
        np.testing.assert_allclose(D, K[b:e, b:e], rtol=1e-14, atol=1e-15)
    for i, Jv in ex["J"].items():
        b, e = t.nodes[i, :2]
        assert np.all((Jv >= b) & (Jv < e))
    assert H.stats.max_rank == max(ranks_gpu.max(), 0)


def test_compress_limits(gpu_lib):
    p = sd.c1_two_gaussians(n=600, m=1)
    # h -> 0: every off-diagonal block is exactly zero, all ranks 0
    t, Xp, H = _compress(gpu_lib, p.X, 40, 1e-3, 1e-6)
    assert H.stats.max_rank == 0
    np.testing.assert_array_equal(oh.assemble(_as_oracle(H.export(), t.nodes)), np.eye(600))
    # h -> infinity: ranks at most d + 2
    t, Xp, H = _compress(gpu_lib, p.X, 40, 100.0, 1e-4)
    assert 1 <= H.stats.max_rank <= p.d + 2


def test_adaptive_growth(gpu_lib):
    p = sd.c1_two_gaussians(n=1000, m=1)
    t, Xp, H = _compress(gpu_lib, p.X, 64, p.h, 1e-6, r0=64, dr=32)
    assert H.stats.regrowths >= 1 and H.stats.r_final > 64
    assert H.stats.max_rank <= H.stats.r_final - 10
    K = ok.kernel_dense(Xp, Xp, p.h)
    err = np.linalg.norm(K - oh.assemble(_as_oracle(H.export(), t.nodes))) / np.linalg.norm(K)
    assert err <= 20e-6


def test_rank_cap_error(gpu_lib):
    p = sd.c1_two_gaussians(n=1000, m=1)
    with pytest.raises(gpu_lib.KrrError) as e:
        _compress(gpu_lib, p.X, 64, p.h, 1e-9, r0=64, dr=32, r_max=96)
    assert e.value.code == -4


@pytest.mark.parametrize("lam", [1.0, 0.05])
def test_ulv_matches_dense_solve_of_exported_hss(gpu_lib, lam):
    p = sd.c1_two_gaussians()
    t, Xp, H = _compress(gpu_lib, p.X, p.leaf, p.h, 1e-4)
    G = _as_oracle(H.export(), t.nodes)
    F = gpu_lib.ULV(H, lam)
    B = np.column_stack([p.y[t.perm], sd.vectors(p.n, 2, seed=4)])
    got = F.solve(_t(B)).cpu().numpy()
    ref = oh.solve_dense(G, lam, B)
    A = oh.assemble(G) + lam * np.eye(p.n)
    cond = np.linalg.cond(A)
    assert np.linalg.norm(got - ref) <= 1e-13 * cond * np.linalg.norm(ref)


def test_ulv_single_leaf_and_exact(gpu_lib):
    # n <= leaf: one node, the ULV solve is a dense Cholesky solve
    p = sd.c1_two_gaussians(n=50, m=1)
    t, Xp, H = _compress(gpu_lib, p.X, 64, p.h, 1e-6)
    assert t.n_nodes == 1
    got = gpu_lib.ULV(H, 0.7).solve(_t(p.y[t.perm])).cpu().numpy()
    np.testing.assert_allclose(got, ok.krr_fit_dense(Xp, p.y[t.perm], p.h, 0.7), rtol=1e-12)
    # rtol = 0 with a full sample: exact HSS, the ULV solve equals the dense KRR solve
    p = sd.c1_two_gaussians(n=400, m=1)
    t, Xp, H = _compress(gpu_lib, p.X, 32, p.h, 0.0, r0=416, oversample=0)
    y = p.y[t.perm]
    got = gpu_lib.ULV(H, p.lam).solve(_t(y)).cpu().numpy()
    ref = ok.krr_fit_dense(Xp, y, p.h, p.lam)
    assert np.linalg.norm(got - ref) <= 1e-9 * np.linalg.norm(ref)


def test_lambda_refactor_without_recompression(gpu_lib):
    # Section 5.3: a new lambda changes only the diagonal; the same HSS serves both
    p = sd.c1_two_gaussians()
    t, Xp, H = _compress(gpu_lib, p.X, p.leaf, p.h, 1e-5)
    G = _as_oracle(H.export(), t.nodes)
    y = p.y[t.perm]
    for lam in (0.3, 3.0):
        got = gpu_lib.ULV(H, lam).solve(_t(y)).cpu().numpy()
        np.testing.assert_allclose(got, oh.solve_dense(G, lam, y), rtol=1e-9, atol=1e-12)


def test_small_config_fit_and_accuracy(gpu_lib):
    # the n = 1000 two-Gaussian workload: FP64 sampling, rtol 1e-6, ULV solve
    p = sd.c1_two_gaussians()
    X = _t(p.X)
    res = gpu_lib.fit(X, _t(p.y), p.h, p.lam, leaf=p.leaf,
                      opts=gpu_lib.HssOptions(rtol=p.rtol, prec="f64", r0=256),
                      refine_solution=False)
    a_ref = ok.krr_fit_dense(p.X, p.y, p.h, p.lam)
    a = res.alpha.cpu().numpy()
    assert np.linalg.norm(a - a_ref) / np.linalg.norm(a_ref) <= 1e-4
    sc, lab = gpu_lib.predict(_t(p.Xt), res.Xp, p.h, res.alpha_perm, prec="f64")
    ref_scores = ok.scores(p.Xt, p.X, a_ref, p.h)
    acc_gpu = ok.accuracy(lab.cpu().numpy(), p.yt)
    acc_ref = ok.accuracy(ok.labels_binary(ref_scores), p.yt)
    assert abs(acc_gpu - acc_ref) <= 1.0 / 200 + 1e-12
    confident = np.abs(ref_scores) > 1e-3 * np.abs(ref_scores).max()
    assert np.all(lab.cpu().numpy()[confident] == ok.labels_binary(ref_scores)[confident])


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_refined_fit_reaches_tolerance(gpu_lib, prec):
    # 16-Gaussian workload at a reduced size: reduced-precision sampling,
    # PCG with the ULV preconditioner on the FP32 kernel product; the FP64
    # oracle certifies the residual and compares alpha with the dense solve
    p = sd.c2_sixteen_gaussians(n=8192, m=2000)
    res = gpu_lib.fit(_t(p.X), _t(p.y), p.h, p.lam, leaf=128,
                      opts=gpu_lib.HssOptions(rtol=1e-2, prec=prec, r0=256), tol=1e-6)
    a = res.alpha.cpu().numpy()
    rr = cmath.residual(p.X, a, p.y, p.h, p.lam)
    assert np.linalg.norm(rr) / np.linalg.norm(p.y) <= 1.5e-6
    a_ref = ok.krr_fit_dense(p.X, p.y, p.h, p.lam)
    assert np.linalg.norm(a - a_ref) / np.linalg.norm(a_ref) <= 1e-4
    assert res.info["refine"]["converged"]


def test_hss_matvec_matches_assembled(gpu_lib):
    p = sd.c1_two_gaussians()
    t, Xp, H = _compress(gpu_lib, p.X, p.leaf, p.h, 1e-3)
    A = oh.assemble(_as_oracle(H.export(), t.nodes))
    x = sd.vectors(p.n, 3, seed=21)
    got = H.matvec(_t(x)).cpu().numpy()
    np.testing.assert_allclose(got, A @ x, rtol=1e-12, atol=1e-12 * np.abs(A @ x).max())


def test_ulv_graph_replays_match_eager(gpu_lib):
    # the captured solve graph replayed several times, with other device work
    # and synchronizations in between, gives exactly the direct launches' result
    p = sd.c1_two_gaussians()
    t, Xp, H = _compress(gpu_lib, p.X, p.leaf, p.h, 1e-4)
    F = gpu_lib.ULV(H, p.lam)
    for nrhs in (1, 3):
        Bs = [_t(sd.vectors(p.n, nrhs, seed=20 + i)) for i in range(4)]
        F.use_graph(False)
        eager = [F.solve(B).clone() for B in Bs]
        F.use_graph(True)
        for rep in range(3):
            for i, B in enumerate(Bs):
                junk = torch.randn(1 << 16, device="cuda").sum()  # unrelated work on the stream
                got = F.solve(B)
                torch.cuda.synchronize()
                assert torch.equal(got, eager[i]), (nrhs, rep, i)
                del junk
        # in place (B and the solution share memory)
        B = Bs[0].clone()
        F.solve(B, out=B)
        assert torch.equal(B, eager[0])
