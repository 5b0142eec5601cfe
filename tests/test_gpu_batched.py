"""The batched form: many independent problems stored one after the other.

The kernel matrix of a batch is block diagonal, so the oracle of a batch is
the oracle of each problem alone: the 2MN forest tree by tree (bit-exact,
positions shifted by the problem's offset), the sampling product and kernel
product per problem, the compression against the oracle's randomized
construction on the problem's rows of the same random block, the ULV solve
against a dense solve of each exported problem, and the fitted coefficients
against the dense KRR solution of each problem with its own h and lambda."""
import numpy as np
import pytest
import torch

import synthdata as sd
from gpu_util import fp32_product_bound, leaf_ranges, mfma_sample_bound
from oracle import cluster as oc, cmath, hss as oh, kernel as ok

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _problems(count=7, n_lo=40, n_hi=1500, d=8, dtype=np.float32, seed=5):
    """A ragged batch of the two-Gaussian problems (sizes log-uniform, one
    below the leaf size so that its tree is a single leaf)."""
    ps = sd.c4_ragged_batch(count=count, n_lo=n_lo, n_hi=n_hi, dims=(d,), m=16, config=seed)
    ps[0].X, ps[0].y = ps[0].X[:50], ps[0].y[:50]
    for p in ps:
        p.X = np.ascontiguousarray(p.X.astype(dtype))
    return ps


def _concat(ps):
    X = np.concatenate([p.X for p in ps], 0)
    off = np.zeros(len(ps) + 1, dtype=np.int64)
    off[1:] = np.cumsum([p.X.shape[0] for p in ps])
    return X, off


def _tree_part(nodes, roots, k, off):
    """Nodes of tree k of a forest, renumbered as a tree of its own."""
    first = 0 if k == 0 else roots[k - 1] + 1
    sub = nodes[first:roots[k] + 1].copy()
    sub[:, :2] -= off[k]
    for c in (2, 3, 4):
        sub[:, c] = np.where(sub[:, c] >= 0, sub[:, c] - first, -1)
    return sub


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_forest_clustering_is_each_problem_alone(gpu_lib, dtype):
    ps = _problems(dtype=dtype)
    X, off = _concat(ps)
    perm, tree = gpu_lib.cluster_2mn_batched(_t(X), off, 64, 11)
    perm = perm.cpu().numpy()
    assert len(tree.roots) == len(ps)
    for k, p in enumerate(ps):
        t = oc.cluster2mn(p.X, 64, 11)
        np.testing.assert_array_equal(perm[off[k]:off[k + 1]] - off[k], t.perm)
        np.testing.assert_array_equal(_tree_part(tree.nodes, tree.roots, k, off), t.nodes)


@pytest.mark.parametrize("prec,split", [("f64", 1), ("f32", 1), ("f16", 2), ("bf16", 2)])
def test_batched_sample_per_problem(gpu_lib, prec, split):
    ps = _problems()
    X, off = _concat(ps)
    perm, tree = gpu_lib.cluster_2mn_batched(_t(X), off, 64, 3)
    Xp = X[perm.cpu().numpy()]
    lb, le = leaf_ranges(tree.nodes, X.shape[0])
    r = 64
    R = sd.random_block(X.shape[0], r, seed=4)
    hs = [p.h for p in ps]
    S = gpu_lib.kernel_sample_batched(_t(Xp), off, hs, _t(R), _t(lb), _t(le), prec=prec,
                                      split_terms=split).cpu().numpy()
    for k, p in enumerate(ps):
        a, b = off[k], off[k + 1]
        Xk, Rk = Xp[a:b], R[a:b]
        lbk, lek = lb[a:b] - a, le[a:b] - a
        rows = np.arange(b - a)
        ref = cmath.sample_masked(Xk, Rk, p.h, lbk, lek, rows)
        if prec == "f64":
            np.testing.assert_allclose(S[a:b], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
        else:
            bound = mfma_sample_bound(Xk, Rk, p.h, lbk, lek, prec, split, rows)
            assert np.all(np.abs(S[a:b] - ref) <= bound), k


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batched_matvec_per_problem(gpu_lib, prec):
    ps = _problems(d=18, n_hi=1200)
    X, off = _concat(ps)
    W = sd.vectors(X.shape[0], 3, seed=8)
    hs = [p.h for p in ps]
    out = gpu_lib.kernel_matvec_batched(_t(X), off, hs, _t(W), prec=prec).cpu().numpy()
    for k, p in enumerate(ps):
        a, b = off[k], off[k + 1]
        ref = cmath.kmv(X[a:b], X[a:b], W[a:b], p.h)
        if prec == "f64":
            np.testing.assert_allclose(out[a:b], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
        else:
            bound = fp32_product_bound(X[a:b], X[a:b], W[a:b], p.h)
            assert np.all(np.abs(out[a:b] - ref) <= bound), k


def _compress_batch(krr, ps, leaf, rtol, prec="f64", r0=256, seed=3):
    X, off = _concat(ps)
    perm, tree = krr.cluster_2mn_batched(_t(X), off, leaf, 1)
    Xp = np.ascontiguousarray(X[perm.cpu().numpy()])
    opts = krr.HssOptions(rtol=rtol, r0=r0, dr=64, r_max=2048, prec=prec, seed=seed)
    H = krr.BatchedHSS(tree, _t(Xp), [p.h for p in ps], opts)
    return X, off, Xp, tree, H


def _split_export(ex, tree, off, k):
    """Generators of problem k (node indices and positions of its own)."""
    roots = tree.roots
    first = 0 if k == 0 else roots[k - 1] + 1
    nodes = _tree_part(tree.nodes, roots, k, off)
    G = oh.HSS(nodes=nodes[:, :4])
    G.U = {i - first: u for i, u in ex["U"].items() if first <= i <= roots[k]}
    G.D = {i - first: dm for i, dm in ex["D"].items() if first <= i <= roots[k]}
    G.B = {i - first: bm for i, bm in ex["B"].items() if first <= i <= roots[k]}
    G.J = {i - first: j - off[k] for i, j in ex["J"].items() if first <= i <= roots[k]}
    return nodes, G


def test_batched_compress_matches_oracle_per_problem(gpu_lib):
    ps = _problems(dtype=np.float64, n_hi=900)
    rtol = 1e-6
    X, off, Xp, tree, H = _compress_batch(gpu_lib, ps, 64, rtol)
    ex = H.export()
    r = H.stats.r_final
    R = gpu_lib.random_block(3, X.shape[0], r).cpu().numpy().astype(np.float64)
    for k, p in enumerate(ps):
        a, b = off[k], off[k + 1]
        nodes, G = _split_export(ex, tree, off, k)
        K = ok.kernel_dense(Xp[a:b], Xp[a:b], p.h)
        err_gpu = np.linalg.norm(K - oh.assemble(G)) / np.linalg.norm(K)
        Ho = oh.randomized(Xp[a:b], nodes, p.h, rtol, R[a:b], K=K)
        err_or = np.linalg.norm(K - oh.assemble(Ho)) / np.linalg.norm(K)
        # the GPU takes each ID from the Gram matrix of the sample rows (pivoted
        # Cholesky); its backward error grows like u kappa(R11), and the rank
        # rule bounds kappa(R11) by 1 / rtol: where the oracle's construction
        # is exact (every rank full) the GPU's differs by up to ~u / rtol
        assert err_gpu <= 2 * err_or + 100 * 2.0 ** -53 / rtol, k
        assert err_gpu <= 20 * rtol, k
        ranks_gpu = np.array([G.U[i].shape[1] for i in sorted(G.U)], dtype=np.int64)
        ranks_or = np.array([Ho.U[i].shape[1] for i in sorted(Ho.U)], dtype=np.int64)
        assert ranks_gpu.shape == ranks_or.shape
        if ranks_gpu.size:
            assert np.max(np.abs(ranks_gpu - ranks_or)) <= 2, k
        for i, D in G.D.items():
            nb, ne = nodes[i, :2]
            np.testing.assert_allclose(D, K[nb:ne, nb:ne], rtol=1e-14, atol=1e-15)


def test_batched_ulv_matches_dense_per_problem(gpu_lib):
    ps = _problems(dtype=np.float64, n_hi=900)
    X, off, Xp, tree, H = _compress_batch(gpu_lib, ps, 64, 1e-4)
    lams = [p.lam for p in ps]
    F = gpu_lib.BatchedULV(H, lams)
    B = sd.vectors(X.shape[0], 2, seed=12)
    got = F.solve(_t(B)).cpu().numpy()
    ex = H.export()
    for k, p in enumerate(ps):
        a, b = off[k], off[k + 1]
        _, G = _split_export(ex, tree, off, k)
        ref = oh.solve_dense(G, p.lam, B[a:b])
        cond = np.linalg.cond(oh.assemble(G) + p.lam * np.eye(b - a))
        assert np.linalg.norm(got[a:b] - ref) <= 1e-13 * cond * np.linalg.norm(ref), k


@pytest.mark.parametrize("prec,mv", [("f64", "f64"), ("f16", "f32")])
def test_fit_batched_matches_dense_krr(gpu_lib, prec, mv):
    # two groups of different dimension, each a batch of its own
    ps = _problems(count=5, d=8, n_hi=1200, seed=6) + _problems(count=4, d=18, n_hi=1200, seed=7)
    tol = 1e-10 if mv == "f64" else 1e-6
    probs = [(_t(p.X), _t(p.y), p.h, p.lam) for p in ps]
    res = gpu_lib.fit_batched(probs, leaf=64, opts=gpu_lib.HssOptions(rtol=1e-3, r0=128, prec=prec, atol=0.0),
                              tol=tol, max_iter=300, mv_prec=mv)
    assert len(res.groups) == 2
    for rf in res.info["refine"]:
        assert rf["converged"] and np.all(rf["relres"] <= tol)
    for k, p in enumerate(ps):
        a = res.alphas[k].cpu().numpy()
        ref = ok.krr_fit_dense(p.X.astype(np.float64), p.y, p.h, p.lam)
        # the coefficients of a residual-tol solve are within cond * tol
        K = ok.kernel_dense(p.X.astype(np.float64), p.X.astype(np.float64), p.h)
        cond = np.linalg.cond(K + p.lam * np.eye(K.shape[0]))
        err = np.linalg.norm(a - ref) / np.linalg.norm(ref)
        slack = 10.0 if mv == "f64" else 50.0  # FP32 products: residual measured in FP32 arithmetic
        assert err <= slack * cond * tol, (k, err, cond)


def test_batched_refine_without_preconditioner(gpu_lib):
    ps = _problems(count=4, d=8, n_hi=700, dtype=np.float64, seed=9)
    X, off = _concat(ps)
    y = np.concatenate([p.y for p in ps])
    alpha = torch.zeros(X.shape[0], dtype=torch.float64, device="cuda")
    st = gpu_lib.refine_batched(None, _t(X), off, [p.h for p in ps], [p.lam for p in ps], _t(y), alpha,
                                tol=1e-10, max_iter=500, mv_prec="f64")
    assert st["converged"]
    a = alpha.cpu().numpy()
    for k, p in enumerate(ps):
        ref = ok.krr_fit_dense(p.X, p.y, p.h, p.lam)
        assert np.linalg.norm(a[off[k]:off[k + 1]] - ref) <= 1e-7 * np.linalg.norm(ref), k


def test_batched_shift_per_problem(gpu_lib):
    # one problem whose truncated compression needs a diagonal shift to factor
    # (16-Gaussian data, rank capped at r - p) beside one with K = I exactly
    # (h -> 0): only the first is shifted, and each problem's factor solves
    # its own K_hss + lambda_k (1 + s_k) I
    hard = sd.c2_sixteen_gaussians(n=16384, m=1)
    easy = sd.c1_two_gaussians(n=1000, m=1)
    X = np.concatenate([hard.X, easy.X.astype(np.float32)])
    off = np.array([0, 16384, 17384], dtype=np.int64)
    hs = [hard.h, 1e-3]
    lams = [hard.lam, 0.5]
    perm, tree = gpu_lib.cluster_2mn_batched(_t(X), off, 128, 7)
    Xp = X[perm.cpu().numpy()]
    opts = gpu_lib.HssOptions(rtol=1e-2, atol=3.0, r0=128, dr=128, r_max=128, prec="f16", cap_policy=1)
    H = gpu_lib.BatchedHSS(tree, _t(Xp), hs, opts)
    F = gpu_lib.BatchedULV(H, lams, shifted=True)
    s = F.shift_mults
    assert s[1] == 0.0
    B = sd.vectors(X.shape[0], 2, seed=3)
    x = F.solve(_t(B))
    r = (H.matvec(x)).cpu().numpy() - B
    xs = x.cpu().numpy()
    for k in range(2):
        a, b = off[k], off[k + 1]
        rk = r[a:b] + lams[k] * (1.0 + s[k]) * xs[a:b]
        assert np.linalg.norm(rk) <= 1e-9 * np.linalg.norm(B[a:b]), (k, s)
    # the easy problem is the identity plus its lambda: x = b / (1 + lambda)
    np.testing.assert_allclose(xs[off[1]:], B[off[1]:] / (1.0 + lams[1]), rtol=1e-13)


def test_batched_symmetric_matvec_per_problem(gpu_lib):
    # d = 8: the batched product takes the symmetric path (each problem's
    # off-diagonal entries once), with per-problem widths
    ps = _problems(d=8, n_hi=3000, seed=11)
    X, off = _concat(ps)
    W = sd.vectors(X.shape[0], 1, seed=2)
    out = gpu_lib.kernel_matvec_batched(_t(X), off, [p.h for p in ps], _t(W), prec="f32").cpu().numpy()
    for k, p in enumerate(ps):
        a, b = off[k], off[k + 1]
        ref = cmath.kmv(X[a:b], X[a:b], W[a:b], p.h)
        assert np.all(np.abs(out[a:b] - ref) <= fp32_product_bound(X[a:b], X[a:b], W[a:b], p.h)), k


def test_batched_wide_sample_per_problem(gpu_lib):
    # a batch of wide points (d = 100) through the matrix-core wide sampler
    ps = _problems(count=4, d=8, n_hi=900, seed=13)
    rng = np.random.default_rng(1)
    for p in ps:  # widen each problem's points to d = 100 (seeded extra coordinates)
        p.X = np.ascontiguousarray(np.concatenate([p.X, 0.3 * rng.standard_normal((p.X.shape[0], 92))], 1)
                                   .astype(np.float32))
        p.h = 0.4 * np.sqrt(100) * (0.5 + p.h / 2)
    X, off = _concat(ps)
    perm, tree = gpu_lib.cluster_2mn_batched(_t(X), off, 64, 3)
    Xp = X[perm.cpu().numpy()]
    lb, le = leaf_ranges(tree.nodes, X.shape[0])
    R = sd.random_block(X.shape[0], 64, seed=5)
    S = gpu_lib.kernel_sample_batched(_t(Xp), off, [p.h for p in ps], _t(R), _t(lb), _t(le), prec="f16",
                                      split_terms=2).cpu().numpy()
    mean = Xp.astype(np.float64).mean(axis=0)
    for k, p in enumerate(ps):
        a, b = off[k], off[k + 1]
        Xk, Rk = Xp[a:b], R[a:b]
        lbk, lek = lb[a:b] - a, le[a:b] - a
        rows = np.arange(b - a)
        ref = cmath.sample_masked(Xk, Rk, p.h, lbk, lek, rows)
        bound = mfma_sample_bound(Xk, Rk, p.h, lbk, lek, "f16", 2, rows, anchor=mean)
        assert np.all(np.abs(S[a:b] - ref) <= bound), k


def test_fit_batched_wide_group_with_ranks(gpu_lib):
    # the d = 54 group of the ragged batch through the D = 64 sampler with an
    # h large enough (h^2 about half the within-cluster squared distance) that
    # the off-diagonal blocks have rank: the compressed ranks are not all zero,
    # and every problem's coefficients match dense KRR
    ps = _problems(count=3, d=54, n_lo=1500, n_hi=3000, seed=14)
    for p in ps:
        p.h = 4.0 + p.h  # h in [4.5, 6]: within-cluster K ~ exp(-108 / 2 h^2) in 0.07 .. 0.22
    probs = [(_t(p.X), _t(p.y), p.h, p.lam) for p in ps]
    tol = 1e-6
    res = gpu_lib.fit_batched(probs, leaf=128, opts=gpu_lib.HssOptions(rtol=1e-3, r0=128, prec="f16", atol=0.0),
                              tol=tol, max_iter=300, mv_prec="f32")
    assert len(res.groups) == 1
    assert res.info["hss"][0]["max_rank"] > 0
    for rf in res.info["refine"]:
        assert rf["converged"] and np.all(rf["relres"] <= tol)
    for k, p in enumerate(ps):
        a = res.alphas[k].cpu().numpy()
        Xd = p.X.astype(np.float64)
        ref = ok.krr_fit_dense(Xd, p.y, p.h, p.lam)
        K = ok.kernel_dense(Xd, Xd, p.h)
        cond = np.linalg.cond(K + p.lam * np.eye(K.shape[0]))
        err = np.linalg.norm(a - ref) / np.linalg.norm(ref)
        assert err <= 50.0 * cond * tol, (k, err, cond)


def test_fit_batched_top_of_size_range(gpu_lib):
    # a problem at the top of the ragged batch's size range (n = 32,767)
    # beside two small ones; the FP64 residual of every problem's
    # coefficients is recomputed by the oracle over all rows
    big = sd.c4_ragged_batch(count=1, n_lo=32768, n_hi=32768, dims=(8,), m=16, config=15)[0]
    small = _problems(count=2, d=8, n_lo=400, n_hi=2000, seed=16)
    ps = [big] + small
    probs = [(_t(p.X), _t(p.y), p.h, p.lam) for p in ps]
    tol = 1e-6
    res = gpu_lib.fit_batched(probs, leaf=128, opts=gpu_lib.HssOptions(rtol=1e-2, r0=256, prec="f16"),
                              tol=tol, max_iter=300, mv_prec="f32")
    for rf in res.info["refine"]:
        assert rf["converged"] and np.all(rf["relres"] <= tol)
    for k, p in enumerate(ps):
        a = res.alphas[k].cpu().numpy()
        r = cmath.residual(p.X, a, p.y, p.h, p.lam)
        # FP32-entry products stop the solve at 1e-6; in FP64 the residual is
        # within the products' error, ~1e-7 of |K||alpha| / |y|
        assert np.linalg.norm(r) <= 2e-6 * np.linalg.norm(p.y), k


@pytest.mark.parametrize("mv", ["f32", "f64"])
def test_batched_refine_leaves_out_converged_problems(gpu_lib, mv):
    # problems that converge at very different rates in one batch: a nearly
    # diagonal kernel (h = 0.05: a few iterations) beside smooth, weakly
    # regularised ones (lambda = 0.1: many).  Once a problem has converged the
    # batched products leave it out (its rows of the product are not
    # computed); every problem still reaches the tolerance and matches dense
    # KRR, including the d > 64 and FP64 product paths through mv
    ps = _problems(count=4, d=8, n_lo=600, n_hi=1200, seed=13)
    ps[0].h, ps[0].lam = 0.05, 1.0
    for p in ps[1:]:
        p.h, p.lam = 1.5, 0.1
    tol = 1e-6 if mv == "f32" else 1e-10
    probs = [(_t(p.X), _t(p.y), p.h, p.lam) for p in ps]
    res = gpu_lib.fit_batched(probs, leaf=64, opts=gpu_lib.HssOptions(rtol=1e-2, r0=64, prec="f16", atol=0.0),
                              tol=tol, max_iter=400, mv_prec=mv)
    rf = res.info["refine"][0]
    assert rf["converged"] and np.all(rf["relres"] <= tol)
    for k, p in enumerate(ps):
        a = res.alphas[k].cpu().numpy()
        ref = ok.krr_fit_dense(p.X.astype(np.float64), p.y, p.h, p.lam)
        K = ok.kernel_dense(p.X.astype(np.float64), p.X.astype(np.float64), p.h)
        cond = np.linalg.cond(K + p.lam * np.eye(K.shape[0]))
        err = np.linalg.norm(a - ref) / np.linalg.norm(ref)
        assert err <= (50.0 if mv == "f32" else 10.0) * cond * tol, (k, err, cond)
