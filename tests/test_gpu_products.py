"""GPU kernel products against the oracle's FP64 matrix-free products:
kernel_matvec (FP64 and FP32 entries), the masked sampling product, the
random block, gather / scatter, prediction labels and the matvec backward."""
import numpy as np
import pytest
import torch

import synthdata as sd
from oracle import cmath, grad as og, cluster as oc, kernel as ok
from gpu_util import (fp32_product_bound, fp32_sym_anchored_bound, fp32_wide_product_bound, fp64_wide_product_bound,
                      leaf_ranges, negligible_mass, sqdist, sym_rows_per_block, U32)

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("d", [8, 18, 54, 100, 784])
@pytest.mark.parametrize("nrhs", [1, 5, 17])
def test_matvec_fp64(gpu_lib, d, nrhs):
    X = sd.points(301, d, seed=1, scale=0.3, dtype=np.float64)
    Y = sd.points(517, d, seed=2, scale=0.3, dtype=np.float64)
    W = sd.vectors(517, nrhs, seed=3)
    h = 0.2 * np.sqrt(d)
    got = gpu_lib.kernel_matvec(_t(X), _t(Y), h, _t(W), prec="f64").cpu().numpy()
    ref = cmath.kmv(X, Y, W, h)
    if d <= 64:  # exact coordinate differences
        scale = cmath.kmv(X, Y, np.abs(W), h)
        assert np.all(np.abs(got - ref) <= 1e-13 * scale + 1e-300)
    else:  # FP64 matrix-core norm expansion on centred coordinates
        assert np.all(np.abs(got - ref) <= fp64_wide_product_bound(X, Y, W, h))


@pytest.mark.parametrize("xdtype", [np.float32, np.float64])
def test_matvec_fp64_wide_batched_and_ragged(gpu_lib, xdtype):
    # FP64 entries of wide points: three problems of ragged sizes (row blocks
    # of 128, panels of 128 points), per-problem widths, 20 right-hand sides
    # (a pass of 16 and one of 4)
    sizes, d = [130, 7, 300], 100
    rng = np.random.default_rng(4)
    Xs = [(0.3 * rng.standard_normal((k, d))).astype(xdtype) for k in sizes]
    hs = [2.0, 3.0, 2.5]
    X = np.concatenate(Xs)
    off = np.concatenate([[0], np.cumsum(sizes)])
    W = sd.vectors(X.shape[0], 20, seed=5)
    got = gpu_lib.kernel_matvec_batched(_t(X), off, hs, _t(W), prec="f64").cpu().numpy()
    for k in range(3):
        a, b = off[k], off[k + 1]
        ref = cmath.kmv(Xs[k], Xs[k], W[a:b], hs[k])
        # the batch centres every problem on the mean of all points
        bound = fp64_wide_product_bound(Xs[k], Xs[k], W[a:b], hs[k], anchor=X.astype(np.float64).mean(axis=0))
        assert np.all(np.abs(got[a:b] - ref) <= bound), k


@pytest.mark.parametrize("d", [8, 18, 54, 784])
@pytest.mark.parametrize("nrhs", [1, 2, 10])
def test_matvec_fp32(gpu_lib, d, nrhs):
    X = sd.points(333, d, seed=4, scale=0.3)
    Y = sd.points(1029, d, seed=5, scale=0.3)
    W = sd.vectors(1029, nrhs, seed=6)
    h = 0.2 * np.sqrt(d)
    got = gpu_lib.kernel_matvec(_t(X), _t(Y), h, _t(W), prec="f32").cpu().numpy()
    ref = cmath.kmv(X, Y, W, h)
    # points wider than 64 take the matrix-core exponent GEMM on centred coordinates
    bound = fp32_product_bound(X, Y, W, h) if d <= 64 else fp32_wide_product_bound(X, Y, W, h)
    assert np.all(np.abs(got - ref) <= bound)


@pytest.mark.parametrize("d", [65, 100, 784])
@pytest.mark.parametrize("nrhs", [1, 10, 40])
def test_matvec_wide_symmetric_and_ragged(gpu_lib, d, nrhs):
    # K(X, X) W with 700 points: 6 row blocks, ragged panels, two passes of
    # right-hand sides at nrhs = 40, and the image-like data at d = 784
    if d == 784:
        X = sd.c3_image_like(n=700, m=1).X
        h = 4.0
    else:
        X = sd.points(700, d, seed=d, scale=0.3)
        h = 0.3 * np.sqrt(d)
    W = sd.vectors(700, nrhs, seed=nrhs)
    got = gpu_lib.kernel_matvec(_t(X), _t(X), h, _t(W), prec="f32").cpu().numpy()
    ref = cmath.kmv(X, X, W, h)
    assert np.all(np.abs(got - ref) <= fp32_wide_product_bound(X, X, W, h))


def test_matvec_fp32_wide_batched_and_ragged(gpu_lib):
    # FP32 entries of wide points through the per-problem row-block tables:
    # three problems of ragged sizes against row blocks and panels of
    # 128 points, per-problem widths, 40 right-hand sides (passes of 32 and 8)
    sizes, d = [300, 7, 530], 100
    rng = np.random.default_rng(6)
    Xs = [(0.3 * rng.standard_normal((k, d))).astype(np.float32) for k in sizes]
    hs = [2.0, 3.0, 2.5]
    X = np.concatenate(Xs)
    off = np.concatenate([[0], np.cumsum(sizes)])
    W = sd.vectors(X.shape[0], 40, seed=7)
    got = gpu_lib.kernel_matvec_batched(_t(X), off, hs, _t(W), prec="f32").cpu().numpy()
    for k in range(3):
        a, b = off[k], off[k + 1]
        ref = cmath.kmv(Xs[k], Xs[k], W[a:b], hs[k])
        bound = fp32_wide_product_bound(Xs[k], Xs[k], W[a:b], hs[k], anchor=X.astype(np.float64).mean(axis=0))
        assert np.all(np.abs(got[a:b] - ref) <= bound), k


def test_matvec_beta_and_empty(gpu_lib):
    X = sd.points(70, 3, seed=7, dtype=np.float64)
    W = sd.vectors(70, 2, seed=8)
    out0 = sd.vectors(70, 2, seed=9)
    out = _t(out0)
    gpu_lib.kernel_matvec(_t(X), _t(X), 0.7, _t(W), beta=-2.0, out=out, prec="f64")
    ref = cmath.kmv(X, X, W, 0.7) - 2.0 * out0
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=1e-12, atol=1e-12)
    empty = gpu_lib.kernel_matvec(_t(X[:0]), _t(X), 0.7, _t(W), prec="f64")
    assert empty.shape == (0, 2)


def test_matvec_large_sampled_rows(gpu_lib):
    # the refinement product at the 16-Gaussian workload size, checked on sampled rows
    p = sd.c2_sixteen_gaussians(n=1 << 18, m=1)
    W = sd.vectors(p.n, 1, seed=10)
    got = gpu_lib.kernel_matvec(_t(p.X), _t(p.X), p.h, _t(W), prec="f32").cpu().numpy()
    rows = np.random.default_rng(0).choice(p.n, 64, replace=False)
    ref = cmath.kmv(p.X, p.X, W, p.h, rows=rows)
    bound = fp32_product_bound(p.X[rows], p.X, W, p.h)
    assert np.all(np.abs(got[rows] - ref) <= bound)


def _tree_ranges(X, leaf, seed=1):
    t = oc.cluster2mn(X, leaf, seed)
    Xp = np.ascontiguousarray(X[t.perm])
    lb, le = leaf_ranges(t.nodes, X.shape[0])
    return Xp, lb, le


@pytest.mark.parametrize("n,d,r", [(200, 8, 32), (777, 18, 64), (1500, 8, 256)])
def test_sample_fp64(gpu_lib, n, d, r):
    X = sd.c1_two_gaussians(n=n, m=1, d=d).X
    Xp, lb, le = _tree_ranges(X, 48)
    R = sd.random_block(n, r, seed=3)
    S = gpu_lib.kernel_sample(_t(Xp), 1.0, _t(R), _t(lb), _t(le), prec="f64").cpu().numpy()
    ref = cmath.sample_masked(Xp, R, 1.0, lb, le, np.arange(n))
    scale = cmath.sample_masked(Xp, np.abs(R), 1.0, lb, le, np.arange(n))
    assert np.all(np.abs(S - ref) <= 1e-13 * scale + 1e-300)


def test_sample_unmasked_matches_matvec(gpu_lib):
    X = sd.points(300, 5, seed=11, dtype=np.float64)
    R = sd.random_block(300, 32, seed=5)
    S = gpu_lib.kernel_sample(_t(X), 0.9, _t(R), prec="f64").cpu().numpy()
    ref = cmath.kmv(X, X, R.astype(np.float64), 0.9)
    np.testing.assert_allclose(S, ref, rtol=1e-12, atol=1e-12)


def test_random_block(gpu_lib):
    R = gpu_lib.random_block(5, 1000, 64).cpu().numpy()
    assert set(np.unique(R)) == {-1.0, 1.0}
    assert abs(R.mean()) < 0.02
    R2 = gpu_lib.random_block(5, 1000, 32, c0=32).cpu().numpy()
    np.testing.assert_array_equal(R[:, 32:], R2)


def test_gather_scatter(gpu_lib):
    X = sd.points(1000, 7, seed=12)
    perm = np.random.default_rng(1).permutation(1000)
    g = gpu_lib.gather_rows(_t(X), _t(perm.astype(np.int64))).cpu().numpy()
    np.testing.assert_array_equal(g, X[perm])
    s = gpu_lib.scatter_rows(_t(g), _t(perm.astype(np.int64))).cpu().numpy()
    np.testing.assert_array_equal(s, X)


def test_predict_labels(gpu_lib):
    p = sd.c1_two_gaussians(n=500, m=300)
    a = ok.krr_fit_dense(p.X, p.y, p.h, p.lam)
    sc, lab = gpu_lib.predict(_t(p.Xt), _t(p.X), p.h, _t(a), prec="f64")
    ref = ok.scores(p.Xt, p.X, a, p.h)
    np.testing.assert_allclose(sc.cpu().numpy()[:, 0], ref, rtol=1e-11, atol=1e-12)
    np.testing.assert_array_equal(lab.cpu().numpy(), ok.labels_binary(ref).astype(np.int32))
    # one-vs-all argmax over three score columns
    A = sd.vectors(500, 3, seed=13)
    sc, lab = gpu_lib.predict(_t(p.Xt), _t(p.X), p.h, _t(A), prec="f64")
    np.testing.assert_array_equal(lab.cpu().numpy(), ok.labels_one_vs_all(ok.scores(p.Xt, p.X, A, p.h)))


@pytest.mark.parametrize("prec,tol", [("f64", 1e-11), ("f32", 2e-5)])
def test_matvec_backward(gpu_lib, prec, tol):
    X = sd.points(211, 6, seed=14, scale=0.5, dtype=np.float64)
    Y = sd.points(157, 6, seed=15, scale=0.5, dtype=np.float64)
    W = sd.vectors(157, 3, seed=16)
    G = sd.vectors(211, 3, seed=17)
    h = 0.8
    out = gpu_lib.kernel_matvec_bwd(_t(X), _t(Y), h, _t(W), _t(G), prec=prec)
    dX, dY, dW, dh = og.matvec_bwd(X, Y, W, G, h)
    for name, ref in (("dX", dX), ("dY", dY), ("dW", dW)):
        got = out[name].cpu().numpy()
        assert np.linalg.norm(got - ref) <= tol * np.linalg.norm(ref), name
    assert abs(out["dh"].item() - dh) <= tol * abs(dh)


@pytest.fixture
def sym_chunk(gpu_lib):
    """Small symmetric-product items (many chunks per row block), restored after."""
    old = gpu_lib.get_tuning("sym_chunk")
    gpu_lib.set_tuning("sym_chunk", 1024)
    yield
    gpu_lib.set_tuning("sym_chunk", old)


@pytest.fixture(params=[1, 2, 3, 4], ids=["matrix_core_f64", "vector", "matrix_core_f32", "matrix_core_bf16x3"])
def sym_form(gpu_lib, request):
    """The symmetric product's exponents: FP64 on the matrix cores (1), FP64 on
    the vector ALUs (2), FP32 on the matrix cores re-centred per row block (3),
    BF16 three-term splits of the same on the matrix cores (4)."""
    old = gpu_lib.get_tuning("symmetric")
    gpu_lib.set_tuning("symmetric", request.param)
    yield request.param
    gpu_lib.set_tuning("symmetric", old)


@pytest.mark.parametrize("d", [3, 8, 16, 18, 24, 30])
@pytest.mark.parametrize("nrhs", [1, 2])
def test_symmetric_product(gpu_lib, sym_chunk, sym_form, d, nrhs):
    # K(X, X) W with each off-diagonal entry evaluated once: 5000 points are
    # several row blocks (a ragged last one) and several column chunks per block
    # (a ragged last panel of points for the matrix-core form)
    n, h = 5000, 0.9
    X = sd.points(n, d, seed=d, scale=0.7)
    W = sd.vectors(n, nrhs, seed=nrhs)
    Xd = _t(X)
    out = gpu_lib.kernel_matvec(Xd, Xd, h, _t(W), prec="f32").cpu().numpy().reshape(n, nrhs)
    ref = cmath.kmv(X, X, W, h)
    if sym_form in (3, 4) and nrhs == 1:
        sym_bound = fp32_sym_anchored_bound(X, W, h, sym_rows_per_block(d, sym_form), form=sym_form)
    else:
        sym_bound = fp32_product_bound(X, X, W, h)
    assert np.all(np.abs(out - ref) <= sym_bound)
    # the plain product (the same points at another address) agrees to the same bound
    plain = gpu_lib.kernel_matvec(Xd, Xd.clone(), h, _t(W), prec="f32").cpu().numpy().reshape(n, nrhs)
    assert np.all(np.abs(plain - ref) <= fp32_product_bound(X, X, W, h))
    # beta accumulates into the output
    base = _t(W)
    got = gpu_lib.kernel_matvec(Xd, Xd, h, _t(W), beta=0.5, out=base.clone(), prec="f32").cpu().numpy()
    np.testing.assert_allclose(got.reshape(n, nrhs), out + 0.5 * W, rtol=0, atol=1e-12 + 1e-6 * np.abs(out).max())


def test_symmetric_product_switch(gpu_lib):
    n, d, h = 3000, 8, 1.1
    X = sd.points(n, d, seed=4)
    W = sd.vectors(n, 1, seed=5)
    Xd = _t(X)
    old = gpu_lib.get_tuning("symmetric")
    gpu_lib.set_tuning("symmetric", 0)
    try:
        a = gpu_lib.kernel_matvec(Xd, Xd, h, _t(W), prec="f32").cpu().numpy()
    finally:
        gpu_lib.set_tuning("symmetric", old)
    b = gpu_lib.kernel_matvec(Xd, Xd, h, _t(W), prec="f32").cpu().numpy()
    ref = cmath.kmv(X, X, W, h)
    bound = fp32_product_bound(X, X, W, h)
    assert np.all(np.abs(a - ref) <= bound) and np.all(np.abs(b - ref) <= bound)


@pytest.mark.parametrize("n,d", [(1, 8), (15, 8), (511, 8), (513, 3), (1023, 8), (1025, 8), (2049, 5), (3000, 20),
                                 (1500, 15)])
def test_symmetric_forms_agree_ragged(gpu_lib, sym_chunk, n, d):
    # sizes around the row blocks (BF16 form: 512 rows at d <= 9, 256 up to
    # d = 20; FP32 form: 1024 rows at d <= 8, 512 above) and the
    # 256-point panels: both symmetric forms against the oracle
    X = sd.points(n, d, seed=n, scale=0.6)
    W = sd.vectors(n, 1, seed=3)
    Xd = _t(X)
    ref = cmath.kmv(X, X, W, 0.8)
    bound = fp32_product_bound(X, X, W, 0.8)
    old = gpu_lib.get_tuning("symmetric")
    try:
        for form in (1, 2, 3, 4):
            gpu_lib.set_tuning("symmetric", form)
            got = gpu_lib.kernel_matvec(Xd, Xd, 0.8, _t(W), prec="f32").cpu().numpy()
            if form >= 3:
                bound = fp32_sym_anchored_bound(X, W, 0.8, sym_rows_per_block(d, form), form=form)
            assert np.all(np.abs(got - ref) <= bound), form
        # the BF16 form recording its negligible-tile map, then skipping
        # those tiles (every item's map words, ragged panels and row blocks)
        gpu_lib.set_tuning("symmetric", 4)
        gpu_lib.set_tuning("sym_skip", 2)
        got = gpu_lib.kernel_matvec(Xd, Xd, 0.8, _t(W), prec="f32").cpu().numpy()
        bound = fp32_sym_anchored_bound(X, W, 0.8, sym_rows_per_block(d, 4), form=4)
        assert np.all(np.abs(got - ref) <= bound + negligible_mass(X, W, 0.8))
    finally:
        gpu_lib.set_tuning("symmetric", old)
        gpu_lib.set_tuning("sym_skip", 1)


def _line_clusters(n, seed):
    """Eight tight clusters (sigma 0.02) on a line, 6.87 apart, in cluster
    order, and positive weights near 1e9 on every other cluster."""
    rng = np.random.default_rng(seed)
    lab = np.sort(rng.integers(0, 8, n))
    X = (0.02 * rng.standard_normal((n, 8))).astype(np.float32)
    X[:, 0] += (6.87 * lab).astype(np.float32)
    W = (1.0 + 0.5 * rng.random((n, 1))) * np.where(lab % 2 == 1, 1e9, 1.0)[:, None]
    return X, W


def test_tile_map_entry_point(gpu_lib, sym_chunk):
    # kernel_matvec_mapped: the first call records (every entry evaluated:
    # the plain bound), the next ones with the same points and width leave
    # out the negligible tiles (bound widened by the mass below 2^-31.5); a
    # new width or another address of the points records again
    n, h = 6037, 1.0
    X, W = _line_clusters(n, 11)
    Xh = X.astype(np.float64)
    W2 = W[::-1].copy()
    Xd = _t(X)
    tm = gpu_lib.TileMap()
    assert tm.counts() == (0, 0, 0)
    rows = sym_rows_per_block(8, 4)
    b1 = fp32_sym_anchored_bound(Xh, W, h, rows, form=4)
    first = tm.matvec(Xd, h, _t(W)).cpu().numpy()
    assert np.all(np.abs(first - cmath.kmv(Xh, Xh, W, h)) <= b1)
    kept, tiles, per_tile = tm.counts()
    assert per_tile == rows // 8 * 16 and 0 < kept < tiles
    # the map covers every wave tile (8 waves x 16 tiles of a 256-point
    # panel) of each item: a row block against a 1024-column chunk right of
    # its diagonal block
    want = 0
    for i0 in range(0, n, rows):
        off = min(n, i0 + rows)
        for c in range(off // 1024, (n - 1) // 1024 + 1) if off < n else ():
            j0, j1 = max(off, c * 1024), min(n, (c + 1) * 1024)
            want += -(-(j1 - j0) // 256) * 8 * 16
    assert tiles == want
    ref2 = cmath.kmv(Xh, Xh, W2, h)
    b2 = fp32_sym_anchored_bound(Xh, W2, h, rows, form=4)
    second = tm.matvec(Xd, h, _t(W2)).cpu().numpy()
    assert np.all(np.abs(second - ref2) <= b2 + negligible_mass(Xh, W2, h))
    assert np.any(np.abs(second - ref2) > b2)
    assert tm.counts() == (kept, tiles, per_tile)
    # beta accumulates as in kernel_matvec (the same tiles again)
    got = tm.matvec(Xd, h, _t(W2), beta=0.5, out=_t(W2)).cpu().numpy()
    np.testing.assert_allclose(got, second + 0.5 * W2, rtol=1e-15, atol=0)
    # a wider kernel: recorded again, every entry evaluated
    h3 = 1.6
    third = tm.matvec(Xd, h3, _t(W)).cpu().numpy()
    assert np.all(np.abs(third - cmath.kmv(Xh, Xh, W, h3)) <= fp32_sym_anchored_bound(Xh, W, h3, rows, form=4))
    assert tm.counts()[0] > kept
    # the points at another address: recorded again
    Xc = Xd.clone()
    fourth = tm.matvec(Xc, h, _t(W2)).cpu().numpy()
    assert np.all(np.abs(fourth - ref2) <= b2)


def test_batched_symmetric_product_tile_map(gpu_lib, sym_chunk):
    # a batch of three line-cluster problems (per-problem widths) through the
    # batched symmetric product, recording its map and then skipping: each
    # item's map words are found by its index among every problem's items
    parts = [_line_clusters(n, 20 + n) for n in (1500, 2300, 777)]
    hs = [1.0, 1.05, 0.95]
    X = np.concatenate([x for x, _ in parts]).astype(np.float32)
    W = np.concatenate([w for _, w in parts])
    off = np.cumsum([0] + [x.shape[0] for x, _ in parts])
    old = gpu_lib.get_tuning("symmetric")
    try:
        gpu_lib.set_tuning("symmetric", 4)
        gpu_lib.set_tuning("sym_skip", 2)
        out = gpu_lib.kernel_matvec_batched(_t(X), off, hs, _t(W), prec="f32").cpu().numpy()
    finally:
        gpu_lib.set_tuning("symmetric", old)
        gpu_lib.set_tuning("sym_skip", 1)
    dropped = False
    for k, h in enumerate(hs):
        a, b = off[k], off[k + 1]
        Xk = X[a:b].astype(np.float64)
        ref = cmath.kmv(Xk, Xk, W[a:b], h)
        bound = fp32_sym_anchored_bound(Xk, W[a:b], h, sym_rows_per_block(8, 4), form=4)
        assert np.all(np.abs(out[a:b] - ref) <= bound + negligible_mass(Xk, W[a:b], h)), k
        dropped = dropped or bool(np.any(np.abs(out[a:b] - ref) > bound))
    assert dropped


def test_symmetric_product_tile_map(gpu_lib, sym_chunk):
    # Eight tight clusters on a line, 6.87 h apart: entries between neighbours
    # are about 2^-34 and the rest underflow, so most wave tiles are
    # negligible.  Positive weights near 1e9 on every other cluster make the
    # skipped entries' share visible (about 40 on the other clusters' rows).  With the map (record, then skip) the product is within
    # the FP32 bound widened by the mass of the entries below 2^-31.5; it does
    # leave that mass out (beyond the bound on some rows), and without the
    # map every entry is evaluated (the plain bound).
    n, d, h = 6037, 8, 1.0
    X, W = _line_clusters(n, 11)
    Xd = _t(X)
    Xh = X.astype(np.float64)
    ref = cmath.kmv(Xh, Xh, W, h)
    bound = fp32_sym_anchored_bound(Xh, W, h, sym_rows_per_block(d, 4), form=4)
    bmap = fp32_sym_anchored_bound(Xh, W, h, sym_rows_per_block(d, 4), form=4)
    old = gpu_lib.get_tuning("symmetric")
    try:
        gpu_lib.set_tuning("symmetric", 4)
        gpu_lib.set_tuning("sym_skip", 0)
        full = gpu_lib.kernel_matvec(Xd, Xd, h, _t(W), prec="f32").cpu().numpy()
        gpu_lib.set_tuning("sym_skip", 2)
        skip = gpu_lib.kernel_matvec(Xd, Xd, h, _t(W), prec="f32").cpu().numpy()
    finally:
        gpu_lib.set_tuning("symmetric", old)
        gpu_lib.set_tuning("sym_skip", 1)
    assert np.all(np.abs(full - ref) <= bound)
    assert np.all(np.abs(skip - ref) <= bmap + negligible_mass(Xh, W, h))
    assert np.any(np.abs(skip - ref) > bmap)
