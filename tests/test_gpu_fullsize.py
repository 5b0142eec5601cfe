"""The benchmark configuration at full size (16-Gaussian workload, n = 2^20,
d = 8, FP16 2-term sampling, r0 = 256 grown adaptively, refinement on the FP32-entry product to
1e-6), certified in FP64: the residual of the fitted coefficients is
recomputed with the FP64 kernel product over all n^2 entries, its rows are
checked one by one against the oracle's matrix-free FP64 residual on sampled
rows, and the predicted labels of test points against the oracle's scores of
the same coefficients."""
import numpy as np
import pytest
import torch

import synthdata as sd
from oracle import cmath, kernel as ok

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fitted(gpu_lib):
    p = sd.c2_sixteen_gaussians(m=2000)
    X = torch.from_numpy(p.X).cuda()
    y = torch.from_numpy(p.y).cuda()
    # the benchmark's options: C2's rtol 1e-2 and r0 = 256 grown adaptively,
    # with the absolute tolerance the benchmark uses
    opts = gpu_lib.HssOptions(rtol=1e-2, atol=6.0, r0=256, dr=256, r_max=4096, prec="f16", split_terms=2,
                              cap_policy=0)
    res = gpu_lib.fit(X, y, p.h, p.lam, leaf=p.leaf, opts=opts, tol=1e-6, max_iter=300)
    return p, res


def test_fullsize_fp64_residual(gpu_lib, fitted):
    p, res = fitted
    assert res.info["refine"]["converged"]
    Xp, a = res.Xp, res.alpha_perm.reshape(-1, 1).contiguous()
    yp = gpu_lib.gather_rows(torch.from_numpy(p.y).cuda().reshape(-1, 1).contiguous(), res.perm)
    Ka = gpu_lib.kernel_matvec(Xp, Xp, p.h, a, prec="f64")
    r = (yp - Ka - p.lam * a).cpu().numpy().ravel()
    ynorm = float(np.linalg.norm(p.y))
    # the solve stops at relres <= 1e-6 measured with FP32-entry products; the
    # target is the FP64 residual, which must be within it too
    assert np.linalg.norm(r) <= 1e-6 * ynorm
    # the FP64 product row by row against the oracle's matrix-free residual
    rows = np.concatenate([np.arange(4), np.random.default_rng(0).choice(p.n, 28, replace=False), [p.n - 1]])
    Xh = Xp.cpu().numpy()
    ah = a.cpu().numpy().ravel()
    ref = cmath.residual(Xh, ah, yp.cpu().numpy().ravel(), p.h, p.lam, rows=rows)
    scale = np.abs(ah).max() * 1e4 + 1.0  # |K| row sums are below ~1e4 here
    np.testing.assert_allclose(r[rows], ref, rtol=0, atol=1e-12 * scale)


def test_fullsize_prediction_labels(gpu_lib, fitted):
    p, res = fitted
    Xt = torch.from_numpy(p.Xt).cuda()
    scores, labels = gpu_lib.predict(Xt, res.Xp, p.h, res.alpha_perm)
    s_ref = cmath.kmv(p.Xt, res.Xp.cpu().numpy(), res.alpha_perm.cpu().numpy().ravel(), p.h)
    lab_ref = ok.labels_binary(s_ref)
    sure = np.abs(s_ref) > 1e-3 * np.abs(s_ref).max()
    assert np.all(labels.cpu().numpy()[sure] == lab_ref[sure])
    acc = ok.accuracy(labels.cpu().numpy(), p.yt)
    assert acc >= 0.99
