"""The image-like workload (d = 784, ten one-vs-all right-hand sides) at a
size the dense oracle solves: the wide-point kernels (coordinates streamed,
no register tiles), the fit of all ten right-hand sides, and one-vs-all
prediction against dense FP64 KRR."""
import numpy as np
import pytest
import torch

import synthdata as sd
from oracle import kernel as ok

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_image_like_fit_matches_dense(gpu_lib, prec):
    p = sd.c3_image_like(n=3000, m=500)
    X = torch.from_numpy(p.X).cuda()
    Y = torch.from_numpy(np.ascontiguousarray(p.y)).cuda()
    opts = gpu_lib.HssOptions(rtol=1e-6, r0=256, dr=256, r_max=2048, prec=prec, cap_policy=1)
    res = gpu_lib.fit(X, Y, p.h, p.lam, leaf=p.leaf, opts=opts, tol=1e-10, max_iter=1000, mv_prec="f64")
    assert res.info["refine"]["converged"]
    a = res.alpha.cpu().numpy()
    Xd = p.X.astype(np.float64)
    K = ok.kernel_dense(Xd, Xd, p.h)
    ref = ok.krr_solve_dense(K, p.y, p.lam)
    cond = np.linalg.cond(K + p.lam * np.eye(K.shape[0]))
    assert np.linalg.norm(a - ref) <= 10 * cond * 1e-10 * np.linalg.norm(ref)
    # one-vs-all: argmax of the signed class scores
    Xt = torch.from_numpy(p.Xt).cuda()
    scores, labels = gpu_lib.predict(Xt, res.Xp, p.h, res.alpha_perm, prec="f64")
    s_ref = ok.scores(p.Xt.astype(np.float64), Xd, ref, p.h)
    np.testing.assert_allclose(scores.cpu().numpy(), s_ref, rtol=0, atol=1e-6 * np.abs(s_ref).max())
    lab_ref = ok.labels_one_vs_all(s_ref)
    srt = np.sort(s_ref, axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 1e-6 * np.abs(s_ref).max()
    assert np.all(labels.cpu().numpy()[clear] == lab_ref[clear])
    assert abs(ok.accuracy(labels.cpu().numpy(), p.yt) - ok.accuracy(lab_ref, p.yt)) <= 1.0 / 500


def test_image_like_mixed_precision_refinement(gpu_lib):
    # FP32-entry products inside the iteration, FP64 residuals outside: the
    # iteration restarts from the FP64 residual until it meets a tolerance
    # the FP32 products alone cannot certify
    p = sd.c3_image_like(n=3000, m=1)
    X = torch.from_numpy(p.X).cuda()
    Y = torch.from_numpy(np.ascontiguousarray(p.y[:, :2])).cuda()
    opts = gpu_lib.HssOptions(rtol=1e-2, r0=256, dr=256, r_max=512, prec="f16", cap_policy=1)
    res = gpu_lib.fit(X, Y, p.h, p.lam, leaf=p.leaf, opts=opts, tol=1e-10, max_iter=1000, mv_prec="f32",
                      res_prec="f64")
    assert res.info["refine"]["converged"]
    Xd = p.X.astype(np.float64)
    K = ok.kernel_dense(Xd, Xd, p.h)
    a = res.alpha.cpu().numpy()
    r = p.y[:, :2] - K @ a - p.lam * a
    assert np.all(np.linalg.norm(r, axis=0) <= 1e-10 * np.linalg.norm(p.y[:, :2], axis=0) * 1.01)
