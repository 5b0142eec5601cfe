"""Differentiation on the GPU: the fused kernel-product backward through
torch.autograd against the oracle's dense FP64 gradients, and the validation
loss gradient in (log h, log lambda) (adjoint through the ULV-preconditioned
refinement) against the oracle's analytic gradient and against central
finite differences of the GPU objective itself."""
import math

import numpy as np
import pytest
import torch

import synthdata as sd
from oracle import grad as og

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_kernel_matvec_autograd(gpu_lib):
    from paper_1803_10274_amd.autograd import KernelMatvec
    X = sd.points(300, 18, seed=31, scale=0.4, dtype=np.float64)
    Y = sd.points(250, 18, seed=32, scale=0.4, dtype=np.float64)
    W = sd.vectors(250, 2, seed=33)
    G = sd.vectors(300, 2, seed=34)
    h = 1.3
    Xt = _t(X).requires_grad_(True)
    Yt = _t(Y).requires_grad_(True)
    Wt = _t(W).requires_grad_(True)
    ht = torch.tensor(h, dtype=torch.float64, device="cuda", requires_grad=True)
    out = KernelMatvec.apply(Xt, Yt, Wt, ht, "f64")
    (out * _t(G)).sum().backward()
    dX, dY, dW, dh = og.matvec_bwd(X, Y, W, G, h)
    for got, ref in ((Xt.grad, dX), (Yt.grad, dY), (Wt.grad, dW)):
        assert np.linalg.norm(got.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)
    assert abs(ht.grad.item() - dh) <= 1e-10 * abs(dh)


@pytest.mark.parametrize("m,n,d,same", [(3001, 2500, 18, False), (1000, 1000, 8, True), (3000, 3000, 18, True),
                                         (777, 4099, 40, False)])
def test_fused_backward_dh_fp32(gpu_lib, m, n, d, same):
    # dh alone with FP32 entries runs as the product with the entry exp2(t) t.
    # d <= 31: BF16 three-term exponents on the matrix cores, for X = Y in the
    # symmetric form (each off-diagonal entry once; 2 and 12 row blocks here),
    # otherwise in the rectangular form (6 row blocks x column chunks); d = 40:
    # the split-K kernel with FP64 exponents rounded to FP32.  FP32 tile sums,
    # FP64 across tiles: within 1e-5 of sum_ab |P_ab| q_ab / h^3
    Y = sd.points(n, d, seed=41 + d, scale=0.4)
    X = Y if same else sd.points(m, d, seed=42 + d, scale=0.4)
    W = sd.vectors(n, 1, seed=43)
    G = sd.vectors(X.shape[0], 1, seed=44)
    h = 0.3 * np.sqrt(d)
    Xt = _t(X)
    Yt = Xt if same else _t(Y)
    got = gpu_lib.kernel_matvec_bwd(Xt, Yt, h, _t(W), _t(G), prec="f32", want=("dh",))["dh"].item()
    _, _, _, dh = og.matvec_bwd(X.astype(np.float64), Y.astype(np.float64), W, G, h)
    Xd, Yd = X.astype(np.float64), Y.astype(np.float64)
    Q = np.maximum((Xd * Xd).sum(1)[:, None] + (Yd * Yd).sum(1)[None, :] - 2.0 * Xd @ Yd.T, 0.0)
    mag = float((np.abs(G) * (np.exp(-Q / (2 * h * h)) * Q) @ np.abs(W)).sum() / h**3)
    assert abs(got - dh) <= 1e-5 * mag, (got, dh, mag)


@pytest.mark.parametrize("n,mv", [(2048, 512), (8192, 1024)])
def test_validation_gradient_against_oracle(gpu_lib, n, mv):
    from paper_1803_10274_amd.autograd import validation_loss
    p = sd.c5_eight_gaussians(n=n, m=mv)
    lh = torch.tensor(math.log(p.h), dtype=torch.float64, device="cuda", requires_grad=True)
    ll = torch.tensor(math.log(p.lam), dtype=torch.float64, device="cuda", requires_grad=True)
    L, st = validation_loss(lh, ll, _t(p.X), _t(p.y), _t(p.Xt), _t(p.yt), tol=1e-7)
    L.backward()
    L_ref, gh_ref, gl_ref = og.val_loss_grad(p.X.astype(np.float64), p.y, p.Xt.astype(np.float64), p.yt,
                                             p.h, p.lam)
    assert abs(L.item() - L_ref) <= 1e-6 * abs(L_ref)
    assert abs(lh.grad.item() - gh_ref) <= 1e-3 * abs(gh_ref)
    assert abs(ll.grad.item() - gl_ref) <= 1e-3 * abs(gl_ref)


def test_validation_gradient_against_stored_oracle_32k(gpu_lib):
    # n = 32,768, m_v = 4,096 (the gradient workload at a quarter of its size):
    # the dense FP64 oracle's value was written by tests/golden/make_c5_gradient.py
    import json
    import os
    from paper_1803_10274_amd.autograd import validation_loss
    with open(os.path.join(os.path.dirname(__file__), "golden", "c5_gradient_n32768.json")) as f:
        ref = json.load(f)
    p = sd.c5_eight_gaussians(n=ref["n"], m=ref["m_v"])
    assert (p.h, p.lam) == (ref["h"], ref["lam"])
    lh = torch.tensor(math.log(p.h), dtype=torch.float64, device="cuda", requires_grad=True)
    ll = torch.tensor(math.log(p.lam), dtype=torch.float64, device="cuda", requires_grad=True)
    L, st = validation_loss(lh, ll, _t(p.X), _t(p.y), _t(p.Xt), _t(p.yt), tol=1e-7)
    L.backward()
    assert abs(L.item() - ref["loss"]) <= 1e-6 * abs(ref["loss"])
    assert abs(lh.grad.item() - ref["dL_dlogh"]) <= 1e-3 * abs(ref["dL_dlogh"])
    assert abs(ll.grad.item() - ref["dL_dloglam"]) <= 1e-3 * abs(ref["dL_dloglam"])


def test_validation_gradient_finite_differences(gpu_lib):
    # central differences of the GPU objective (tightly refined, so smooth in h)
    from paper_1803_10274_amd.autograd import validation_loss
    p = sd.c5_eight_gaussians(n=16384, m=2048)
    X, y, Xv, yv = _t(p.X), _t(p.y), _t(p.Xt), _t(p.yt)
    lh = torch.tensor(math.log(p.h), dtype=torch.float64, device="cuda", requires_grad=True)
    ll = torch.tensor(math.log(p.lam), dtype=torch.float64, device="cuda", requires_grad=True)
    L, st = validation_loss(lh, ll, X, y, Xv, yv, tol=1e-10, prec="f64")
    L.backward()
    s = 1e-3

    def f(a, b):
        v, _ = validation_loss(torch.tensor(a, dtype=torch.float64, device="cuda"),
                               torch.tensor(b, dtype=torch.float64, device="cuda"), X, y, Xv, yv, state=st)
        return v.item()

    fh = (f(math.log(p.h) + s, math.log(p.lam)) - f(math.log(p.h) - s, math.log(p.lam))) / (2 * s)
    fl = (f(math.log(p.h), math.log(p.lam) + s) - f(math.log(p.h), math.log(p.lam) - s)) / (2 * s)
    assert abs(lh.grad.item() - fh) <= 2e-3 * abs(fh) + 1e-7
    assert abs(ll.grad.item() - fl) <= 2e-3 * abs(fl) + 1e-7


def test_hyperparameter_descent(gpu_lib):
    # gradient steps on (log h, log lambda) from a poor start: accepted losses
    # fall, lambda trials refactor without recompressing, a compression is
    # built only for a new h (an h still cached is reused), and the loss
    # reported at the end is the oracle's at the final parameters
    from paper_1803_10274_amd.autograd import tune_hyperparameters
    p = sd.c5_eight_gaussians(n=2048, m=512)
    res = tune_hyperparameters(_t(p.X), _t(p.y), _t(p.Xt), _t(p.yt), p.h / 4, p.lam * 8, steps=4, tol=1e-7)
    hist = res["history"]
    print("hyperparameter descent:", [(k, round(h, 4), round(l, 4), round(L, 6), ok, c)
                                      for k, h, l, L, ok, c in hist], flush=True)
    acc = [e[3] for e in hist if e[4]]
    assert len(acc) >= 2
    assert all(b < a for a, b in zip(acc, acc[1:]))
    assert hist[0][5] and all(not e[5] for e in hist if e[0] == "lambda")
    assert all(e[1] != prev[1] for prev, e in zip(hist, hist[1:]) if e[5])  # compress only for a new h
    assert res["n_fits"] == len(hist)
    assert res["n_compress"] == sum(1 for e in hist if e[5])
    L_ref = og.val_loss(p.X.astype(np.float64), p.y, p.Xt.astype(np.float64), p.yt, res["h"], res["lam"])
    assert abs(res["loss"] - L_ref) <= 1e-6 * abs(L_ref)
