"""Pins for the gradient oracle: central finite differences of the dense FP64
objective (step 1e-4 in log h and log lambda), linearity in W, and the
adjoint identity of the kernel product."""
import numpy as np

import synthdata as sd
from oracle import grad as og
from oracle import kernel as ok


def test_val_loss_gradient_matches_central_differences():
    p = sd.c5_eight_gaussians(n=400, m=120, d=6)
    X, y, Xv, yv = p.X.astype(np.float64), p.y, p.Xt.astype(np.float64), p.yt
    h, lam = 2.0, 1.0
    L, gh, gl = og.val_loss_grad(X, y, Xv, yv, h, lam)
    assert L == og.val_loss(X, y, Xv, yv, h, lam) or abs(L - og.val_loss(X, y, Xv, yv, h, lam)) < 1e-12
    s = 1e-4
    fh = (og.val_loss(X, y, Xv, yv, h * np.exp(s), lam)
          - og.val_loss(X, y, Xv, yv, h * np.exp(-s), lam)) / (2 * s)
    fl = (og.val_loss(X, y, Xv, yv, h, lam * np.exp(s))
          - og.val_loss(X, y, Xv, yv, h, lam * np.exp(-s))) / (2 * s)
    assert abs(gh - fh) <= 1e-6 * max(abs(fh), 1e-3)
    assert abs(gl - fl) <= 1e-6 * max(abs(fl), 1e-3)


def test_matvec_backward_finite_differences():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((9, 3))
    Y = rng.standard_normal((11, 3))
    W = rng.standard_normal((11, 2))
    G = rng.standard_normal((9, 2))
    h = 0.9

    def f(X, Y, W, h):
        return float(np.sum(G * (ok.kernel_dense(X, Y, h) @ W)))

    dX, dY, dW, dh = og.matvec_bwd(X, Y, W, G, h)
    s = 1e-6
    for (i, k) in [(0, 0), (4, 2), (8, 1)]:
        E = np.zeros_like(X)
        E[i, k] = s
        fd = (f(X + E, Y, W, h) - f(X - E, Y, W, h)) / (2 * s)
        assert abs(dX[i, k] - fd) < 1e-7 * max(1, abs(fd))
    for (j, k) in [(0, 1), (10, 2), (5, 0)]:
        E = np.zeros_like(Y)
        E[j, k] = s
        fd = (f(X, Y + E, W, h) - f(X, Y - E, W, h)) / (2 * s)
        assert abs(dY[j, k] - fd) < 1e-7 * max(1, abs(fd))
    fd = (f(X, Y, W, h + s) - f(X, Y, W, h - s)) / (2 * s)
    assert abs(dh - fd) < 1e-7 * max(1, abs(fd))
    # f is linear in W: a finite difference is exact up to rounding
    E = np.zeros_like(W)
    E[3, 1] = 1.0
    assert abs(dW[3, 1] - (f(X, Y, W + E, h) - f(X, Y, W, h))) < 1e-12
    # translation invariance of the kernel: sum of dX and dY is zero
    np.testing.assert_allclose(dX.sum(axis=0) + dY.sum(axis=0), 0, atol=1e-12)


def test_adjoint_identity():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((7, 2))
    Y = rng.standard_normal((5, 2))
    u = rng.standard_normal(7)
    v = rng.standard_normal(5)
    lhs = u @ (ok.kernel_dense(X, Y, 1.2) @ v)
    rhs = (ok.kernel_dense(Y, X, 1.2) @ u) @ v
    assert abs(lhs - rhs) < 1e-13
