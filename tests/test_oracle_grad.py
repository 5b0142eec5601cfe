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


def test_val_loss_closed_forms():
    # training points 100 apart at h = 1: K = I exactly (off-diagonal entries
    # underflow to 0), so alpha = y / (1 + lambda).  Validating on the training
    # points gives f = alpha, L = |y / (1 + lambda) - y_v|^2 / m and
    #   dL/dlog lambda = lambda * sum 2 (f - y_v) (-y / (1 + lambda)^2) / m;
    # every entry of K and K_v is 0 or 1 (q = 0 or huge), so dK/dh = 0 and
    # dL/dlog h = 0.  Validation points far from all training points give
    # K_v = 0, f = 0 and L = |y_v|^2 / m.
    m, lam = 12, 0.7
    X = np.arange(m, dtype=np.float64)[:, None] * np.array([[100.0, 0.0, 50.0]])
    rng = np.random.default_rng(9)
    y, yv = rng.standard_normal(m), rng.standard_normal(m)
    f = y / (1 + lam)
    L_ref = float(np.sum((f - yv) ** 2) / m)
    gl_ref = lam * float(np.sum(2 * (f - yv) * (-y / (1 + lam) ** 2)) / m)
    assert abs(og.val_loss(X, y, X, yv, 1.0, lam) - L_ref) <= 1e-15 * max(1.0, L_ref)
    L, gh, gl = og.val_loss_grad(X, y, X, yv, 1.0, lam)
    assert abs(L - L_ref) <= 1e-15 * max(1.0, L_ref)
    assert abs(gl - gl_ref) <= 1e-14 * max(1.0, abs(gl_ref))
    assert gh == 0.0
    Xv = X + np.array([[0.0, 1e4, 0.0]])
    assert abs(og.val_loss(X, y, Xv, yv, 1.0, lam) - float(yv @ yv / m)) <= 1e-15 * float(yv @ yv)


def test_blocked_gradient_matches_central_differences():
    # the blocked form (rows in blocks smaller than n, a ragged last block)
    # against central differences of the dense objective, and against the
    # unblocked form
    p = sd.c5_eight_gaussians(n=700, m=150, d=5)
    X, y, Xv, yv = p.X.astype(np.float64), p.y, p.Xt.astype(np.float64), p.yt
    h, lam = 1.7, 0.6
    L, gh, gl = og.val_loss_grad_blocked(X, y, Xv, yv, h, lam, block=128)
    s = 1e-4
    fh = (og.val_loss(X, y, Xv, yv, h * np.exp(s), lam)
          - og.val_loss(X, y, Xv, yv, h * np.exp(-s), lam)) / (2 * s)
    fl = (og.val_loss(X, y, Xv, yv, h, lam * np.exp(s))
          - og.val_loss(X, y, Xv, yv, h, lam * np.exp(-s))) / (2 * s)
    assert abs(L - og.val_loss(X, y, Xv, yv, h, lam)) <= 1e-12 * L
    assert abs(gh - fh) <= 1e-6 * max(abs(fh), 1e-3)
    assert abs(gl - fl) <= 1e-6 * max(abs(fl), 1e-3)
    L2, gh2, gl2 = og.val_loss_grad(X, y, Xv, yv, h, lam)
    assert abs(gh - gh2) <= 1e-10 * abs(gh2) and abs(gl - gl2) <= 1e-10 * abs(gl2)
