"""Gradients for tuning (h, lambda) by the validation loss, dense FP64.

The paper picks (h, lambda) by grid search or black-box tuning (Section 5.3)
and notes that a change of lambda touches only the diagonal while a change of
h needs a new compression.  The GPU path replaces the search by gradients of
the validation mean squared error; these are the plain dense definitions the
GPU gradients are checked against.  Derivation (alpha = (K + lambda I)^{-1} y,
f = K_v alpha, e = f - y_v, L = |e|^2 / m_v, g = (2 / m_v) K_v^T e,
beta = (K + lambda I)^{-1} g, dK_ij/dh = K_ij ||x_i - x_j||^2 / h^3):
  dL/dlambda = -beta^T alpha
  dL/dh      = (2 / m_v) e^T (dK_v/dh) alpha - beta^T (dK/dh) alpha
Fused kernel product Out = K(X, Y; h) W with upstream gradient G:
  dW = K(X, Y)^T G,   P = K o (G W^T),
  dX_i = -(1/h^2) [ (sum_j P_ij) x_i - (P Y)_i ],
  dY_j =  (1/h^2) [ (P^T X)_j - (sum_i P_ij) y_j ],
  dh   = sum_ij P_ij ||x_i - y_j||^2 / h^3.

Test infrastructure only (see the package docstring)."""
import numpy as np
import scipy.linalg as sla

from .kernel import kernel_dense


def _sqdist(X, Y):
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    q = np.zeros((X.shape[0], Y.shape[0]))
    for k in range(X.shape[1]):
        diff = X[:, k][:, None] - Y[:, k][None, :]
        q += diff * diff
    return q


def val_loss(X, y, Xv, yv, h, lam):
    """Validation MSE of the KRR fit at (h, lambda)."""
    K = kernel_dense(X, X, h)
    K[np.diag_indices_from(K)] += lam
    alpha = sla.cho_solve(sla.cho_factor(K, lower=True), np.asarray(y, dtype=np.float64))
    e = kernel_dense(Xv, X, h) @ alpha - yv
    return float(np.sum(e * e) / e.shape[0])


def val_loss_grad(X, y, Xv, yv, h, lam):
    """(L, dL/dlog h, dL/dlog lambda), analytic, dense FP64."""
    y = np.asarray(y, dtype=np.float64)
    yv = np.asarray(yv, dtype=np.float64)
    Q = _sqdist(X, X)
    K = np.exp(-Q / (2 * h * h))
    Qv = _sqdist(Xv, X)
    Kv = np.exp(-Qv / (2 * h * h))
    A = K.copy()
    A[np.diag_indices_from(A)] += lam
    c = sla.cho_factor(A, lower=True)
    alpha = sla.cho_solve(c, y)
    e = Kv @ alpha - yv
    mv = e.shape[0]
    L = float(e @ e / mv)
    g = (2.0 / mv) * (Kv.T @ e)
    beta = sla.cho_solve(c, g)
    dL_dlam = -float(beta @ alpha)
    dKv = Kv * Qv / h**3
    dK = K * Q / h**3
    dL_dh = float((2.0 / mv) * e @ (dKv @ alpha) - beta @ (dK @ alpha))
    return L, h * dL_dh, lam * dL_dlam


def matvec_bwd(X, Y, W, G, h):
    """Backward of Out = K(X, Y; h) W for upstream G: (dX, dY, dW, dh)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64).reshape(Y.shape[0], -1)
    G = np.asarray(G, dtype=np.float64).reshape(X.shape[0], -1)
    Q = _sqdist(X, Y)
    K = np.exp(-Q / (2 * h * h))
    dW = K.T @ G
    P = K * (G @ W.T)
    dX = -(P.sum(axis=1)[:, None] * X - P @ Y) / h**2
    dY = (P.T @ X - P.sum(axis=0)[:, None] * Y) / h**2
    dh = float(np.sum(P * Q) / h**3)
    return dX, dY, dW, dh


def val_loss_grad_blocked(X, y, Xv, yv, h, lam, block=4096):
    """(L, dL/dlog h, dL/dlog lambda) by the same formulas as val_loss_grad,
    dense FP64 with one n x n array (K + lambda I) and its Cholesky factor
    (torch's CPU Cholesky: SciPy's LAPACK build fails at n = 32,768 here): the
    products with K_v, dK_v/dh and dK/dh are formed block of rows by block of
    rows from the differences, so n = 32,768 fits in ~20 GB."""
    import torch
    X = np.asarray(X, dtype=np.float64)
    Xv = np.asarray(Xv, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    yv = np.asarray(yv, dtype=np.float64)
    n = X.shape[0]
    A = np.empty((n, n))
    for b in range(0, n, block):
        e = min(b + block, n)
        A[b:e] = np.exp(-_sqdist(X[b:e], X) / (2 * h * h))
    A[np.diag_indices_from(A)] += lam
    Lc = torch.linalg.cholesky(torch.from_numpy(A))
    del A

    def solve(rhs):
        return torch.cholesky_solve(torch.from_numpy(rhs.reshape(-1, 1).copy()), Lc).numpy().ravel()

    alpha = solve(y)
    mv = Xv.shape[0]
    f = np.empty(mv)
    dKva = np.empty(mv)
    g = np.zeros(n)
    for b in range(0, mv, block):
        e = min(b + block, mv)
        Qv = _sqdist(Xv[b:e], X)
        Kv = np.exp(-Qv / (2 * h * h))
        f[b:e] = Kv @ alpha
        dKva[b:e] = (Kv * Qv / h**3) @ alpha
    err = f - yv
    L = float(err @ err / mv)
    for b in range(0, mv, block):
        e = min(b + block, mv)
        Kv = np.exp(-_sqdist(Xv[b:e], X) / (2 * h * h))
        g += Kv.T @ err[b:e]
    g *= 2.0 / mv
    beta = solve(g)
    del Lc
    dKa = np.empty(n)
    for b in range(0, n, block):
        e = min(b + block, n)
        Q = _sqdist(X[b:e], X)
        dKa[b:e] = (np.exp(-Q / (2 * h * h)) * Q / h**3) @ alpha
    dL_dlam = -float(beta @ alpha)
    dL_dh = float((2.0 / mv) * err @ dKva - beta @ dKa)
    return L, h * dL_dh, lam * dL_dlam
