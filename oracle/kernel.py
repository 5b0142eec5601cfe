"""Dense FP64 Gaussian-kernel ridge regression (Algorithm 1, eq. (1.1), eq. (2.1)).

Test infrastructure only (see the package docstring)."""
import numpy as np
import scipy.linalg as sla


def kernel_dense(X, Y, h):
    """K_ij = exp(-||x_i - y_j||^2 / (2 h^2)), eq. (1.1) and Algorithm 1 step 1.

    Formed from the differences x_i - y_j (no norm expansion), in FP64."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    q = np.zeros((X.shape[0], Y.shape[0]))
    for k in range(X.shape[1]):
        diff = X[:, k][:, None] - Y[:, k][None, :]
        q += diff * diff
    return np.exp(-q / (2.0 * h * h))


def krr_solve_dense(K, y, lam):
    """w = (K + lambda I)^{-1} y by Cholesky (Algorithm 1 step 2)."""
    A = np.array(K, dtype=np.float64, copy=True)
    A[np.diag_indices_from(A)] += lam
    c = sla.cho_factor(A, lower=True)
    return sla.cho_solve(c, np.asarray(y, dtype=np.float64))


def krr_fit_dense(X, y, h, lam):
    """Algorithm 1 steps 1-2 on the given ordering."""
    return krr_solve_dense(kernel_dense(X, X, h), y, lam)


def scores(Xt, X, w, h):
    """w^T K'(i) for every test point (Algorithm 1 step 3)."""
    return kernel_dense(Xt, X, h) @ np.asarray(w, dtype=np.float64)


def labels_binary(s):
    """Algorithm 1 step 4: sign of the score; a zero score counts as +1."""
    return np.where(np.asarray(s) >= 0.0, 1.0, -1.0)


def labels_one_vs_all(S):
    """One-vs-all class (Section 2): argmax over classes of the signed score
    (the printed absolute value is read as a typo); ties to the lowest class."""
    return np.argmax(np.asarray(S), axis=1)


def accuracy(pred, truth):
    """eq. (2.1): fraction of test points whose predicted label equals the truth."""
    pred = np.asarray(pred)
    truth = np.asarray(truth)
    return float(np.count_nonzero(pred == truth)) / float(pred.shape[0])


def relres(K, lam, alpha, y):
    """||y - (K + lambda I) alpha|| / ||y|| (per column for a block)."""
    r = y - (K @ alpha + lam * alpha)
    return np.linalg.norm(r, axis=0) / np.linalg.norm(y, axis=0)
