"""FP64 matrix-free Gaussian-kernel products on the CPU (C + OpenMP).

Test infrastructure only (see the package docstring).  Used where n is too
large for a dense K: residual certification of a solution and sampled rows of
the HSS sampling product."""
import ctypes

import numpy as np

from ._clib import lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def kmv(X, Y, W, h, rows=None):
    """Out = K(X, Y; h) W with K of eq. (1.1), entry by entry, FP64.

    rows: optional subset of row indices of X (returns len(rows) x nrhs)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    vec = W.ndim == 1
    W = np.ascontiguousarray(W.reshape(W.shape[0], -1))
    assert X.shape[1] == Y.shape[1] and W.shape[0] == Y.shape[0]
    if rows is None:
        r = None
        m = X.shape[0]
    else:
        r = np.ascontiguousarray(rows, dtype=np.int64)
        m = r.shape[0]
    out = np.empty((m, W.shape[1]))
    lib().oracle_kmv(_p(X), _p(Y), Y.shape[0], X.shape[1], float(h), _p(W), W.shape[1],
                     None if r is None else _p(r), m, _p(out))
    return out[:, 0] if vec else out


def residual(X, alpha, y, h, lam, rows=None):
    """y - (K + lambda I) alpha, matrix-free in FP64 (optionally on a row subset)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    Ka = kmv(X, X, alpha, h, rows=rows)
    if rows is None:
        return y - Ka - lam * alpha
    return y[rows] - Ka - lam * alpha[rows]


def sample_masked(X, R, h, leaf_begin, leaf_end, rows):
    """Rows of the off-diagonal sample S = K(X, X) R where each row i skips the
    columns of its own leaf [leaf_begin[i], leaf_end[i]) (Section 3.1)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64)
    lb = np.ascontiguousarray(leaf_begin, dtype=np.int64)
    le = np.ascontiguousarray(leaf_end, dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((rows.shape[0], R.shape[1]))
    lib().oracle_sample_masked(_p(X), X.shape[0], X.shape[1], float(h), _p(R), R.shape[1],
                               _p(lb), _p(le), _p(rows), rows.shape[0], _p(out))
    return out
