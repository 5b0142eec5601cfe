"""Pins for the C matrix-free FP64 kernel products: brute force on small inputs
written out here with explicit loops (not the oracle's dense code path)."""
import math

import numpy as np

import synthdata as sd
from oracle import cmath


def _brute(X, Y, W, h):
    out = np.zeros((X.shape[0], W.shape[1]))
    for i in range(X.shape[0]):
        for j in range(Y.shape[0]):
            q = sum((X[i, k] - Y[j, k]) ** 2 for k in range(X.shape[1]))
            out[i] += math.exp(-q / (2 * h * h)) * W[j]
    return out


def test_kmv_brute_force():
    X = sd.points(13, 3, seed=2).astype(np.float64)
    Y = sd.points(17, 3, seed=3).astype(np.float64)
    W = sd.vectors(17, 2, seed=4)
    got = cmath.kmv(X, Y, W, 0.8)
    np.testing.assert_allclose(got, _brute(X, Y, W, 0.8), rtol=1e-13, atol=1e-14)
    rows = np.array([5, 0, 12])
    np.testing.assert_allclose(cmath.kmv(X, Y, W, 0.8, rows=rows), got[rows], rtol=0, atol=0)


def test_sample_masked_brute_force():
    X = sd.points(20, 2, seed=5).astype(np.float64)
    R = sd.random_block(20, 4, seed=1).astype(np.float64)
    lb = np.array([0] * 7 + [7] * 6 + [13] * 7)
    le = np.array([7] * 7 + [13] * 6 + [20] * 7)
    rows = np.arange(20)
    got = cmath.sample_masked(X, R, 1.1, lb, le, rows)
    for i in range(20):
        keep = [j for j in range(20) if not (lb[i] <= j < le[i])]
        exp = _brute(X[i:i + 1], X[keep], R[keep], 1.1)[0]
        np.testing.assert_allclose(got[i], exp, rtol=1e-13, atol=1e-14)


def test_residual_zero_for_exact_solution():
    # alpha = y / (1 + lam) is exact when K = I (h -> 0 with distinct points)
    X = sd.points(50, 4, seed=6).astype(np.float64)
    y = sd.vectors(50, 1, seed=7)[:, 0]
    r = cmath.residual(X, y / 1.5, y, 1e-3, 0.5)
    assert np.max(np.abs(r)) < 1e-15
