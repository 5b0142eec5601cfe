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


def test_kmv_brute_force_wide_points():
    # widths of the wide-point products (d = 100, 784) on a tiny grid, so a
    # stride or loop-bound slip past the first coordinates shows
    for d, h in ((100, 3.0), (784, 4.0)):
        X = sd.points(5, d, seed=d, scale=0.3).astype(np.float64)
        Y = sd.points(7, d, seed=d + 1, scale=0.3).astype(np.float64)
        W = sd.vectors(7, 3, seed=d + 2)
        np.testing.assert_allclose(cmath.kmv(X, Y, W, h), _brute(X, Y, W, h), rtol=1e-12, atol=1e-14)


def test_kmv_closed_forms():
    # eq. (1.1) at coincident points is 1, so K W is the column sums of W; at
    # points much farther apart than h it is 0 off the coincident pairs
    x = sd.points(1, 9, seed=8).astype(np.float64)
    W = sd.vectors(6, 2, seed=9)
    np.testing.assert_allclose(cmath.kmv(np.repeat(x, 4, axis=0), np.repeat(x, 6, axis=0), W, 0.7),
                               np.tile(W.sum(axis=0), (4, 1)), rtol=1e-15, atol=0)
    far = np.arange(6, dtype=np.float64)[:, None] * np.full((1, 3), 100.0)
    np.testing.assert_allclose(cmath.kmv(far, far, W, 1.0), W, rtol=0, atol=0)


def test_kmv_invariances():
    # the kernel depends on |x - y| / h only: translating both sets, or
    # scaling points and h together, leaves K W unchanged; K(X, Y) = K(Y, X)^T
    X = sd.points(11, 5, seed=10).astype(np.float64)
    Y = sd.points(8, 5, seed=11).astype(np.float64)
    W = sd.vectors(8, 2, seed=12)
    ref = cmath.kmv(X, Y, W, 0.9)
    shift = np.array([3.0, -2.0, 0.5, 7.0, -1.25])
    np.testing.assert_allclose(cmath.kmv(X + shift, Y + shift, W, 0.9), ref, rtol=1e-12)
    np.testing.assert_allclose(cmath.kmv(2.5 * X, 2.5 * Y, W, 2.25), ref, rtol=1e-12)
    KXY = cmath.kmv(X, Y, np.eye(8), 0.9)
    KYX = cmath.kmv(Y, X, np.eye(11), 0.9)
    np.testing.assert_allclose(KXY, KYX.T, rtol=0, atol=0)


def test_sample_masked_empty_mask_is_the_product():
    # with every leaf range empty nothing is skipped: the sample is K R
    X = sd.points(30, 4, seed=13).astype(np.float64)
    R = sd.random_block(30, 5, seed=2).astype(np.float64)
    rows = np.array([29, 3, 0, 17])
    z = np.zeros(30, dtype=np.int64)
    got = cmath.sample_masked(X, R, 0.6, z, z, rows)
    np.testing.assert_allclose(got, cmath.kmv(X, X, R, 0.6, rows=rows), rtol=1e-14, atol=1e-15)
