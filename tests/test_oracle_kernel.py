"""Pins for the dense FP64 oracle (eq. (1.1), Algorithm 1, eq. (2.1)) against
closed forms and limits that do not reuse the oracle's own code."""
import math

import numpy as np
import pytest

import synthdata as sd
from oracle import kernel as ok


def test_kernel_closed_form_pairs():
    # ||x - y||^2 = 2 h^2  =>  K = e^{-1};  ||x - y||^2 = 0  =>  K = 1
    h = 0.7
    X = np.array([[0.0, 0.0], [h, h], [0.0, 0.0]])
    K = ok.kernel_dense(X, X, h)
    assert K[0, 1] == pytest.approx(math.exp(-1.0), rel=1e-15)
    assert K[0, 2] == 1.0
    assert K[1, 1] == 1.0
    # a 3-4-5 triangle at h = 5/sqrt(2): K = exp(-25/25) = e^{-1}
    Y = np.array([[3.0, 4.0]])
    assert ok.kernel_dense(np.zeros((1, 2)), Y, 5 / math.sqrt(2))[0, 0] == \
        pytest.approx(math.exp(-1.0), rel=1e-15)


def test_kernel_structure():
    # symmetric, unit diagonal, entries in (0, 1], positive semidefinite
    X = sd.points(150, 5, seed=1)
    K = ok.kernel_dense(X, X, 1.3)
    assert np.array_equal(K, K.T)
    assert np.all(np.diag(K) == 1.0)
    assert K.min() > 0.0 and K.max() <= 1.0
    assert np.linalg.eigvalsh(K).min() > -1e-12


def test_h_to_zero_identity():
    # Section 1: K -> I as h -> 0; in FP64 the off-diagonals underflow to 0
    p = sd.c1_two_gaussians(n=300, m=50)
    K = ok.kernel_dense(p.X, p.X, 1e-3)
    assert np.array_equal(K, np.eye(300))
    lam = 0.5
    a = ok.krr_solve_dense(K, p.y, lam)
    np.testing.assert_allclose(a, p.y / (1 + lam), rtol=1e-15)
    assert np.all(ok.scores(p.Xt, p.X, a, 1e-3) == 0.0)


def test_h_to_infinity_rank_one():
    # Section 1: K -> 1 1^T; Sherman-Morrison gives
    # (1 1^T + lam I)^{-1} y = (y - 1 sum(y) / (n + lam)) / lam
    p = sd.c1_two_gaussians(n=400, m=60)
    lam = 2.0
    a = ok.krr_fit_dense(p.X, p.y, 1e4, lam)
    n = p.n
    closed = (p.y - p.y.sum() / (n + lam)) / lam
    assert np.linalg.norm(a - closed) / np.linalg.norm(closed) < 1e-4
    s = ok.scores(p.Xt, p.X, a, 1e4)
    assert np.all(ok.labels_binary(s) == (1.0 if p.y.sum() >= 0 else -1.0))


def test_two_point_solve_closed_form():
    # n = 2: K = [[1, k], [k, 1]]; (K + lam I)^{-1} by the 2x2 inverse formula
    h, lam = 0.9, 0.3
    X = np.array([[0.1, -0.2], [0.5, 0.4]])
    y = np.array([1.0, -1.0])
    k = math.exp(-((0.4) ** 2 + (0.6) ** 2) / (2 * h * h))
    a11 = 1 + lam
    det = a11 * a11 - k * k
    expect = np.array([(a11 * y[0] - k * y[1]) / det, (a11 * y[1] - k * y[0]) / det])
    np.testing.assert_allclose(ok.krr_fit_dense(X, y, h, lam), expect, rtol=1e-14)


def test_accuracy_and_sign_rule():
    assert ok.accuracy([1, -1, 1, 1], [1, 1, 1, -1]) == 0.5
    assert list(ok.labels_binary([0.0, -1e-300, 2.0])) == [1.0, -1.0, 1.0]
    S = np.array([[0.1, 0.3, 0.3], [-2.0, -1.0, -3.0]])
    assert list(ok.labels_one_vs_all(S)) == [1, 1]


def test_small_config_accuracy_below_bayes():
    # two Gaussians +-1 per axis, sigma 1, d = 8: Bayes accuracy Phi(sqrt(8)) = 0.99766
    p = sd.c1_two_gaussians()
    a = ok.krr_fit_dense(p.X, p.y, p.h, p.lam)
    acc = ok.accuracy(ok.labels_binary(ok.scores(p.Xt, p.X, a, p.h)), p.yt)
    bayes = 0.5 * (1 + math.erf(math.sqrt(8) / math.sqrt(2)))
    assert bayes == pytest.approx(0.99766, abs=1e-5)
    # at most bayes + 3 binomial standard deviations on m = 200 test points
    assert 0.93 <= acc <= bayes + 3 * math.sqrt(bayes * (1 - bayes) / 200) + 1e-12
