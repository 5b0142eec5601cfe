"""The seeded generators: reproducible, right shapes, and the stated value
distributions of the stand-in workloads."""
import numpy as np

import synthdata as sd


def test_reproducible_and_independent_streams():
    a = sd.c2_sixteen_gaussians(n=1000, m=100)
    b = sd.c2_sixteen_gaussians(n=1000, m=100)
    assert np.array_equal(a.X, b.X) and np.array_equal(a.Xt, b.Xt)
    assert a.X.dtype == np.float32 and a.X.shape == (1000, 8)
    assert not np.array_equal(a.X[:100], a.Xt)
    assert set(np.unique(a.y)) == {-1.0, 1.0}


def test_small_config_shape():
    p = sd.c1_two_gaussians()
    assert p.X.shape == (1000, 8) and p.X.dtype == np.float64 and p.Xt.shape == (200, 8)
    assert (p.h, p.lam, p.leaf, p.rtol) == (1.0, 1.0, 64, 1e-6)


def test_image_like_statistics():
    p = sd.c3_image_like(n=3000, m=10)
    X = p.X
    assert X.shape == (3000, 784) and X.min() >= 0 and X.max() <= 1
    zero = np.mean(X == 0)
    assert 0.76 < zero < 0.84
    nz = X[X > 0]
    assert abs(nz.mean() - 2 / 7) < 0.01  # Beta(2, 5) mean
    assert p.y.shape == (3000, 10) and np.all(p.y.sum(axis=1) == -8)


def test_ragged_batch_ranges():
    ps = sd.c4_ragged_batch(count=64, m=8)
    ns = np.array([q.n for q in ps])
    assert ns.min() >= 2048 and ns.max() <= 32768
    assert {q.d for q in ps} <= {8, 18, 54}
    assert all(0.5 <= q.h <= 2 and 0.1 <= q.lam <= 10 for q in ps)


def test_random_block_is_signs():
    R = sd.random_block(100, 7, seed=3)
    assert set(np.unique(R)) == {-1.0, 1.0}
