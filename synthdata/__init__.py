"""Seeded synthetic inputs for the Gaussian-kernel ridge regression workloads.

This module only draws random numbers and lays them out; it contains none of
the method's arithmetic (no kernel values, no clustering, no solves).  Both the
CPU oracle and the GPU path take their inputs from here, so a test can hand the
very same arrays to each side.

The paper evaluates on UCI / LIBSVM datasets (SUSY, HEPMASS, COVTYPE, GAS, PEN,
LETTER, MNIST; Section 5.1) which are not available here.  The generators below
stand in for them with Gaussian mixtures and image-like sparse vectors of the
same dimensions (d = 8 for SUSY, 784 for MNIST, 18 / 54 for the wider tabular
sets).  No dataset item is reproduced.

Every array comes from numpy's PCG64 generator keyed by (base seed + config
index, stream index), so the train, test and auxiliary arrays of a config are
independent streams and reproducible across runs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 180310274

# stream indices inside one config's seed sequence
_S_TRAIN, _S_TEST, _S_MEANS, _S_AUX, _S_BLOCK = 0, 1, 2, 3, 4


def _rng(config: int, stream: int, extra: int = 0) -> np.random.Generator:
    return np.random.Generator(
        np.random.PCG64(np.random.SeedSequence([BASE_SEED + config, stream, extra])))


@dataclass
class Problem:
    """One kernel ridge regression problem: training/test data plus parameters."""
    name: str
    X: np.ndarray            # n x d, row-major
    y: np.ndarray            # n (binary +-1) or n x c (one-vs-all +-1)
    Xt: np.ndarray           # m x d test / validation points
    yt: np.ndarray           # m labels (+-1, or class index for multi-class)
    h: float
    lam: float
    leaf: int
    rtol: float
    r0: int = 256
    classes: int = 2
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def d(self) -> int:
        return self.X.shape[1]


def _mixture(rng, n, means, sigma, dtype):
    comp = rng.integers(0, means.shape[0], size=n)
    noise = rng.standard_normal((n, means.shape[1]))
    X = means[comp] + sigma * noise
    return X.astype(dtype), comp


def c1_two_gaussians(n: int = 1000, m: int = 200, d: int = 8, config: int = 0,
                     dtype=np.float64) -> Problem:
    """Two isotropic Gaussians with means +1 and -1 on every axis, sigma 1;
    label = +1 for the first component, -1 for the second."""
    means = np.stack([np.ones(d), -np.ones(d)])
    X, cx = _mixture(_rng(config, _S_TRAIN), n, means, 1.0, dtype)
    Xt, ct = _mixture(_rng(config, _S_TEST), m, means, 1.0, dtype)
    y = np.where(cx == 0, 1.0, -1.0)
    yt = np.where(ct == 0, 1.0, -1.0)
    return Problem("two_gaussians", X, y, Xt, yt, h=1.0, lam=1.0, leaf=64, rtol=1e-6)


def c2_sixteen_gaussians(n: int = 1 << 20, m: int = 100_000, d: int = 8,
                         config: int = 1) -> Problem:
    """Sixteen Gaussians, means uniform in [-3, 3]^d, sigma 0.5; label +1 for an
    even component index, -1 for an odd one.  FP32 points."""
    means = _rng(config, _S_MEANS).uniform(-3.0, 3.0, size=(16, d))
    X, cx = _mixture(_rng(config, _S_TRAIN), n, means, 0.5, np.float32)
    Xt, ct = _mixture(_rng(config, _S_TEST), m, means, 0.5, np.float32)
    y = np.where(cx % 2 == 0, 1.0, -1.0)
    yt = np.where(ct % 2 == 0, 1.0, -1.0)
    return Problem("sixteen_gaussians", X, y, Xt, yt, h=0.75, lam=10.0, leaf=128,
                   rtol=1e-2, r0=256, extra={"means": means})


def c3_image_like(n: int = 60_000, m: int = 10_000, d: int = 784, classes: int = 10,
                  config: int = 2) -> Problem:
    """Image-like vectors in [0, 1]: each class has a seeded support mask over 20%
    of the pixels; a sample keeps a support pixel with probability 0.85 and
    lights an off-support pixel with probability 0.0125 (about 80% exact zeros);
    nonzero values are Beta(2, 5).  Ten one-vs-all right-hand sides."""
    masks = _rng(config, _S_MEANS).random((classes, d)) < 0.2

    def draw(rng, count):
        cls = rng.integers(0, classes, size=count)
        on = np.where(masks[cls], rng.random((count, d)) < 0.85,
                      rng.random((count, d)) < 0.0125)
        vals = rng.beta(2.0, 5.0, size=(count, d))
        return np.where(on, vals, 0.0).astype(np.float32), cls

    X, cx = draw(_rng(config, _S_TRAIN), n)
    Xt, ct = draw(_rng(config, _S_TEST), m)
    Y = np.where(cx[:, None] == np.arange(classes)[None, :], 1.0, -1.0)
    return Problem("image_like", X, Y, Xt, ct.astype(np.int64), h=4.0, lam=1.0,
                   leaf=128, rtol=1e-2, classes=classes)


def c4_ragged_batch(count: int = 64, n_lo: int = 2048, n_hi: int = 32768,
                    dims=(8, 18, 54), m: int = 256, config: int = 3) -> list[Problem]:
    """Many independent problems: n log-uniform in [n_lo, n_hi], d drawn from
    `dims`, the two-Gaussian mixture of the small config generalised to d,
    h uniform in [0.5, 2], lambda uniform in [0.1, 10].  FP32 points."""
    aux = _rng(config, _S_AUX)
    ns = np.exp(aux.uniform(math.log(n_lo), math.log(n_hi), size=count)).astype(np.int64)
    ds = aux.choice(np.asarray(dims), size=count)
    hs = aux.uniform(0.5, 2.0, size=count)
    lams = aux.uniform(0.1, 10.0, size=count)
    out = []
    for i in range(count):
        d = int(ds[i])
        means = np.stack([np.ones(d), -np.ones(d)])
        X, cx = _mixture(_rng(config, _S_TRAIN, i), int(ns[i]), means, 1.0, np.float32)
        Xt, ct = _mixture(_rng(config, _S_TEST, i), m, means, 1.0, np.float32)
        out.append(Problem(f"ragged_{i}", X, np.where(cx == 0, 1.0, -1.0), Xt,
                           np.where(ct == 0, 1.0, -1.0), h=float(hs[i]),
                           lam=float(lams[i]), leaf=128, rtol=1e-2))
    return out


def c5_eight_gaussians(n: int = 131_072, m: int = 16_384, d: int = 18,
                       config: int = 4) -> Problem:
    """Eight Gaussians, means uniform in [-3, 3]^d, sigma 1; label by component
    parity.  FP32 points; the held-out set is the validation set.  The
    evaluation point (h, lambda) = (2, 1)."""
    means = _rng(config, _S_MEANS).uniform(-3.0, 3.0, size=(8, d))
    X, cx = _mixture(_rng(config, _S_TRAIN), n, means, 1.0, np.float32)
    Xt, ct = _mixture(_rng(config, _S_TEST), m, means, 1.0, np.float32)
    return Problem("eight_gaussians", X, np.where(cx % 2 == 0, 1.0, -1.0), Xt,
                   np.where(ct % 2 == 0, 1.0, -1.0), h=2.0, lam=1.0, leaf=128,
                   rtol=1e-2)


def random_block(n: int, r: int, seed: int = 0, kind: str = "rademacher",
                 dtype=np.float32) -> np.ndarray:
    """An n x r random block for sampling tests: +-1 entries (rademacher) or
    standard normals (normal)."""
    rng = _rng(99, _S_BLOCK, seed)
    if kind == "rademacher":
        return np.where(rng.random((n, r)) < 0.5, -1.0, 1.0).astype(dtype)
    return rng.standard_normal((n, r)).astype(dtype)


def points(n: int, d: int, seed: int = 0, scale: float = 1.0,
           dtype=np.float32) -> np.ndarray:
    """Plain standard-normal points scaled by `scale` (for edge-case tests)."""
    return (scale * _rng(98, _S_AUX, seed).standard_normal((n, d))).astype(dtype)


def vectors(n: int, k: int, seed: int = 0, dtype=np.float64) -> np.ndarray:
    """Plain standard-normal right-hand sides / weights, n x k."""
    return _rng(97, _S_AUX, seed).standard_normal((n, k)).astype(dtype)
