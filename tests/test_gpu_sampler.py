"""The matrix-core sampling kernel (FP32 / FP16-split / BF16-split) against
the oracle's FP64 masked sample, on ragged sizes that exercise every column
pass (r = 32, 64, 256, 288), the point-width variants, the leaf mask and no
mask, and on sampled rows at the full sample width of the 16-Gaussian
workload."""
import numpy as np
import pytest
import torch

import synthdata as sd
from oracle import cluster as oc, cmath
from gpu_util import leaf_ranges, mfma_sample_bound

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _case(n, d, leaf, seed=1):
    X = sd.c2_sixteen_gaussians(n=n, m=1, d=d).X
    t = oc.cluster2mn(X, leaf, seed)
    Xp = np.ascontiguousarray(X[t.perm])
    lb, le = leaf_ranges(t.nodes, n)
    return Xp, lb, le


@pytest.mark.parametrize("prec,split", [("f32", 1), ("f16", 1), ("f16", 2), ("bf16", 1), ("bf16", 2)])
@pytest.mark.parametrize("r", [32, 64, 256, 288])
def test_sampler_all_rows(gpu_lib, prec, split, r):
    n, d, h = 1000, 8, 0.75
    Xp, lb, le = _case(n, d, 100)
    R = sd.random_block(n, r, seed=r)
    S = gpu_lib.kernel_sample(_t(Xp), h, _t(R), _t(lb), _t(le), prec=prec, split_terms=split).cpu().numpy()
    ref = cmath.sample_masked(Xp, R, h, lb, le, np.arange(n))
    rows = np.arange(n)
    bound = mfma_sample_bound(Xp, R, h, lb, le, prec, split, rows)
    assert np.all(np.abs(S - ref) <= bound)


SPLIT_MODES = [("f32", 1), ("f16", 1), ("f16", 2), ("bf16", 1), ("bf16", 2)]


@pytest.mark.parametrize("prec,split", SPLIT_MODES)
@pytest.mark.parametrize("d", [3, 12, 16, 18, 30, 40, 54, 64])
@pytest.mark.parametrize("kind", ["mixture", "smooth"])
def test_sampler_point_widths(gpu_lib, prec, split, d, kind):
    # every narrow instantiation: D = 8 (d 3), D = 16 (d 12, 16: BF16 split
    # exponents in the split modes), D = 32 (18, 30), D = 64 (40, 54, 64).
    # mixture: the 16-Gaussian data with h = 0.35 sqrt(d) (within-cluster
    # kernel values near e^-2 at every width); smooth: one Gaussian cloud
    # (sigma 0.3) with h = 0.4 sqrt(d), so most of each row's sample comes
    # from outside its own leaf.
    n = 777
    if kind == "mixture":
        h = 0.35 * np.sqrt(d)
        Xp, lb, le = _case(n, d, 64)
    else:
        h = 0.4 * np.sqrt(d)
        X = sd.points(n, d, seed=d, scale=0.3)
        t = oc.cluster2mn(X, 64, 1)
        Xp = np.ascontiguousarray(X[t.perm])
        lb, le = leaf_ranges(t.nodes, n)
    R = sd.random_block(n, 64, seed=d)
    S = gpu_lib.kernel_sample(_t(Xp), h, _t(R), _t(lb), _t(le), prec=prec, split_terms=split).cpu().numpy()
    ref = cmath.sample_masked(Xp, R, h, lb, le, np.arange(n))
    if kind == "smooth":
        assert np.abs(ref).mean() > 1.0
    assert np.all(np.abs(S - ref) <= mfma_sample_bound(Xp, R, h, lb, le, prec, split, np.arange(n)))


def test_sampler_no_mask_and_fp64_points(gpu_lib):
    n, d, h = 600, 8, 1.0
    X = sd.c1_two_gaussians(n=n, m=1).X  # FP64 points
    R = sd.random_block(n, 32, seed=9)
    S = gpu_lib.kernel_sample(_t(X), h, _t(R), prec="f16", split_terms=2).cpu().numpy()
    ref = cmath.kmv(X, X, R.astype(np.float64), h)
    lb = np.zeros(n, dtype=np.int32)
    le = np.zeros(n, dtype=np.int32)
    bound = mfma_sample_bound(X.astype(np.float32).astype(np.float64), R, h, lb, le, "f16", 2, np.arange(n))
    # FP32 rounding of the FP64 points adds u |x| per coordinate
    assert np.all(np.abs(S - ref) <= bound + 1e-5 * np.abs(ref).max())


@pytest.mark.parametrize("prec,split", [("f16", 2), ("f32", 1)])
def test_sampler_sampled_rows_large(gpu_lib, prec, split):
    n, h = 1 << 17, 0.75
    Xp, lb, le = _case(n, 8, 128)
    R = sd.random_block(n, 256, seed=3)
    S = gpu_lib.kernel_sample(_t(Xp), h, _t(R), _t(lb), _t(le), prec=prec, split_terms=split).cpu().numpy()
    rows = np.concatenate([np.arange(0, 5), np.random.default_rng(2).choice(n, 20, replace=False),
                           np.arange(n - 5, n)])
    ref = cmath.sample_masked(Xp, R, h, lb, le, rows)
    bound = mfma_sample_bound(Xp, R, h, lb, le, prec, split, rows)
    assert np.all(np.abs(S[rows] - ref) <= bound)


@pytest.mark.parametrize("prec,split", [("f16", 1), ("f16", 2), ("bf16", 2)])
@pytest.mark.parametrize("d,r", [(65, 64), (100, 288), (784, 128)])
def test_sampler_wide_points(gpu_lib, prec, split, d, r):
    # points wider than 64: exponents as a chunked GEMM on the matrix cores,
    # coordinates centred on the mean point; 700 points are 6 row blocks and
    # a ragged panel, r = 288 leaves a ragged last column pass
    n = 700
    if d == 784:
        X = sd.c3_image_like(n=n, m=1).X
        h = 4.0
    else:
        X = sd.points(n, d, seed=d, scale=0.3)
        h = 0.4 * np.sqrt(d)
    t = oc.cluster2mn(X, 64, 1)
    Xp = np.ascontiguousarray(X[t.perm])
    lb, le = leaf_ranges(t.nodes, n)
    R = sd.random_block(n, r, seed=r)
    S = gpu_lib.kernel_sample(_t(Xp), h, _t(R), _t(lb), _t(le), prec=prec, split_terms=split).cpu().numpy()
    rows = np.arange(n)
    ref = cmath.sample_masked(Xp, R, h, lb, le, rows)
    mean = Xp.astype(np.float64).mean(axis=0)
    bound = mfma_sample_bound(Xp, R, h, lb, le, prec, split, rows, anchor=mean)
    assert np.all(np.abs(S - ref) <= bound)
