"""GPU recursive two-means ordering: bit-exact against the oracle's spec
(permutation, tree and statistics) on every workload shape, and the
degenerate inputs (all-equal points, n <= leaf, leaf = 1)."""
import numpy as np
import pytest
import torch

import synthdata as sd
from oracle import cluster as oc

pytestmark = pytest.mark.gpu


def _run(krr, X, leaf, seed, max_iter=100):
    Xg = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    perm, tree = krr.cluster_2mn(Xg, leaf, seed, max_iter)
    torch.cuda.synchronize()
    ref = oc.cluster2mn(X, leaf, seed, max_iter)
    return perm.cpu().numpy(), tree, ref


def _assert_same(perm, tree, ref):
    assert np.array_equal(perm, ref.perm)
    assert np.array_equal(tree.nodes, ref.nodes)
    assert tuple(tree.stats[:3]) == (ref.fallbacks, ref.capped, ref.iterations)


@pytest.mark.parametrize("seed", [0, 11])
def test_small_fp64(gpu_lib, seed):
    p = sd.c1_two_gaussians()
    _assert_same(*_run(gpu_lib, p.X, p.leaf, seed))


def test_sixteen_gaussians_fp32(gpu_lib):
    p = sd.c2_sixteen_gaussians(n=50_000, m=1)
    _assert_same(*_run(gpu_lib, p.X, 128, 3))


def test_image_like_wide(gpu_lib):
    p = sd.c3_image_like(n=3000, m=1)
    _assert_same(*_run(gpu_lib, p.X, 128, 5))


def test_iteration_cap(gpu_lib):
    p = sd.c2_sixteen_gaussians(n=20_000, m=1)
    perm, tree, ref = _run(gpu_lib, p.X, 64, 9, max_iter=2)
    _assert_same(perm, tree, ref)
    assert ref.capped > 0


def test_degenerate(gpu_lib):
    _assert_same(*_run(gpu_lib, np.ones((100, 4)), 10, 1))
    _assert_same(*_run(gpu_lib, sd.points(10, 3), 16, 0))
    _assert_same(*_run(gpu_lib, sd.points(33, 2, seed=4), 1, 2))
    # duplicated points: many exact ties in the assignment
    X = np.repeat(sd.points(40, 3, seed=5), 7, axis=0)
    _assert_same(*_run(gpu_lib, X, 16, 4))


def test_full_size_sixteen_gaussians(gpu_lib):
    p = sd.c2_sixteen_gaussians(m=1)
    _assert_same(*_run(gpu_lib, p.X, 128, 7))
