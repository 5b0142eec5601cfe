"""The orderings the paper compares with recursive two-means (Section 4.3,
"Selected Preprocessing Methods": NP, KD with its median fallback, PCA) on
the GPU against the oracle: permutation and tree bit-exact, for FP32 and FP64
points, clustered and smooth data, data with many ties (KD median splits),
forests of ragged problems, and one size where every level runs many nodes.
Then the paper's memory / rank comparison (Table 2) on a synthetic stand-in:
the HSS memory and maximum rank of each ordering."""
import numpy as np
import pytest
import torch

import synthdata as sd
from oracle import cluster as oc

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _same(gpu_lib, X, leaf, method, offsets=None):
    perm, tree = gpu_lib.cluster_order(_t(X), leaf, method, offsets=offsets)
    perm = perm.cpu().numpy()
    if offsets is None:
        t = oc.order(X, leaf, method)
        np.testing.assert_array_equal(perm, t.perm)
        np.testing.assert_array_equal(tree.nodes, t.nodes)
        st = tree.stats
        assert st[0] == t.fallbacks and st[1] == t.capped, (st, t.fallbacks, t.capped)
        return t
    for k in range(len(offsets) - 1):
        a, b = offsets[k], offsets[k + 1]
        t = oc.order(X[a:b], leaf, method)
        np.testing.assert_array_equal(perm[a:b] - a, t.perm)
    return None


def _tied(n, d, seed):
    # coordinates on a coarse grid (many equal values), and coordinate 0 zero
    # except for one point in 200 far out: the first KD split is more than
    # 100x unbalanced, so it takes the median, with ties at the median value
    X = np.round(sd.points(n, d, seed=seed) * 2.0) / 2.0
    X[:, 0] = 0.0
    X[::200, 0] = 1000.0
    return X.astype(np.float32)


@pytest.mark.parametrize("method", ["np", "kd", "pca"])
@pytest.mark.parametrize("data", ["mixture32", "two_gauss64", "smooth32", "tied32"])
def test_ordering_bit_exact(gpu_lib, method, data):
    if data == "mixture32":
        X = sd.c2_sixteen_gaussians(n=5000, m=1, d=8).X
    elif data == "two_gauss64":
        X = sd.c1_two_gaussians(n=3001, m=1).X
    elif data == "smooth32":
        X = sd.points(4097, 5, seed=3, scale=0.5)
    else:
        X = _tied(6000, 3, 5)
    t = _same(gpu_lib, X, 64, method)
    if method == "kd" and data == "tied32":
        assert t.capped > 0  # the median path ran


@pytest.mark.parametrize("method", ["kd", "pca"])
def test_ordering_bit_exact_large(gpu_lib, method):
    X = sd.c2_sixteen_gaussians(n=1 << 17, m=1).X
    _same(gpu_lib, X, 128, method)


@pytest.mark.parametrize("method", ["np", "kd", "pca"])
def test_ordering_forest(gpu_lib, method):
    sizes = [40, 777, 3000, 129, 2048]
    Xs = [sd.c2_sixteen_gaussians(n=s, m=1, d=6, config=10 + i).X for i, s in enumerate(sizes)]
    Xs[2] = _tied(3000, 6, 8)
    X = np.concatenate(Xs)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    _same(gpu_lib, X, 64, method, offsets=off)


def test_ordering_degenerate(gpu_lib):
    # all points equal: KD and PCA fall back to halves everywhere; n <= leaf
    X = np.ones((300, 4), dtype=np.float32)
    for m in ("kd", "pca"):
        t = _same(gpu_lib, X, 16, m)
        assert np.array_equal(t.perm, np.arange(300)) and t.fallbacks == t.n_nodes // 2
    for m in ("np", "kd", "pca"):
        _same(gpu_lib, sd.points(10, 3, seed=1), 16, m)
        _same(gpu_lib, sd.points(33, 2, seed=2), 1, m)


def test_ordering_memory_comparison(gpu_lib):
    # Table 2 on a synthetic stand-in (16-Gaussian data, 10,000 points, leaf
    # 16, tolerance 0.1): the HSS memory and maximum rank of each ordering.
    # As in the paper, the natural order needs the most memory and every
    # clustering saves a large factor; which clustering is best depends on the
    # data (here PCA and KD come out slightly ahead of 2MN).
    p = sd.c2_sixteen_gaussians(n=10000, m=1)
    X = _t(p.X)
    mem, rank = {}, {}
    for m in ("np", "kd", "pca", "2mn"):
        perm, tree = gpu_lib.cluster_order(X, 16, m)
        Xp = gpu_lib.gather_rows(X, perm)
        H = gpu_lib.HSS(tree, Xp, p.h, gpu_lib.HssOptions(rtol=0.1, r0=128, dr=128, prec="f32"))
        mem[m], rank[m] = H.stats.bytes_paper, H.stats.max_rank
    print("HSS memory (MB) by ordering:", {k: round(v / 1e6, 2) for k, v in mem.items()}, "max rank:", rank)
    assert mem["2mn"] < mem["np"]
    assert min(mem["kd"], mem["pca"], mem["2mn"]) < mem["np"]
