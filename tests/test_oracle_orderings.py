"""Pins for the oracle's NP, KD and PCA orderings (Section 4.3, "Selected
Preprocessing Methods"): closed forms (NP is the complete halving tree of the
natural order), hand-built cases for each split rule (KD: maximum-spread
coordinate, mean split, the 100x imbalance fallback to the median; PCA: the
direction of maximum spread), invariants of every split checked against a
brute-force recomputation with numpy, and tree validity."""
import numpy as np
import pytest

import synthdata as sd
from oracle import cluster as oc


def check_tree(t, n, leaf):
    assert sorted(t.perm.tolist()) == list(range(n))
    nodes = t.nodes
    root = nodes.shape[0] - 1
    assert tuple(nodes[root, :2]) == (0, n)
    for i, (b, e, l, r, par) in enumerate(nodes):
        if l < 0:
            assert e - b <= leaf
        else:
            assert e - b > leaf and l < i and r < i
            assert nodes[l, 0] == b and nodes[l, 1] == nodes[r, 0] and nodes[r, 1] == e
            assert nodes[l, 4] == i and nodes[r, 4] == i


def test_np_is_the_halving_tree():
    X = sd.points(1000, 3, seed=1)
    t = oc.order(X, 64, "np")
    check_tree(t, 1000, 64)
    assert np.array_equal(t.perm, np.arange(1000))
    for b, e, l, r, _ in t.nodes:
        if l >= 0:
            assert t.nodes[l, 1] - b == (e - b) // 2
    # 1000 -> 500 -> 250 -> 125 -> 62/63: 16 leaves, 31 nodes
    assert t.n_nodes == 31 and t.fallbacks == 0


def test_kd_splits_max_spread_coordinate_at_the_mean():
    # spread 10 along x, 1 along y: the root splits x at its mean (4.5 for
    # the values 0..9), so the left part is x <= 4.5 in original order
    xs = np.array([3, 9, 0, 7, 1, 8, 4, 6, 2, 5], dtype=np.float64)
    ys = np.linspace(0, 1, 10)
    X = np.stack([xs, ys], 1)
    t = oc.order(X, 5, "kd")
    left = [i for i in range(10) if xs[i] <= 4.5]
    assert t.perm[:5].tolist() == left
    assert t.perm[5:].tolist() == [i for i in range(10) if xs[i] > 4.5]
    check_tree(t, 10, 5)


def test_kd_falls_back_to_the_median_when_imbalanced():
    # 300 points at 0 and one far outlier: the mean split puts 300 left and 1
    # right (100 * 1 < 300), so the split is at the median: the 150 first in
    # (value, position) order go left
    x = np.zeros(301)
    x[17] = 1000.0
    X = np.stack([x, np.zeros(301)], 1)
    t = oc.order(X, 200, "kd")
    assert t.capped == 1
    root = t.n_nodes - 1
    assert t.nodes[t.nodes[root, 2], 1] == 150
    assert t.perm[:150].tolist() == [i for i in range(301) if i != 17][:150]
    # a milder imbalance (3 : 1) keeps the mean split
    x = np.concatenate([np.zeros(150), np.ones(50)])
    t = oc.order(np.stack([x, np.zeros(200)], 1), 100, "kd")
    assert t.capped == 0 and t.nodes[t.nodes[t.n_nodes - 1, 2], 1] == 150


def test_kd_zero_spread_splits_in_halves():
    t = oc.order(np.ones((40, 3)), 8, "kd")
    check_tree(t, 40, 8)
    assert np.array_equal(t.perm, np.arange(40)) and t.fallbacks == t.n_nodes // 2


def _splits(t, Xp):
    for b, e, l, r, _ in t.nodes:
        if l >= 0:
            yield Xp[b:e], t.nodes[l, 1] - b


def test_kd_split_invariants_brute_force():
    X = sd.c2_sixteen_gaussians(n=3000, m=1, d=5).X.astype(np.float64)
    t = oc.order(X, 40, "kd")
    check_tree(t, 3000, 40)
    Xp = X[t.perm]
    for P, nl in _splits(t, Xp):
        k = int(np.argmax(P.max(0) - P.min(0)))
        key = P[:, k]
        mean = key.mean()
        n0 = int(np.sum(key <= mean))
        if 100 * min(n0, len(key) - n0) < max(n0, len(key) - n0):
            assert nl == len(key) // 2
            assert key[:nl].max() <= key[nl:].min()
        else:
            # the mean computed in another order may differ in the last bit
            assert abs(nl - n0) <= np.sum(np.abs(key - mean) <= 1e-12 * np.abs(key).max())
            assert key[:nl].max() <= mean + 1e-12 * abs(mean) + 1e-300
            assert key[nl:].min() >= mean - 1e-12 * abs(mean)


def test_pca_splits_along_the_dominant_direction():
    # an elongated cloud along u = (3, 4) / 5 with small spread across it: the
    # root split separates points by the sign of (x - mu) . u
    rng = np.random.default_rng(3)
    u = np.array([0.6, 0.8])
    w = np.array([-0.8, 0.6])
    a = rng.standard_normal(500) * 10.0
    c = rng.standard_normal(500) * 0.1
    X = a[:, None] * u + c[:, None] * w
    t = oc.order(X, 300, "pca")
    proj = (X - X.mean(0)) @ u
    left = set(t.perm[:t.nodes[t.nodes[-1, 2], 1]].tolist())
    side = proj <= proj.mean()
    if not side[list(left)].all():  # v may be -u: the left side is then the other one
        side = ~side
    assert left == set(np.nonzero(side)[0].tolist())


def test_pca_split_invariants_brute_force():
    # at every split the left part is the projection <= its mean onto the
    # node's top eigenvector (numpy eigh), except points within rounding of
    # the threshold or where the eigengap is too small for 32 power steps
    X = sd.c2_sixteen_gaussians(n=2500, m=1, d=4).X.astype(np.float64)
    t = oc.order(X, 40, "pca")
    check_tree(t, 2500, 40)
    Xp = X[t.perm]
    checked = 0
    for P, nl in _splits(t, Xp):
        C = (P - P.mean(0)).T @ (P - P.mean(0))
        ev, V = np.linalg.eigh(C)
        if ev[-1] < 4.0 * ev[-2]:
            continue  # (ev2 / ev1)^32 not small: power iteration direction not pinned
        v = V[:, -1]
        p = (P - P.mean(0)) @ v
        lab = p > p.mean()
        if lab[:nl].any() and (~lab[:nl]).any():
            lab = ~lab
        near = np.abs(p - p.mean()) <= 1e-9 * np.abs(p).max()
        assert np.all((lab[:nl] == lab[0]) | near[:nl])
        assert np.all((lab[nl:] != lab[0]) | near[nl:])
        checked += 1
    assert checked >= 3


@pytest.mark.parametrize("method", ["np", "kd", "pca"])
def test_orderings_are_deterministic_and_valid(method):
    X = sd.points(777, 6, seed=9)
    t1 = oc.order(X, 32, method)
    t2 = oc.order(X, 32, method)
    check_tree(t1, 777, 32)
    assert np.array_equal(t1.perm, t2.perm) and np.array_equal(t1.nodes, t2.nodes)
    # a single leaf and leaf size 1
    t = oc.order(X[:20], 32, method)
    assert t.n_nodes == 1
    check_tree(oc.order(X[:33], 1, method), 33, 1)
