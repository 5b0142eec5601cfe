"""Pins for the recursive two-means (2MN) oracle (Sections 4.2-4.3, Fig. 3).

The exact permutation is this project's seeded spec; what the paper fixes --
recursive splits into consecutive ranges down to the leaf size, Lloyd
iterations run to a fixed point, a postorder tree -- is checked here with
independent code, plus brute force on separated groups."""
import math

import numpy as np
import pytest

import synthdata as sd
from oracle import cluster as oc


def check_tree(t, n, leaf):
    """Valid permutation; children partition parents; leaf sizes; postorder."""
    assert np.array_equal(np.sort(t.perm), np.arange(n))
    nodes = t.nodes
    root = nodes.shape[0] - 1
    assert nodes[root, 0] == 0 and nodes[root, 1] == n and nodes[root, 4] == -1
    nleaves = 0
    covered = np.zeros(n, dtype=int)
    for i in range(nodes.shape[0]):
        b, e, l, r, p = nodes[i]
        if l < 0:
            assert r < 0 and 0 < e - b <= leaf
            covered[b:e] += 1
            nleaves += 1
        else:
            assert e - b > leaf
            assert l < i and r < i  # postorder: children before parent
            assert nodes[l, 0] == b and nodes[l, 1] == nodes[r, 0] and nodes[r, 1] == e
            assert nodes[l, 1] > b and nodes[r, 1] > nodes[r, 0]
            assert nodes[l, 4] == i and nodes[r, 4] == i
    assert np.all(covered == 1)
    assert nodes.shape[0] == 2 * nleaves - 1


def lloyd_violations(Xp, t):
    """Count points of internal nodes that are not on their own centroid's side."""
    bad = 0
    for i in range(t.n_nodes):
        b, e, l, r, _ = t.nodes[i]
        if l < 0:
            continue
        m = t.nodes[l, 1]
        c0 = Xp[b:m].mean(axis=0)
        c1 = Xp[m:e].mean(axis=0)
        d0 = ((Xp[b:e] - c0) ** 2).sum(axis=1)
        d1 = ((Xp[b:e] - c1) ** 2).sum(axis=1)
        tol = 1e-9 * (d0 + d1)
        s = m - b
        bad += int(np.count_nonzero(d0[:s] > d1[:s] + tol[:s]))
        bad += int(np.count_nonzero(d1[s:] >= d0[s:] + tol[s:]))
    return bad


def test_splitmix64_published_sequence():
    # SplitMix64 from state 0 (Steele, Lea, Flood 2014): first three outputs
    g = 0x9E3779B97F4A7C15
    assert oc.sm_step(0) == 0xE220A8397B1DCDAF
    assert oc.sm_step(g) == 0x6E789E6AA1B965F4
    assert oc.sm_step((2 * g) % 2**64) == 0x06C45D188009454F


def test_isqrt64_matches_math_isqrt():
    rng = np.random.default_rng(0)
    vals = [0, 1, 2, 3, 4, 15, 16, 17, 2**62 - 1, 2**62, 2**63, 2**64 - 1]
    vals += [int(v) for v in rng.integers(0, 2**63, size=2000, dtype=np.int64)]
    vals += [k * k + off for k in (3, 1 << 20, (1 << 31) + 5) for off in (-1, 0, 1)]
    for v in vals:
        assert oc.isqrt64(v) == math.isqrt(v)


@pytest.mark.parametrize("seed", [0, 11])
def test_small_config_tree_and_fixed_point(seed):
    p = sd.c1_two_gaussians()
    t = oc.cluster2mn(p.X, p.leaf, seed)
    check_tree(t, p.n, p.leaf)
    assert t.fallbacks == 0 and t.capped == 0
    assert lloyd_violations(p.X[t.perm].astype(np.float64), t) == 0


def test_deterministic_and_seed_dependent():
    X = sd.c2_sixteen_gaussians(n=5000, m=1).X
    a = oc.cluster2mn(X, 128, 5)
    b = oc.cluster2mn(X, 128, 5)
    c = oc.cluster2mn(X, 128, 6)
    assert np.array_equal(a.perm, b.perm) and np.array_equal(a.nodes, b.nodes)
    check_tree(c, 5000, 128)
    assert not np.array_equal(a.perm, c.perm)
    assert lloyd_violations(X[a.perm].astype(np.float64), a) == 0


def test_separated_groups_brute_force():
    # two tight groups far apart: the root split must be exactly the groups,
    # for every seed, and the split keeps each group's relative order
    rng = np.random.default_rng(3)
    for trial in range(20):
        g0 = rng.normal(0, 0.01, size=(5 + trial % 3, 3))
        g1 = rng.normal(100, 0.01, size=(7 - trial % 3, 3))
        X = np.vstack([g0, g1])
        order = rng.permutation(X.shape[0])
        X = X[order]
        is_g0 = order < g0.shape[0]
        t = oc.cluster2mn(X, 7, trial)
        root = t.n_nodes - 1
        left = t.nodes[root, 2]
        m = t.nodes[left, 1]
        first = set(is_g0[t.perm[:m]].tolist())
        second = set(is_g0[t.perm[m:]].tolist())
        assert len(first) == 1 and len(second) == 1 and first != second
        assert np.all(np.diff(t.perm[:m]) > 0) and np.all(np.diff(t.perm[m:]) > 0)


def test_degenerate_inputs():
    # all points equal: every split falls back to halves by position
    X = np.ones((100, 4))
    t = oc.cluster2mn(X, 10, 1)
    check_tree(t, 100, 10)
    assert t.fallbacks == t.n_nodes // 2
    assert np.array_equal(t.perm, np.arange(100))
    root = t.n_nodes - 1
    assert t.nodes[t.nodes[root, 2], 1] == 50
    # n <= leaf: a single leaf
    t = oc.cluster2mn(sd.points(10, 3), 16, 0)
    assert t.n_nodes == 1 and tuple(t.nodes[0, :4]) == (0, 10, -1, -1)
    # leaf size 1 on distinct points: a full binary tree over singletons
    t = oc.cluster2mn(sd.points(33, 2, seed=4), 1, 2)
    check_tree(t, 33, 1)


def test_second_seed_weights_hand_computed():
    # Node of three 1-D points at 0, 1, 3 (Section 4.3: the second seed is
    # drawn proportionally to the distance from the first).  With the first
    # seed at 0: q = (0, 1, 9), qmax = 9 = 0.5625 * 2^4, so the weights are
    # isqrt(q * 2^58) = (0, 2^29, 3 * 2^29), exactly the distances 0 : 1 : 3.
    # Squared-distance weights would give 0 : 1 : 9.
    pts = np.array([0.0, 1.0, 3.0])
    for s in range(200):
        i1, i2, w = oc.seeds(pts, 0, 3, s)
        if i1 == 0:
            assert list(w) == [0, 2**29, 3 * 2**29]
            break
    else:
        pytest.fail("no seed put the first centre at position 0")
    # First seed at 1 (x = 1): q = (1, 0, 4), qmax = 4 = 0.5 * 2^3, shift 59:
    # weights (2^29.5 floored, 0, 2^30.5 floored) = (isqrt(2^59), 0, isqrt(2^61)).
    # isqrt(2^59) = floor(2^29 sqrt 2) = 759250124 (2^29 * 1.41421356237 =
    # 759250124.99), isqrt(2^61) = floor(2^30 sqrt 2) = 1518500249.
    for s in range(200):
        i1, i2, w = oc.seeds(pts, 0, 3, s)
        if i1 == 1:
            assert list(w) == [759250124, 0, 1518500249]
            break
    else:
        pytest.fail("no seed put the first centre at position 1")
    # Every point equal: no second seed (the fallback split applies).
    i1, i2, w = oc.seeds(np.zeros((5, 2)), 0, 5, 7)
    assert 0 <= i1 < 5 and i2 == -1 and not w.any()


def test_second_seed_distribution_follows_distance():
    # Tally the seeds the C oracle itself draws on the node 0 / 1 / 3 over
    # many seeds.  Conditional on the first seed, the second seed lands on
    # each other point with probability distance / (sum of distances):
    #   first at 0: P(3) = 3 / 4   (squared distance would give 9 / 10)
    #   first at 1: P(3) = 2 / 3   (squared: 4 / 5)
    #   first at 3: P(0) = 3 / 5   (squared: 9 / 13)
    pts = np.array([0.0, 1.0, 3.0])
    hits = {0: [0, 0], 1: [0, 0], 2: [0, 0]}   # first seed -> [draws, hits]
    target = {0: 2, 1: 2, 2: 0}
    for s in range(6000):
        i1, i2, _ = oc.seeds(pts, 0, 3, s)
        assert i2 != i1 and 0 <= i2 < 3
        hits[i1][0] += 1
        hits[i1][1] += int(i2 == target[i1])
    for i1, p in ((0, 3 / 4), (1, 2 / 3), (2, 3 / 5)):
        n, k = hits[i1]
        assert n > 1500
        sigma = math.sqrt(p * (1 - p) / n)
        assert abs(k / n - p) < 4.5 * sigma, (i1, k / n, p)
    # The same node embedded in a bigger array draws within its own range.
    big = np.concatenate([np.full(4, 50.0), pts, np.full(2, -9.0)])
    # The counter key includes (b, e), so the draws differ from the node at 0,
    # but the weights depend only on the node's own points.
    for s in range(50):
        i1, i2, w = oc.seeds(big, 4, 7, s)
        assert 4 <= i1 < 7 and 4 <= i2 < 7 and i2 != i1
        if i1 == 4:
            assert list(w) == [0, 2**29, 3 * 2**29]
