"""Pins for the HSS reference (Section 3.1): exact low-rank IDs, exact
reconstruction at zero tolerance, the h -> 0 and h -> infinity limits of the
kernel (Section 1), reconstruction within the tolerance, per-node ID residuals,
the randomized construction against the deterministic one, and the memory
metric of Section 4.2 on a hand-counted example."""
import numpy as np
import pytest

import synthdata as sd
from oracle import cluster as oc
from oracle import hss as oh
from oracle import kernel as ok


def _c1_tree(n=1000, leaf=64, seed=3):
    p = sd.c1_two_gaussians(n=n, m=10)
    t = oc.cluster2mn(p.X, leaf, seed)
    return p, p.X[t.perm].astype(np.float64), t


def test_row_id_exact_low_rank():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((20, 3)) @ rng.standard_normal((3, 30))
    piv, k, U = oh.row_id(A, 1e-10)
    assert k == 3
    J = piv[:k]
    np.testing.assert_allclose(U[J], np.eye(3), atol=0)
    assert np.linalg.norm(A - U @ A[J]) <= 1e-12 * np.linalg.norm(A)


def test_row_id_full_rank_and_empty():
    A = np.diag([3.0, 2.0, 1.0])
    piv, k, U = oh.row_id(A, 0.0)
    assert k == 3 and list(piv) == [0, 1, 2]
    np.testing.assert_array_equal(U, np.eye(3))
    # rtol cuts the trailing pivot 1 < 0.5 * 3
    assert oh.row_id(A, 0.5)[1] == 2
    assert oh.row_id(np.zeros((4, 5)), 0.1)[1] == 0
    assert oh.row_id(np.zeros((0, 5)), 0.1)[1] == 0


def test_zero_tolerance_reconstructs_exactly():
    p, Xp, t = _c1_tree(n=400, leaf=32)
    K = ok.kernel_dense(Xp, Xp, 1.0)
    H = oh.nested_id(Xp, t.nodes, 1.0, 0.0, K=K)
    assert np.linalg.norm(K - oh.assemble(H)) <= 1e-12 * np.linalg.norm(K)


def test_h_to_zero_gives_rank_zero():
    p, Xp, t = _c1_tree(n=300, leaf=20)
    H = oh.nested_id(Xp, t.nodes, 1e-3, 1e-6)
    assert H.max_rank() == 0
    np.testing.assert_array_equal(oh.assemble(H), np.eye(300))


def test_h_to_infinity_rank_at_most_d_plus_2():
    # K = 1 1^T - Dsq / (2 h^2) + O(h^-4); the squared-distance matrix has rank <= d + 2
    p, Xp, t = _c1_tree(n=600, leaf=40)
    H = oh.nested_id(Xp, t.nodes, 100.0, 1e-4)
    assert 1 <= H.max_rank() <= Xp.shape[1] + 2


@pytest.mark.parametrize("rtol", [1e-2, 1e-4, 1e-6])
def test_reconstruction_within_tolerance(rtol):
    p, Xp, t = _c1_tree()
    K = ok.kernel_dense(Xp, Xp, p.h)
    H = oh.nested_id(Xp, t.nodes, p.h, rtol, K=K)
    err = np.linalg.norm(K - oh.assemble(H)) / np.linalg.norm(K)
    assert err <= rtol


def test_per_node_id_residual():
    p, Xp, t = _c1_tree(n=500, leaf=32)
    K = ok.kernel_dense(Xp, Xp, p.h)
    rtol = 1e-4
    H = oh.nested_id(Xp, t.nodes, p.h, rtol, K=K)
    n = Xp.shape[0]
    for i, U in H.U.items():
        b, e, l, r = t.nodes[i, :4]
        rows = np.arange(b, e) if l < 0 else np.concatenate([H.J[l], H.J[r]])
        comp = np.concatenate([np.arange(0, b), np.arange(e, n)])
        A = K[np.ix_(rows, comp)]
        assert set(H.J[i].tolist()) <= set(rows.tolist())
        res = np.linalg.norm(A - U @ K[np.ix_(H.J[i], comp)])
        assert res <= np.sqrt(len(rows)) * rtol * np.linalg.norm(A) + 1e-14


def test_randomized_matches_deterministic_quality():
    # With a finite random block the sampled IDs see the block rows through
    # K(I, I^c) R(I^c); the reconstruction error falls toward the deterministic
    # nested-ID error as the block widens, and with r >= n the sample has the
    # full row space.
    p, Xp, t = _c1_tree(n=800, leaf=48)
    K = ok.kernel_dense(Xp, Xp, p.h)
    rtol = 1e-3
    Hd = oh.nested_id(Xp, t.nodes, p.h, rtol, K=K)
    ed = np.linalg.norm(K - oh.assemble(Hd)) / np.linalg.norm(K)
    errs = []
    for r in (Hd.max_rank() + 40, Hd.max_rank() + 200, 800):
        R = sd.random_block(800, r, seed=2).astype(np.float64)
        Hr = oh.randomized(Xp, t.nodes, p.h, rtol, R, K=K)
        errs.append(np.linalg.norm(K - oh.assemble(Hr)) / np.linalg.norm(K))
        assert Hr.max_rank() <= Hd.max_rank() + 5
    assert errs[0] <= 2 * rtol
    assert errs[0] >= errs[1] >= errs[2]
    assert errs[2] <= 2 * ed


def test_dense_solve_of_exact_hss_equals_krr():
    p, Xp, t = _c1_tree(n=300, leaf=32)
    K = ok.kernel_dense(Xp, Xp, p.h)
    H = oh.nested_id(Xp, t.nodes, p.h, 0.0, K=K)
    y = p.y[t.perm]
    a = oh.solve_dense(H, p.lam, y)
    np.testing.assert_allclose(a, ok.krr_solve_dense(K, y, p.lam), rtol=1e-10, atol=1e-12)


def test_memory_metric_hand_count():
    # 4 points, leaves of 2, the two clusters far apart with h small enough
    # that the off-diagonal block is exactly zero: all ranks 0.
    X = np.array([[0.0], [0.1], [50.0], [50.1]])
    nodes = np.array([[0, 2, -1, -1], [2, 4, -1, -1], [0, 4, 0, 1]])
    H = oh.nested_id(X, nodes, 0.5, 1e-8)
    assert H.ranks() == {0: 0, 1: 0}
    # D blocks 2 x (2 x 2), U blocks 2 x 0, B 0 x 0  ->  8 doubles
    assert H.memory_bytes() == 8 * 8
    # full rank variant (h large): U 2 x 2 twice (counted for U and V),
    # B 2 x 2 (counted for B_ij and B_ji): 8 + 2 * 8 + 2 * 4 = 32 doubles
    H = oh.nested_id(X, nodes, 100.0, 0.0)
    assert H.ranks() == {0: 2, 1: 2}
    assert H.memory_bytes() == 32 * 8
