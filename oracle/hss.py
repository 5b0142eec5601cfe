"""HSS reference for the Gaussian kernel, dense FP64 (Section 3.1).

An HSS matrix (Section 3.1, Figs. 2-3) on a binary cluster tree stores, per
node in postorder: a dense diagonal block D at each leaf; a basis U at every
node but the root, nested so that a parent's big basis is
diag(U_left, U_right) times its small transfer matrix; and a coupling block
B between the two children of every non-leaf node.  K is symmetric, so the
column bases V equal the row bases U and B_right,left = B_left,right^T.

`nested_id` builds this representation deterministically: each node's basis is
the interpolative decomposition (ID, rows kept as skeletons) of its whole
off-diagonal block row -- for a leaf the rows of K(I, complement), for a parent
the skeleton rows of its children restricted to the parent's complement.  This
is the noise-free form of the randomized construction the paper uses, which
replaces the block row by its product with a random block.  `randomized`
follows that randomized construction step by step on a caller-supplied random
block R (sample S = K R, leaf local sample S - D R, parent local sample
stacked skeleton samples minus B times the sibling's reduced random block).

`assemble` turns any HSS given by its generators (this module's, or one read
back from the GPU) into the dense matrix it represents.

Test infrastructure only (see the package docstring)."""
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .kernel import kernel_dense


@dataclass
class HSS:
    nodes: np.ndarray                      # n_nodes x >=4: begin, end, left, right
    U: dict = field(default_factory=dict)  # node -> m x k basis (leaf) / transfer (parent)
    J: dict = field(default_factory=dict)  # node -> skeleton positions (global, permuted order)
    D: dict = field(default_factory=dict)  # leaf -> dense diagonal block
    B: dict = field(default_factory=dict)  # parent -> B_{left,right}

    @property
    def n(self):
        return int(self.nodes[-1, 1] - self.nodes[-1, 0])

    def ranks(self):
        return {i: u.shape[1] for i, u in self.U.items()}

    def max_rank(self):
        return max([u.shape[1] for u in self.U.values()], default=0)

    def memory_bytes(self):
        """Memory metric of Section 4.2: all D, U, V, B_ij and B_ji blocks, with
        V and B_ji counted as if stored separately (nonsymmetric storage)."""
        tot = sum(d.size for d in self.D.values())
        tot += 2 * sum(u.size for u in self.U.values())
        tot += 2 * sum(b.size for b in self.B.values())
        return 8 * tot


def row_id(A, rtol, atol=0.0):
    """Interpolative decomposition of the rows of A (m x c): A ~= U A[J, :].

    Column-pivoted QR of A^T (LAPACK geqp3 through SciPy); the rank k is the
    number of leading pivots with |R_jj| > max(rtol |R_00|, atol).  Returns
    (piv, k, U) where piv is the pivot order (first k = skeleton rows) and U is
    m x k with U[piv[:k]] = I and U[piv[k:]] = (R11^{-1} R12)^T."""
    A = np.asarray(A, dtype=np.float64)
    m = A.shape[0]
    if m == 0 or A.shape[1] == 0:
        return np.arange(m), 0, np.zeros((m, 0))
    _, R, P = sla.qr(A.T, mode="economic", pivoting=True)
    diag = np.abs(np.diag(R))
    if diag.size == 0 or diag[0] == 0.0:
        return P, 0, np.zeros((m, 0))
    thr = max(rtol * diag[0], atol)
    k = 0
    while k < diag.size and diag[k] > thr:
        k += 1
    T = sla.solve_triangular(R[:k, :k], R[:k, k:], lower=False) if k > 0 else np.zeros((0, m))
    U = np.zeros((m, k))
    U[P[:k], :] = np.eye(k)
    U[P[k:], :] = T.T
    return P, k, U


def _postorder_ok(nodes):
    for i in range(nodes.shape[0]):
        l, r = nodes[i, 2], nodes[i, 3]
        if l >= 0:
            assert l < i and r < i


def nested_id(X, nodes, h, rtol, atol=0.0, K=None):
    """Deterministic HSS of K(X, X; h) on the given tree (X in tree order)."""
    nodes = np.asarray(nodes)
    _postorder_ok(nodes)
    if K is None:
        K = kernel_dense(X, X, h)
    n = K.shape[0]
    H = HSS(nodes=nodes)
    root = nodes.shape[0] - 1
    for i in range(nodes.shape[0]):
        b, e, l, r = (int(v) for v in nodes[i, :4])
        leaf = l < 0
        if leaf:
            H.D[i] = K[b:e, b:e].copy()
            rows = np.arange(b, e)
        else:
            H.B[i] = K[np.ix_(H.J[l], H.J[r])].copy()
            rows = np.concatenate([H.J[l], H.J[r]])
        if i == root:
            break
        comp = np.concatenate([np.arange(0, b), np.arange(e, n)])
        piv, k, U = row_id(K[np.ix_(rows, comp)], rtol, atol)
        H.U[i] = U
        H.J[i] = rows[piv[:k]]
    return H


def randomized(X, nodes, h, rtol, R, atol=0.0, K=None):
    """Randomized HSS construction (Section 3.1) from the sample S = K R.

    Leaf: local sample Y = S(I) - D R(I); ID of Y gives U, J; reduced block
    Omega = U^T R(I).  Parent with children a, b: Y = [Y_a(J_a) - B_ab Omega_b ;
    Y_b(J_b) - B_ab^T Omega_a]; ID of Y gives the transfer U and J; Omega =
    U^T [Omega_a; Omega_b].  B_ab = K(J_a, J_b) and D = K(I, I) are extracted."""
    nodes = np.asarray(nodes)
    _postorder_ok(nodes)
    if K is None:
        K = kernel_dense(X, X, h)
    R = np.asarray(R, dtype=np.float64)
    S = K @ R
    H = HSS(nodes=nodes)
    root = nodes.shape[0] - 1
    Ysk, Om = {}, {}
    for i in range(nodes.shape[0]):
        b, e, l, r = (int(v) for v in nodes[i, :4])
        if l < 0:
            H.D[i] = K[b:e, b:e].copy()
            rows = np.arange(b, e)
            Y = S[b:e] - H.D[i] @ R[b:e]
            Rloc = R[b:e]
        else:
            H.B[i] = K[np.ix_(H.J[l], H.J[r])].copy()
            rows = np.concatenate([H.J[l], H.J[r]])
            Y = np.vstack([Ysk[l] - H.B[i] @ Om[r], Ysk[r] - H.B[i].T @ Om[l]])
            Rloc = np.vstack([Om[l], Om[r]])
        if i == root:
            break
        piv, k, U = row_id(Y, rtol, atol)
        H.U[i] = U
        H.J[i] = rows[piv[:k]]
        Ysk[i] = Y[piv[:k]]
        Om[i] = U.T @ Rloc
    return H


def big_basis(H, i):
    """The full basis of node i: U itself at a leaf, diag(children) @ U above."""
    l, r = int(H.nodes[i, 2]), int(H.nodes[i, 3])
    if l < 0:
        return H.U[i]
    Ul, Ur = big_basis(H, l), big_basis(H, r)
    top = Ul @ H.U[i][: Ul.shape[1]]
    bot = Ur @ H.U[i][Ul.shape[1]:]
    return np.vstack([top, bot])


def assemble(H):
    """Dense matrix represented by the HSS generators."""
    nodes = H.nodes
    root = nodes.shape[0] - 1
    n = int(nodes[root, 1] - nodes[root, 0])
    base = int(nodes[root, 0])
    A = np.zeros((n, n))
    for i in range(nodes.shape[0]):
        b, e, l, r = (int(v) for v in nodes[i, :4])
        if l < 0:
            A[b - base:e - base, b - base:e - base] = H.D[i]
        else:
            bl, el = int(nodes[l, 0]) - base, int(nodes[l, 1]) - base
            br, er = int(nodes[r, 0]) - base, int(nodes[r, 1]) - base
            blk = big_basis(H, l) @ H.B[i] @ big_basis(H, r).T
            A[bl:el, br:er] = blk
            A[br:er, bl:el] = blk.T
    return A


def solve_dense(H, lam, rhs):
    """(K_hss + lambda I)^{-1} rhs by dense Cholesky of the assembled matrix:
    the plain definition an HSS factorization and solve must reproduce."""
    A = assemble(H)
    A[np.diag_indices_from(A)] += lam
    return sla.cho_solve(sla.cho_factor(A, lower=True), np.asarray(rhs, dtype=np.float64))
