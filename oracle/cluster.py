"""Recursive two-means (2MN) ordering and cluster tree, and the other
orderings the paper compares it with (NP, KD, PCA).

Section 4.2 (split in two, make each group consecutive, recurse, the ranges are
the HSS tree nodes), Section 4.3 "Recursive two-means" (seeding, Lloyd
iterations until no point changes cluster), leaf-size stopping rule of
Section 4.3, postorder numbering of Fig. 3.  The exact arithmetic is in
oracle/c/oracle.c; this module marshals arrays.

Test infrastructure only (see the package docstring)."""
import ctypes
from dataclasses import dataclass

import numpy as np

from ._clib import lib


@dataclass
class Tree:
    perm: np.ndarray     # perm[new position] = original index
    nodes: np.ndarray    # n_nodes x 5: begin, end, left, right, parent (postorder)
    fallbacks: int
    capped: int
    iterations: int

    @property
    def n_nodes(self):
        return self.nodes.shape[0]

    def is_leaf(self, i):
        return self.nodes[i, 2] < 0

    def leaves(self):
        return [i for i in range(self.n_nodes) if self.nodes[i, 2] < 0]

    @property
    def root(self):
        return self.n_nodes - 1

    def leaf_ranges_per_point(self):
        """Per position i: the [begin, end) of the leaf containing i."""
        n = self.perm.shape[0]
        lb = np.empty(n, dtype=np.int64)
        le = np.empty(n, dtype=np.int64)
        for i in self.leaves():
            b, e = self.nodes[i, 0], self.nodes[i, 1]
            lb[b:e] = b
            le[b:e] = e
        return lb, le


def cluster2mn(X, leaf, seed, max_iter=100):
    """Run the 2MN spec on X (any float dtype, promoted exactly to FP64)."""
    Xd = np.ascontiguousarray(np.asarray(X).astype(np.float64))
    n, d = Xd.shape
    perm = np.empty(n, dtype=np.int64)
    nodes = np.empty((max(2 * n - 1, 1), 5), dtype=np.int64)
    stats = np.zeros(3, dtype=np.int64)
    cnt = lib().oracle_cluster2mn(Xd.ctypes.data_as(ctypes.c_void_p), n, d, int(leaf),
                                  int(max_iter), ctypes.c_uint64(seed & (2**64 - 1)),
                                  perm.ctypes.data_as(ctypes.c_void_p),
                                  nodes.ctypes.data_as(ctypes.c_void_p),
                                  stats.ctypes.data_as(ctypes.c_void_p))
    if cnt < 0:
        raise MemoryError("oracle_cluster2mn: allocation failed")
    return Tree(perm, nodes[:cnt].copy(), int(stats[0]), int(stats[1]), int(stats[2]))


ORDERINGS = {"np": 1, "kd": 2, "pca": 3}


def order(X, leaf, method):
    """The NP, KD or PCA ordering of Section 4.3 ("Selected Preprocessing
    Methods") with its cluster tree; the split rules are spelled out in
    oracle/c/oracle.c.  Tree.fallbacks counts halves splits, Tree.capped the
    KD median splits (Tree.iterations is 0)."""
    Xd = np.ascontiguousarray(np.asarray(X).astype(np.float64))
    n, d = Xd.shape
    perm = np.empty(n, dtype=np.int64)
    nodes = np.empty((max(2 * n - 1, 1), 5), dtype=np.int64)
    stats = np.zeros(2, dtype=np.int64)
    cnt = lib().oracle_order(Xd.ctypes.data_as(ctypes.c_void_p), n, d, int(leaf), ORDERINGS[method],
                             perm.ctypes.data_as(ctypes.c_void_p), nodes.ctypes.data_as(ctypes.c_void_p),
                             stats.ctypes.data_as(ctypes.c_void_p))
    if cnt < 0:
        raise MemoryError("oracle_order: allocation failed")
    return Tree(perm, nodes[:cnt].copy(), int(stats[0]), int(stats[1]), 0)


def seeds(X, b, e, seed):
    """The two seeds (i1, i2) and the integer weights (positions b..e-1) that
    the clustering draws for node [b, e) of X; i2 = -1 means the fallback split
    (all points equal the first seed).  Exposed so tests observe the draw."""
    Xd = np.ascontiguousarray(np.asarray(X).astype(np.float64))
    if Xd.ndim == 1:
        Xd = Xd[:, None]
    n, d = Xd.shape
    out = np.empty(2, dtype=np.int64)
    w = np.zeros(n, dtype=np.uint64)
    rc = lib().oracle_seeds(Xd.ctypes.data_as(ctypes.c_void_p), n, d, int(b), int(e),
                            ctypes.c_uint64(seed & (2**64 - 1)),
                            out.ctypes.data_as(ctypes.c_void_p),
                            w.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise ValueError(f"oracle_seeds: invalid node [{b}, {e}) or allocation failure ({rc})")
    return int(out[0]), int(out[1]), w[b:e].copy()


def node_draw(seed, b, e, k):
    """The counter-based draw the 2MN seeding uses (exposed for tests)."""
    return int(lib().oracle_node_draw(seed & (2**64 - 1), b, e, k))


def isqrt64(v):
    return int(lib().oracle_isqrt64(v))


def sm_step(x):
    """One SplitMix64 output for state x (state advanced by the golden gamma)."""
    return int(lib().oracle_sm_step(x & (2**64 - 1)))
