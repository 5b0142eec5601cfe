"""Python binding of libkrr, the MI355X (gfx950) Gaussian-kernel ridge
regression library (include/krr.h).

This module only marshals arguments: torch tensors provide device memory and
the current stream; every computation runs in the library's HIP kernels.
There is no CPU fallback -- if libkrr.so is missing, every call raises.

Order convention: after clustering, points, labels, samples and solutions are
in the permuted ("tree") order; perm[i] is the original index of position i.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from ._lib import (KRR_BF16_SPLIT, KRR_F16_SPLIT, KRR_F32, KRR_F64, ClusterOpts, HssOpts, HssStats,  # noqa: F401
                   KrrError, RefineStats, check)
from ._lib import LIB_PATH
from ._lib import load as _load_lib

# ------------------------------------------------------------ device memory

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
# every callback pair ever registered stays referenced: the library returns a
# buffer to the allocator that made it, also after another one is registered
_allocators = []
_alloc_live = [True]


def _torch_alloc(size, stream, ctx):
    try:
        return torch.cuda.caching_allocator_alloc(int(size), stream=int(stream or 0))
    except Exception:  # out of memory: the library reports KRR_E_NOMEM
        return None


def _torch_free(ptr, stream, ctx):
    if _alloc_live[0] and ptr:
        torch.cuda.caching_allocator_delete(int(ptr))


def _at_exit():
    # buffers still held at interpreter exit are left to the process's end
    _alloc_live[0] = False


import atexit  # noqa: E402

atexit.register(_at_exit)


def set_allocator(alloc=None, free=None):
    """Register device-memory callbacks for every library buffer:
    alloc(size, stream) -> int device pointer (0 / None on failure),
    free(ptr, stream).  No arguments: torch's caching allocator.  Returns
    the registered pair."""
    if alloc is None and free is None:
        alloc, free = _torch_alloc, _torch_free
    else:
        a_, f_ = alloc, free
        alloc = lambda size, stream, ctx: a_(size, stream)  # noqa: E731
        free = lambda ptr, stream, ctx: f_(ptr, stream)  # noqa: E731
    pair = (ALLOC_FN(alloc), FREE_FN(free))
    _allocators.append(pair)
    check(_load_lib().krr_set_allocator(ctypes.cast(pair[0], ctypes.c_void_p),
                                        ctypes.cast(pair[1], ctypes.c_void_p), None))
    return pair


def use_hip_malloc():
    """New library buffers from hipMalloc / hipFree again."""
    check(_load_lib().krr_set_allocator(None, None, None))


def alloc_counts():
    """(direct hipMalloc allocations, allocations through the registered allocator) so far."""
    d, c = ctypes.c_int64(), ctypes.c_int64()
    check(_load_lib().krr_alloc_counts(ctypes.byref(d), ctypes.byref(c)))
    return d.value, c.value


def load(path: str = LIB_PATH):
    """Load libkrr.so (raises if it is missing); on the first load with a GPU
    present, torch's caching allocator becomes the library's allocator, so
    torch owns all device memory."""
    first = _lib._lib is None
    lib = _load_lib(path)
    if first and torch.cuda.is_available():
        set_allocator()
    return lib

PREC = {"f64": KRR_F64, "f32": KRR_F32, "f16": KRR_F16_SPLIT, "bf16": KRR_BF16_SPLIT}


def _prec(p):
    return PREC[p] if isinstance(p, str) else int(p)


def _xprec(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return KRR_F64
    if t.dtype == torch.float32:
        return KRR_F32
    raise TypeError(f"points must be float32 or float64, got {t.dtype}")


def _dev(t: torch.Tensor, dtype=None) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def device_count() -> int:
    return load().krr_device_count()


# ------------------------------------------------------------------ trees

class Tree:
    """Cluster tree handle (postorder nodes: begin, end, left, right, parent)."""

    def __init__(self, handle):
        self.h = handle
        n, nn = ctypes.c_int64(), ctypes.c_int64()
        check(load().krr_tree_size(handle, ctypes.byref(n), ctypes.byref(nn)))
        self.n, self.n_nodes = n.value, nn.value
        self.nodes = np.empty((self.n_nodes, 5), dtype=np.int64)
        self.stats = np.zeros(4, dtype=np.int64)
        check(load().krr_tree_export(handle, self.nodes.ctypes.data_as(ctypes.c_void_p),
                                     self.stats.ctypes.data_as(ctypes.c_void_p)))
        cnt = ctypes.c_int32()
        check(load().krr_tree_roots(handle, None, ctypes.byref(cnt)))
        self.roots = np.empty(cnt.value, dtype=np.int64)
        check(load().krr_tree_roots(handle, self.roots.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    ctypes.byref(cnt)))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None and _lib._lib is not None:
            _lib._lib.krr_tree_destroy(self.h)
            self.h = None


def cluster_2mn(X: torch.Tensor, leaf: int, seed: int, max_iter: int = 100):
    """Recursive two-means ordering; returns (perm int64 tensor, Tree)."""
    _dev(X)
    n, d = X.shape
    perm = torch.empty(n, dtype=torch.int64, device=X.device)
    opts = ClusterOpts(int(leaf), int(max_iter), int(seed) & (2**64 - 1))
    h = ctypes.c_void_p()
    check(load().krr_cluster_2mn(_p(X), _xprec(X), n, d, ctypes.byref(opts), _stream(), _p(perm),
                                 ctypes.byref(h)))
    return perm, Tree(h)


ORDERINGS = {"2mn": 0, "np": 1, "kd": 2, "pca": 3}


def cluster_order(X: torch.Tensor, leaf: int, method: str, offsets=None, seed: int = 7, max_iter: int = 100):
    """Ordering and cluster tree by "2mn", "np", "kd" or "pca" (a forest when
    offsets, np + 1 host ints, is given); returns (perm int64 tensor, Tree)."""
    _dev(X)
    n, d = X.shape
    perm = torch.empty(n, dtype=torch.int64, device=X.device)
    opts = ClusterOpts(int(leaf), int(max_iter), int(seed) & (2**64 - 1))
    h = ctypes.c_void_p()
    if offsets is None:
        offp, npb = None, 0
    else:
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        offp, npb = _i64p(off), len(off) - 1
    check(load().krr_cluster_order(_p(X), _xprec(X), n, d, ORDERINGS[method], offp, npb, ctypes.byref(opts),
                                   _stream(), _p(perm), ctypes.byref(h)))
    return perm, Tree(h)


def tree_from_nodes(nodes) -> Tree:
    arr = np.ascontiguousarray(np.asarray(nodes, dtype=np.int64)[:, :5])
    h = ctypes.c_void_p()
    check(load().krr_tree_from_host(arr.ctypes.data_as(ctypes.c_void_p), arr.shape[0], ctypes.byref(h)))
    return Tree(h)


def gather_rows(src: torch.Tensor, perm: torch.Tensor) -> torch.Tensor:
    """dst[i] = src[perm[i]]."""
    _dev(src)
    _dev(perm, torch.int64)
    s2 = src.reshape(src.shape[0], -1)
    dst = torch.empty_like(s2)
    check(load().krr_gather_rows(_p(s2), _xprec(s2), s2.shape[0], s2.shape[1], _p(perm), _p(dst), _stream()))
    return dst.reshape(src.shape)


def scatter_rows(src: torch.Tensor, perm: torch.Tensor) -> torch.Tensor:
    """dst[perm[i]] = src[i]."""
    _dev(src)
    _dev(perm, torch.int64)
    s2 = src.reshape(src.shape[0], -1)
    dst = torch.empty_like(s2)
    check(load().krr_scatter_rows(_p(s2), _xprec(s2), s2.shape[0], s2.shape[1], _p(perm), _p(dst), _stream()))
    return dst.reshape(src.shape)


# -------------------------------------------------------------- products

def kernel_matvec(X, Y, h, W, beta=0.0, out=None, prec="f32"):
    """out = K(X, Y; h) W + beta out  (W, out float64)."""
    _dev(X)
    _dev(Y)
    _dev(W, torch.float64)
    W2 = W.reshape(W.shape[0], -1)
    m, n = X.shape[0], Y.shape[0]
    if out is None:
        out = torch.empty((m, W2.shape[1]), dtype=torch.float64, device=X.device)
    _dev(out, torch.float64)
    check(load().kernel_matvec(_p(X), m, _p(Y), n, X.shape[1], _xprec(X), float(h), _p(W2), W2.shape[1],
                               float(beta), _p(out), _prec(prec), _stream()))
    return out.reshape((m,) + tuple(W.shape[1:]))


class TileMap:
    """Negligible-tile map of the symmetric FP32 product K(X, X) W, kept
    across products with the same points and width: the first product records
    which tiles hold an entry of at least 2^-32, later ones evaluate only
    those (krr_tile_map_*).  Make a new map when X changes in place."""

    def __init__(self):
        h = ctypes.c_void_p()
        check(load().krr_tile_map_create(ctypes.byref(h)))
        self.h = h

    def matvec(self, X, h, W, beta=0.0, out=None):
        """out = K(X, X; h) W + beta out through the map (FP32 entries)."""
        _dev(X)
        _dev(W, torch.float64)
        W2 = W.reshape(W.shape[0], -1)
        n = X.shape[0]
        if out is None:
            out = torch.empty((n, W2.shape[1]), dtype=torch.float64, device=X.device)
        _dev(out, torch.float64)
        check(load().kernel_matvec_mapped(_p(X), n, X.shape[1], _xprec(X), float(h), _p(W2), W2.shape[1],
                                          float(beta), _p(out), self.h, _stream()))
        return out.reshape((n,) + tuple(W.shape[1:]))

    def counts(self):
        """(tiles marked for evaluation, tiles covered, kernel entries per tile)."""
        c = (ctypes.c_int64 * 3)()
        check(load().krr_tile_map_counts(self.h, c, _stream()))
        return int(c[0]), int(c[1]), int(c[2])

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None and _lib._lib is not None:
            _lib._lib.krr_tile_map_destroy(self.h)
            self.h = None


def kernel_sample(X, h, R, leaf_begin=None, leaf_end=None, prec="f32", split_terms=2):
    """Off-diagonal sample S = K(X, X; h) R with each row's own leaf removed."""
    _dev(X)
    _dev(R, torch.float32)
    n, r = R.shape
    p = _prec(prec)
    S = torch.empty((n, r), dtype=torch.float64 if p == KRR_F64 else torch.float32, device=X.device)
    check(load().kernel_sample(_p(X), n, X.shape[1], _xprec(X), float(h), _p(R), r,
                               _p(leaf_begin) if leaf_begin is not None else None,
                               _p(leaf_end) if leaf_end is not None else None, _p(S), p, int(split_terms),
                               _stream()))
    return S


def random_block(seed, n, r, c0=0, device="cuda"):
    R = torch.empty((n, r), dtype=torch.float32, device=device)
    check(load().krr_random_block(int(seed) & (2**64 - 1), n, r, c0, _p(R), _stream()))
    return R


def kernel_matvec_bwd(X, Y, h, W, G, prec="f32", want=("dX", "dY", "dW", "dh")):
    """Backward of Out = K(X, Y; h) W: returns dict with the requested grads."""
    _dev(X)
    _dev(Y)
    W2 = _dev(W, torch.float64).reshape(W.shape[0], -1)
    G2 = _dev(G, torch.float64).reshape(G.shape[0], -1)
    m, n, d = X.shape[0], Y.shape[0], X.shape[1]
    dev = X.device
    out = {}
    out["dX"] = torch.empty((m, d), dtype=torch.float64, device=dev) if "dX" in want else None
    out["dY"] = torch.empty((n, d), dtype=torch.float64, device=dev) if "dY" in want else None
    out["dW"] = torch.empty((n, W2.shape[1]), dtype=torch.float64, device=dev) if "dW" in want else None
    out["dh"] = torch.empty(1, dtype=torch.float64, device=dev) if "dh" in want else None
    check(load().kernel_matvec_bwd(_p(X), m, _p(Y), n, d, _xprec(X), float(h), _p(W2), _p(G2), W2.shape[1],
                                   _p(out["dX"]), _p(out["dY"]), _p(out["dW"]), _p(out["dh"]), _prec(prec),
                                   _stream()))
    if out["dW"] is not None:
        out["dW"] = out["dW"].reshape(W.shape)
    return {k: v for k, v in out.items() if v is not None}


TUNE = {"symmetric": _lib.KRR_TUNE_SYMMETRIC, "sample_rb": _lib.KRR_TUNE_SAMPLE_RB,
        "mv_blocks": _lib.KRR_TUNE_MV_BLOCKS, "sym_chunk": _lib.KRR_TUNE_SYM_CHUNK,
        "sample_skip": _lib.KRR_TUNE_SAMPLE_SKIP, "sym_skip": _lib.KRR_TUNE_SYM_SKIP}


def set_tuning(knob: str, value: int):
    """Set a launch-shape knob of the hot kernels (process-wide)."""
    check(load().krr_set_tuning(TUNE[knob], int(value)))


def get_tuning(knob: str) -> int:
    v = ctypes.c_int32()
    check(load().krr_get_tuning(TUNE[knob], ctypes.byref(v)))
    return v.value


def dot_columns(a, b):
    a2 = _dev(a, torch.float64).reshape(a.shape[0], -1)
    b2 = _dev(b, torch.float64).reshape(b.shape[0], -1)
    out = torch.empty(a2.shape[1], dtype=torch.float64, device=a.device)
    check(load().krr_dot_columns(_p(a2), _p(b2), a2.shape[0], a2.shape[1], _p(out), _stream()))
    return out


def val_residual(f, yv):
    """(ge, loss): ge = (2 / m)(f - y_v) and loss = |f - y_v|^2 / m per column
    (FP64 device tensors, libkrr kernel)."""
    f2 = _dev(f, torch.float64).reshape(f.shape[0], -1)
    y2 = _dev(yv, torch.float64).reshape(yv.shape[0], -1)
    if f2.shape != y2.shape:
        raise ValueError("scores and targets differ in shape")
    ge = torch.empty_like(f2)
    loss = torch.empty(f2.shape[1], dtype=torch.float64, device=f2.device)
    check(load().krr_val_residual(_p(f2), _p(y2), f2.shape[0], f2.shape[1], _p(ge), _p(loss), _stream()))
    return ge, loss


def val_grad_finish(bta, dh_v, dh_t, h, lam, gscale=None):
    """Device tensor (2,): gscale (h (dh_v - dh_t), -lambda bta) from device scalars."""
    args = [_dev(t, torch.float64).reshape(1) for t in (bta, dh_v, dh_t)]
    g = None if gscale is None else _dev(gscale, torch.float64).reshape(1)
    out = torch.empty(2, dtype=torch.float64, device=args[0].device)
    check(load().krr_val_grad_finish(_p(args[0]), _p(args[1]), _p(args[2]), None if g is None else _p(g),
                                     float(h), float(lam), _p(out), _stream()))
    return out


# ------------------------------------------------------------ HSS + ULV

@dataclass
class HssOptions:
    rtol: float = 1e-2
    atol: float = 0.0
    r0: int = 256
    dr: int = 256
    r_max: int = 4096
    oversample: int = 10
    prec: str = "f32"
    split_terms: int = 2
    cap_policy: int = 0
    seed: int = 1

    def c(self):
        return HssOpts(self.rtol, self.atol, self.r0, self.dr, self.r_max, self.oversample, _prec(self.prec),
                       self.split_terms, self.cap_policy, self.seed & (2**64 - 1))


class HSS:
    """Compressed HSS generators of K(Xp, Xp; h) (device resident)."""

    def __init__(self, tree: Tree, Xp: torch.Tensor, h: float, opts: HssOptions = HssOptions()):
        _dev(Xp)
        self.tree = tree
        self.stats = HssStats()
        h_ = ctypes.c_void_p()
        check(load().hss_compress(tree.h, _p(Xp), _xprec(Xp), Xp.shape[1], float(h), ctypes.byref(opts.c()),
                                  _stream(), ctypes.byref(h_), ctypes.byref(self.stats)))
        self.h = h_

    def matvec(self, x: torch.Tensor) -> torch.Tensor:
        """K_hss x (permuted order, FP64)."""
        x2 = _dev(x, torch.float64).reshape(x.shape[0], -1)
        y = torch.empty_like(x2)
        check(load().hss_matvec(self.h, _p(x2), x2.shape[1], _p(y), _stream()))
        return y.reshape(x.shape)

    def export(self):
        """Generators on the host: dict with nodes (n x 10 table), U, D, B, J per node."""
        nn, nd, ni = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(load().hss_export_sizes(self.h, ctypes.byref(nn), ctypes.byref(nd), ctypes.byref(ni)))
        table = np.empty((nn.value, 10), dtype=np.int64)
        dbl = np.empty(max(nd.value, 1), dtype=np.float64)
        ints = np.empty(max(ni.value, 1), dtype=np.int64)
        check(load().hss_export(self.h, table.ctypes.data_as(ctypes.c_void_p), dbl.ctypes.data_as(ctypes.c_void_p),
                                ints.ctypes.data_as(ctypes.c_void_p), _stream()))
        U, D, B, J = {}, {}, {}, {}
        for i, (b, e, l, r, m, k, oU, oD, oB, oJ) in enumerate(table):
            if oU >= 0:
                U[i] = dbl[oU:oU + m * k].reshape(m, k).copy()
                J[i] = ints[oJ:oJ + k].copy()
            if oD >= 0:
                D[i] = dbl[oD:oD + (e - b) ** 2].reshape(e - b, e - b).copy()
            if oB >= 0:
                kl, kr = table[l, 5], table[r, 5]
                B[i] = dbl[oB:oB + kl * kr].reshape(kl, kr).copy()
        return {"nodes": table, "U": U, "D": D, "B": B, "J": J}

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None and _lib._lib is not None:
            _lib._lib.hss_destroy(self.h)
            self.h = None


class ULV:
    """ULV factor of K_hss + lambda I.  With pivot_floor > 0 (preconditioner
    use), Cholesky pivots below the floor are raised to it so that the factor
    is always positive definite; `clamped` counts them."""

    def __init__(self, H: HSS, lam: float, pivot_floor: float = 0.0, shifted: bool = False):
        h_ = ctypes.c_void_p()
        self.clamped = 0
        self.shift = 0.0
        if shifted:
            sh = ctypes.c_double()
            check(load().hss_ulv_factor_shifted(H.h, float(lam), _stream(), ctypes.byref(h_), ctypes.byref(sh)))
            self.shift = sh.value
        elif pivot_floor > 0:
            cl = ctypes.c_int64()
            check(load().hss_ulv_factor_spd(H.h, float(lam), float(pivot_floor), _stream(), ctypes.byref(h_),
                                            ctypes.byref(cl)))
            self.clamped = cl.value
        else:
            check(load().hss_ulv_factor(H.h, float(lam), _stream(), ctypes.byref(h_)))
        self.h = h_
        self.hss = H
        self.lam = lam

    def use_graph(self, enable: bool = True):
        """Replay solves as a captured HIP graph (default) or issue them directly."""
        check(load().hss_ulv_use_graph(self.h, int(bool(enable))))
        return self

    def solve(self, B: torch.Tensor, out=None) -> torch.Tensor:
        _dev(B, torch.float64)
        B2 = B.reshape(B.shape[0], -1)
        if out is None:
            out = torch.empty_like(B2)
        check(load().hss_solve(self.h, _p(B2), B2.shape[1], _p(out), _stream()))
        return out.reshape(B.shape)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None and _lib._lib is not None:
            _lib._lib.hss_ulv_destroy(self.h)
            self.h = None


def refine(F, Xp, h, lam, Y, alpha, tol=1e-6, max_iter=100, mv_prec="f32", raise_on_fail=True, res_prec=None):
    """PCG on (K + lam I) alpha = Y preconditioned by the ULV factor F (None:
    plain CG); alpha is updated in place.  res_prec: precision of the true
    residual (default mv_prec; "f64" with mv_prec "f32" is mixed-precision
    iterative refinement)."""
    _dev(Xp)
    Y2 = _dev(Y, torch.float64).reshape(Y.shape[0], -1)
    a2 = _dev(alpha, torch.float64).reshape(alpha.shape[0], -1)
    st = RefineStats()
    rc = load().krr_refine(F.h if F is not None else None, _p(Xp), Xp.shape[0], _xprec(Xp), Xp.shape[1], float(h),
                           float(lam), _p(Y2), Y2.shape[1],
                           _p(a2), float(tol), int(max_iter), _prec(mv_prec), _prec(res_prec or mv_prec), _stream(),
                           ctypes.byref(st))
    if rc != 0 and (raise_on_fail or rc != _lib.KRR_E_NOT_CONVERGED):
        check(rc)
    return {"iterations": st.iterations, "matvecs": st.matvecs, "relres": list(st.relres[:Y2.shape[1]]),
            "t_ms": st.t_ms, "converged": rc == 0}


def predict(Xt, Xp, h, alpha, prec="f32"):
    """(scores, labels): sign for one column, argmax for several."""
    _dev(Xt)
    _dev(Xp)
    a2 = _dev(alpha, torch.float64).reshape(alpha.shape[0], -1)
    m = Xt.shape[0]
    scores = torch.empty((m, a2.shape[1]), dtype=torch.float64, device=Xt.device)
    labels = torch.empty(m, dtype=torch.int32, device=Xt.device)
    check(load().krr_predict(_p(Xt), m, _p(Xp), Xp.shape[0], Xp.shape[1], _xprec(Xt), float(h), _p(a2), a2.shape[1],
                             _p(scores), _p(labels), _prec(prec), _stream()))
    return scores, labels


def predict_noalloc(Xt, Xp, h, alpha, scores, labels=None, prec="f32"):
    """predict into caller tensors with no device allocation by the library
    (krr_predict_noalloc; d <= 64, sizes within its static scratch)."""
    _dev(Xt)
    _dev(Xp)
    a2 = _dev(alpha, torch.float64).reshape(alpha.shape[0], -1)
    _dev(scores, torch.float64)
    if labels is not None:
        _dev(labels, torch.int32)
    check(load().krr_predict_noalloc(_p(Xt), Xt.shape[0], _p(Xp), Xp.shape[0], Xp.shape[1], _xprec(Xt), float(h),
                                     _p(a2), a2.shape[1], _p(scores), _p(labels), _prec(prec), _stream()))
    return scores, labels


# ------------------------------------------------------------------ fit

@dataclass
class FitResult:
    alpha: torch.Tensor        # solution in the original order (n x nrhs or n)
    alpha_perm: torch.Tensor   # solution in tree order
    perm: torch.Tensor
    Xp: torch.Tensor
    tree: Tree
    hss: HSS
    ulv: ULV
    info: dict = field(default_factory=dict)


def fit(X, y, h, lam, leaf=128, opts: HssOptions = HssOptions(), seed=7, tol=1e-6, max_iter=200,
        mv_prec="f32", refine_solution=True, raise_on_fail=True, tune_cache=None, res_prec=None):
    """Algorithm 1 steps 0-2: cluster, compress, factor, solve, refine.

    info["phases"] holds the wall time of each library call (seconds, the
    stream synchronized in between).  tune_cache: an autotuner cache whose
    entry for this shape sets the launch knobs first (see tune.py)."""
    import time

    _dev(X)
    if tune_cache is not None:
        from .tune import apply
        apply(X.shape[1], opts.r0, opts.prec, path=tune_cache)
    y2 = _dev(y, torch.float64).reshape(y.shape[0], -1)
    ph = {}

    def mark(name, t0):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ph[name] = t1 - t0
        return t1

    t = time.perf_counter()
    perm, tree = cluster_2mn(X, leaf, seed)
    t = mark("cluster", t)
    Xp = gather_rows(X, perm)
    yp = gather_rows(y2, perm)
    t = mark("permute", t)
    H = HSS(tree, Xp, h, opts)
    t = mark("compress", t)
    # as a preconditioner the factor only has to be positive definite: shift if needed
    F = ULV(H, lam, shifted=refine_solution)
    t = mark("factor", t)
    ap = F.solve(yp)
    t = mark("solve", t)
    info = {"hss": H.stats.as_dict(), "tree_stats": tree.stats.tolist(), "ulv_shift": F.shift}
    if refine_solution:
        info["refine"] = refine(F, Xp, h, lam, yp, ap, tol=tol, max_iter=max_iter, mv_prec=mv_prec,
                                raise_on_fail=raise_on_fail, res_prec=res_prec)
        t = mark("refine", t)
    alpha = scatter_rows(ap, perm)
    if y.dim() == 1:
        alpha = alpha.reshape(-1)
    mark("unpermute", t)
    info["phases"] = ph
    return FitResult(alpha, ap, perm, Xp, tree, H, F, info)


# ------------------------------------------------------------ batched form

def _i64p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _dblp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def offsets_of(sizes) -> np.ndarray:
    """Problem offsets (np + 1 int64, from 0) of consecutive problems."""
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(np.asarray(sizes, dtype=np.int64))
    return off


def cluster_2mn_batched(X: torch.Tensor, offsets, leaf: int, seed: int, max_iter: int = 100):
    """2MN ordering of every problem of a batch; returns (perm, forest Tree)."""
    _dev(X)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    n, d = X.shape
    if off[-1] != n:
        raise ValueError("offsets must end at the number of points")
    perm = torch.empty(n, dtype=torch.int64, device=X.device)
    opts = ClusterOpts(int(leaf), int(max_iter), int(seed) & (2**64 - 1))
    h = ctypes.c_void_p()
    check(load().krr_cluster_2mn_batched(_p(X), _xprec(X), _i64p(off), len(off) - 1, d, ctypes.byref(opts),
                                         _stream(), _p(perm), ctypes.byref(h)))
    return perm, Tree(h)


class BatchedHSS(HSS):
    """HSS generators of every problem of a forest (problem k: tree k, width h[k])."""

    def __init__(self, tree: Tree, Xp: torch.Tensor, h, opts: HssOptions = HssOptions()):
        _dev(Xp)
        hs = np.ascontiguousarray(h, dtype=np.float64)
        if hs.shape != (len(tree.roots),):
            raise ValueError("one kernel width per tree is required")
        self.tree = tree
        self.stats = HssStats()
        h_ = ctypes.c_void_p()
        check(load().hss_compress_batched(tree.h, _p(Xp), _xprec(Xp), Xp.shape[1], _dblp(hs), ctypes.byref(opts.c()),
                                          _stream(), ctypes.byref(h_), ctypes.byref(self.stats)))
        self.h = h_
        self.hprob = hs


class BatchedULV(ULV):
    """ULV factor of every problem of a BatchedHSS with its own lambda."""

    def __init__(self, H: BatchedHSS, lam, shifted: bool = False):
        lams = np.ascontiguousarray(lam, dtype=np.float64)
        h_ = ctypes.c_void_p()
        mult = np.zeros(lams.shape[0], dtype=np.float64)
        check(load().hss_ulv_factor_batched(H.h, _dblp(lams), int(bool(shifted)), _stream(), ctypes.byref(h_),
                                            _dblp(mult)))
        self.h = h_
        self.hss = H
        self.lam = lams
        self.clamped = 0
        self.shift_mults = mult            # each problem's s_k (shift lambda_k s_k)
        self.shift_mult = float(mult.max()) if mult.size else 0.0
        self.shift = self.shift_mult


def kernel_matvec_batched(X, offsets, h, W, prec="f32"):
    """Block-diagonal product: problem k's rows get K(X_k, X_k; h[k]) W_k."""
    _dev(X)
    W2 = _dev(W, torch.float64).reshape(W.shape[0], -1)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    hs = np.ascontiguousarray(h, dtype=np.float64)
    out = torch.empty_like(W2)
    check(load().kernel_matvec_batched(_p(X), _xprec(X), _i64p(off), len(off) - 1, X.shape[1], _dblp(hs), _p(W2),
                                       W2.shape[1], _p(out), _prec(prec), _stream()))
    return out.reshape(W.shape)


def kernel_sample_batched(X, offsets, h, R, leaf_begin=None, leaf_end=None, prec="f32", split_terms=2):
    """Off-diagonal sample of every problem of a batch (one launch)."""
    _dev(X)
    _dev(R, torch.float32)
    n, r = R.shape
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    hs = np.ascontiguousarray(h, dtype=np.float64)
    p = _prec(prec)
    S = torch.empty((n, r), dtype=torch.float64 if p == KRR_F64 else torch.float32, device=X.device)
    check(load().kernel_sample_batched(_p(X), _xprec(X), _i64p(off), len(off) - 1, X.shape[1], _dblp(hs), _p(R), r,
                                       _p(leaf_begin) if leaf_begin is not None else None,
                                       _p(leaf_end) if leaf_end is not None else None, _p(S), p, int(split_terms),
                                       _stream()))
    return S


def refine_batched(F, Xp, offsets, h, lam, Y, alpha, tol=1e-6, max_iter=100, mv_prec="f32", raise_on_fail=True,
                   res_prec=None):
    """PCG on every problem at once (alpha updated in place); returns stats
    with each problem's final relative residuals."""
    _dev(Xp)
    Y2 = _dev(Y, torch.float64).reshape(Y.shape[0], -1)
    a2 = _dev(alpha, torch.float64).reshape(alpha.shape[0], -1)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    hs = np.ascontiguousarray(h, dtype=np.float64)
    ls = np.ascontiguousarray(lam, dtype=np.float64)
    npb = len(off) - 1
    rel = np.zeros(npb * Y2.shape[1], dtype=np.float64)
    st = RefineStats()
    rc = load().krr_refine_batched(F.h if F is not None else None, _p(Xp), _xprec(Xp), _i64p(off), npb, Xp.shape[1],
                                   _dblp(hs), _dblp(ls), _p(Y2), Y2.shape[1], _p(a2), float(tol), int(max_iter),
                                   _prec(mv_prec), _prec(res_prec or mv_prec), _stream(), ctypes.byref(st),
                                   _dblp(rel))
    if rc != 0 and (raise_on_fail or rc != _lib.KRR_E_NOT_CONVERGED):
        check(rc)
    return {"iterations": st.iterations, "matvecs": st.matvecs, "relres": rel.reshape(npb, Y2.shape[1]),
            "t_ms": st.t_ms, "converged": rc == 0}


@dataclass
class BatchedFitResult:
    alphas: list               # per problem, original order within the problem
    groups: list               # per group of equal d: dict with perm, Xp, tree, hss, ulv, offsets, members
    info: dict = field(default_factory=dict)


def fit_batched(problems, leaf=128, opts: HssOptions = HssOptions(), seed=7, tol=1e-6, max_iter=200,
                mv_prec="f32", refine_solution=True, raise_on_fail=True, concurrent=True):
    """Algorithm 1 steps 0-2 for many independent problems at once.

    problems: sequence of (X_k, y_k, h_k, lam_k) with X_k an n_k x d_k GPU
    tensor.  Problems of equal d (and dtype) form one batch: they are stored
    one after the other and every library call covers all of them (one launch
    per phase and tree level).  With several such groups and `concurrent`,
    each group runs in a host thread of its own on a stream of its own, so
    that one group's kernels fill the gaps of another's host decisions; the
    phase times are then summed over the groups.  Returns each problem's
    alpha in its own order."""
    import threading
    import time

    groups = {}
    for idx, (X, y, h, lam) in enumerate(problems):
        _dev(X)
        groups.setdefault((X.shape[1], X.dtype), []).append(idx)
    keys = list(groups.items())
    alphas = [None] * len(problems)
    results = [None] * len(keys)
    errors = [None] * len(keys)
    caller = torch.cuda.current_stream()

    def run_group(gi, members):
        ph = {}

        def mark(name, t0):
            torch.cuda.current_stream().synchronize()
            t1 = time.perf_counter()
            ph[name] = ph.get(name, 0.0) + (t1 - t0)
            return t1

        t = time.perf_counter()
        Xs = [problems[i][0] for i in members]
        ys = [_dev(problems[i][1], torch.float64).reshape(problems[i][1].shape[0], -1) for i in members]
        if len({y.shape[1] for y in ys}) != 1:
            raise ValueError("problems of one batch need the same number of right-hand sides")
        hs = np.array([problems[i][2] for i in members], dtype=np.float64)
        ls = np.array([problems[i][3] for i in members], dtype=np.float64)
        off = offsets_of([x.shape[0] for x in Xs])
        X = torch.cat(Xs, 0).contiguous()
        Y = torch.cat(ys, 0).contiguous()
        t = mark("concat", t)
        perm, tree = cluster_2mn_batched(X, off, leaf, seed)
        t = mark("cluster", t)
        Xp = gather_rows(X, perm)
        Yp = gather_rows(Y, perm)
        t = mark("permute", t)
        H = BatchedHSS(tree, Xp, hs, opts)
        t = mark("compress", t)
        F = BatchedULV(H, ls, shifted=refine_solution)
        t = mark("factor", t)
        ap = F.solve(Yp)
        t = mark("solve", t)
        ref = None
        if refine_solution:
            ref = refine_batched(F, Xp, off, hs, ls, Yp, ap, tol=tol, max_iter=max_iter, mv_prec=mv_prec,
                                 raise_on_fail=raise_on_fail)
            t = mark("refine", t)
        alpha = scatter_rows(ap, perm)
        mark("unpermute", t)
        results[gi] = {"members": members, "offsets": off, "perm": perm, "Xp": Xp, "tree": tree, "hss": H,
                       "ulv": F, "h": hs, "lam": ls, "alpha_perm": ap, "alpha": alpha, "refine": ref,
                       "phases": ph}

    def run_on_stream(gi, members, stream):
        try:
            with torch.cuda.stream(stream):
                run_group(gi, members)
        except BaseException as e:  # re-raised by the caller's thread
            errors[gi] = e

    t_all = time.perf_counter()
    if concurrent and len(keys) > 1:
        caller.synchronize()  # the inputs are ready before other streams read them
        streams = [torch.cuda.Stream() for _ in keys]
        threads = [threading.Thread(target=run_on_stream, args=(gi, members, streams[gi]))
                   for gi, (_, members) in enumerate(keys)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        for st in streams:
            st.synchronize()
        for e in errors:
            if e is not None:
                raise e
        # the results are used on the caller's stream from here on
        for r in results:
            for name in ("perm", "Xp", "alpha_perm", "alpha"):
                r[name].record_stream(caller)
    else:
        for gi, (_, members) in enumerate(keys):
            run_group(gi, members)
    wall = time.perf_counter() - t_all
    out_groups, ph = [], {}
    info = {"refine": [], "hss": [], "ulv_shift_mult": []}
    for r in results:
        alpha, off = r.pop("alpha"), r["offsets"]
        for j, i in enumerate(r["members"]):
            a = alpha[off[j]:off[j + 1]]
            alphas[i] = a.reshape(-1) if problems[i][1].dim() == 1 else a
        for k, v in r.pop("phases").items():
            ph[k] = ph.get(k, 0.0) + v
        info["hss"].append(r["hss"].stats.as_dict())
        info["ulv_shift_mult"].append(r["ulv"].shift_mults.tolist())
        ref = r.pop("refine")
        if ref is not None:
            info["refine"].append(ref)
        out_groups.append(r)
    info["phases"] = ph
    info["wall_s"] = wall
    info["concurrent_groups"] = bool(concurrent and len(keys) > 1)
    return BatchedFitResult(alphas, out_groups, info)
