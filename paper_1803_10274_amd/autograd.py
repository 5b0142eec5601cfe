"""Differentiation of the kernel ridge regression fit (torch.autograd).

KernelMatvec: Out = K(X, Y; h) W with the hand-written backward of libkrr
(dX, dY, dW, dh formed on the fly, K never stored).

ValidationLoss: L(log h, log lambda) = |K(Xv, X) alpha - yv|^2 / m_v with
alpha = (K + lambda I)^{-1} y solved by the HSS path (compression, ULV factor
as preconditioner, refinement).  Its backward is the adjoint method:
    e = K_v alpha - y_v,  g = (2 / m_v) K_v^T e,  (K + lambda I) beta = g
    dL/dlambda = -beta^T alpha
    dL/dh      = (2 / m_v) e^T (dK_v/dh) alpha - beta^T (dK/dh) alpha
where the adjoint system is solved with the same factor (K and K_hss are
symmetric) and both dK/dh contractions are the dh output of the fused
backward.  A change of lambda needs no new compression (Section 5.3); a new h
does.  Every product and solve runs in libkrr; this module only orders calls.
"""
import math

import torch

from . import (HssOptions, ULV, cluster_2mn, gather_rows, kernel_matvec, kernel_matvec_bwd, refine, HSS,
               scatter_rows)


class KernelMatvec(torch.autograd.Function):
    """Out = K(X, Y; h) W (FP64 W and Out); gradients for X, Y, W and h."""

    @staticmethod
    def forward(ctx, X, Y, W, h, prec="f32"):
        hv = float(h)
        ctx.save_for_backward(X, Y, W)
        ctx.h, ctx.prec = hv, prec
        return kernel_matvec(X, Y, hv, W.contiguous(), prec=prec)

    @staticmethod
    def backward(ctx, G):
        X, Y, W = ctx.saved_tensors
        want = []
        if ctx.needs_input_grad[0]:
            want.append("dX")
        if ctx.needs_input_grad[1]:
            want.append("dY")
        if ctx.needs_input_grad[2]:
            want.append("dW")
        if ctx.needs_input_grad[3]:
            want.append("dh")
        if not want:
            return None, None, None, None, None
        out = kernel_matvec_bwd(X, Y, ctx.h, W.contiguous(), G.contiguous().to(torch.float64), prec=ctx.prec,
                                want=tuple(want))
        dX = out.get("dX")
        dY = out.get("dY")
        dW = out.get("dW")
        dh = out.get("dh")
        if dX is not None:
            dX = dX.to(X.dtype)
        if dY is not None:
            dY = dY.to(Y.dtype)
        if dh is not None:
            dh = dh.reshape(()).to(torch.float64)
        return dX, dY, dW, dh, None


class _State:
    pass


def _fit_alpha(st, h, lam, opts, tol, max_iter):
    st.tree_perm, st.tree = cluster_2mn(st.X, st.leaf, st.seed) if st.tree is None else (st.tree_perm, st.tree)
    if st.Xp is None:
        st.Xp = gather_rows(st.X, st.tree_perm)
        st.yp = gather_rows(st.y.reshape(-1, 1), st.tree_perm)
    H = HSS(st.tree, st.Xp, h, opts)
    F = ULV(H, lam, shifted=True)
    a = F.solve(st.yp)
    info = refine(F, st.Xp, h, lam, st.yp, a, tol=tol, max_iter=max_iter, mv_prec=st.prec)
    return H, F, a, info


class ValidationLoss(torch.autograd.Function):
    """L(log h, log lambda) for fixed training / validation data."""

    @staticmethod
    def forward(ctx, log_h, log_lam, st):
        h = math.exp(float(log_h))
        lam = math.exp(float(log_lam))
        H, F, a, info = _fit_alpha(st, h, lam, st.opts, st.tol, st.max_iter)
        f = kernel_matvec(st.Xv, st.Xp, h, a, prec=st.prec)
        e = f[:, 0] - st.yv
        mv = st.Xv.shape[0]
        L = float((e * e).sum().item() / mv)
        ctx.st, ctx.h, ctx.lam = st, h, lam
        ctx.keep = (H, F, a, e)
        st.last_info = info
        return torch.tensor(L, dtype=torch.float64, device=log_h.device)

    @staticmethod
    def backward(ctx, gL):
        st, h, lam = ctx.st, ctx.h, ctx.lam
        H, F, a, e = ctx.keep
        mv = st.Xv.shape[0]
        Ge = (2.0 / mv) * e.reshape(-1, 1)
        # g = (2 / m_v) K(Xp, Xv) e
        g = kernel_matvec(st.Xp, st.Xv, h, Ge.contiguous(), prec=st.prec)
        # adjoint solve with the same (symmetric) preconditioner
        beta = F.solve(g)
        refine(F, st.Xp, h, lam, g, beta, tol=st.tol, max_iter=st.max_iter, mv_prec=st.prec)
        dL_dlam = -float((beta * a).sum().item())
        # (2 / m_v) e^T dK_v/dh alpha and beta^T dK/dh alpha, both the fused backward's dh
        t1 = kernel_matvec_bwd(st.Xv, st.Xp, h, a, Ge.contiguous(), prec=st.prec, want=("dh",))["dh"].item()
        t2 = kernel_matvec_bwd(st.Xp, st.Xp, h, a, beta.contiguous(), prec=st.prec, want=("dh",))["dh"].item()
        dL_dh = t1 - t2
        st.last_grad = (h * dL_dh, lam * dL_dlam)
        go = float(gL)
        dev = gL.device
        return (torch.tensor(go * h * dL_dh, dtype=torch.float64, device=dev),
                torch.tensor(go * lam * dL_dlam, dtype=torch.float64, device=dev), None)


def validation_loss(log_h, log_lam, X, y, Xv, yv, leaf=128, opts: HssOptions = None, tol=1e-6, max_iter=300,
                    prec="f32", seed=7, state=None):
    """Differentiable validation MSE; reuse `state` to keep the cluster tree.

    prec: arithmetic of the kernel products (refinement, validation scores,
    backward); the refinement stops at relative residual tol."""
    st = state if state is not None else _State()
    if state is None:
        st.X, st.y, st.Xv, st.yv = X, y.to(torch.float64), Xv, yv.to(torch.float64)
        st.leaf, st.seed, st.tree, st.tree_perm, st.Xp, st.yp = leaf, seed, None, None, None, None
        st.opts = opts if opts is not None else HssOptions(rtol=1e-2, atol=1.0, r0=256, dr=256, r_max=256,
                                                           prec="f16", cap_policy=1)
        st.tol, st.max_iter, st.prec = tol, max_iter, prec
    return ValidationLoss.apply(log_h, log_lam, st), st
