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

from . import (HSS, HssOptions, ULV, cluster_2mn, dot_columns, gather_rows, kernel_matvec, kernel_matvec_bwd,
               refine, val_grad_finish, val_residual)


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
    # the compression depends on h only (fixed points, options and seed): a new
    # lambda refactors the one it has.  Kept: the latest and a pinned h's.
    cache = st.__dict__.setdefault("hss_cache", {})
    H = cache.get(h)
    st.compressed = H is None
    if H is None:
        H = HSS(st.tree, st.Xp, h, opts)
        st.n_compress = getattr(st, "n_compress", 0) + 1
        for k in [k for k in cache if k != getattr(st, "pin_h", None)]:
            del cache[k]
        cache[h] = H
    st.n_fits = getattr(st, "n_fits", 0) + 1
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
        # ge = (2 / m_v)(f - y_v), L = |f - y_v|^2 / m_v
        ge, loss = val_residual(f, st.yv.reshape(-1, 1))
        ctx.st, ctx.h, ctx.lam = st, h, lam
        ctx.keep = (H, F, a, ge)
        st.last_info = info
        return loss.reshape(())

    @staticmethod
    def backward(ctx, gL):
        st, h, lam = ctx.st, ctx.h, ctx.lam
        H, F, a, ge = ctx.keep
        # g = (2 / m_v) K(Xp, Xv) e
        g = kernel_matvec(st.Xp, st.Xv, h, ge, prec=st.prec)
        # adjoint solve with the same (symmetric) preconditioner
        beta = F.solve(g)
        refine(F, st.Xp, h, lam, g, beta, tol=st.tol, max_iter=st.max_iter, mv_prec=st.prec)
        bta = dot_columns(beta, a)
        # (2 / m_v) e^T dK_v/dh alpha and beta^T dK/dh alpha, both the fused backward's dh
        dh_v = kernel_matvec_bwd(st.Xv, st.Xp, h, a, ge, prec=st.prec, want=("dh",))["dh"]
        dh_t = kernel_matvec_bwd(st.Xp, st.Xp, h, a, beta.contiguous(), prec=st.prec, want=("dh",))["dh"]
        # (dL/dlog h, dL/dlog lambda) scaled by the upstream gradient
        out = val_grad_finish(bta, dh_v, dh_t, h, lam, gscale=gL)
        st.last_grad = out
        return out[0], out[1], None


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


def tune_hyperparameters(X, y, Xv, yv, h, lam, steps=8, step=0.5, shrink=3, leaf=128, opts: HssOptions = None,
                         tol=1e-6, max_iter=300, prec="f32", seed=7):
    """Gradient-driven choice of (h, lambda) by the validation MSE.

    The paper tunes these two by grid search or a black-box tuner, and notes
    that a new lambda changes only the diagonal while a new h needs a new
    compression (Section 5.3).  Here the steps alternate between the two
    coordinates, lambda first.  A lambda step refactors the compressed matrix
    it already has; an h step recompresses.  Each step moves its coordinate by
    `step` (log units) against the sign of its adjoint gradient.  It is halved,
    up to `shrink` times, until the loss falls, and is skipped if it never does.
    The gradient is taken only at accepted points.

    Returns a dict: h, lam, loss (at the accepted point), n_compress
    (compressions built), n_fits (factor + refinement runs), and history: one
    (kind, h, lam, loss, accepted, compressed) per fit, kind "start", "lambda"
    or "h"."""
    dev = X.device
    st = None

    def fit(lh, ll):
        nonlocal st
        a = torch.tensor(lh, dtype=torch.float64, device=dev, requires_grad=True)
        b = torch.tensor(ll, dtype=torch.float64, device=dev, requires_grad=True)
        L, st = validation_loss(a, b, X, y, Xv, yv, leaf=leaf, opts=opts, tol=tol, max_iter=max_iter, prec=prec,
                                seed=seed, state=st)
        return L, a, b

    def grad(L, a, b):
        L.backward()
        return a.grad.item(), b.grad.item()

    lh, ll = math.log(h), math.log(lam)
    L, a, b = fit(lh, ll)
    st.pin_h = math.exp(lh)
    loss = L.item()
    history = [("start", math.exp(lh), math.exp(ll), loss, True, st.compressed)]
    g = grad(L, a, b)
    for it in range(steps):
        k = 1 - it % 2  # index into g: 0 = log h, 1 = log lambda
        if g[k] == 0.0:
            continue
        d = -step if g[k] > 0 else step
        for _ in range(shrink + 1):
            cand = (lh + d, ll) if k == 0 else (lh, ll + d)
            Lc, a, b = fit(*cand)
            ok = Lc.item() < loss
            history.append(("h" if k == 0 else "lambda", math.exp(cand[0]), math.exp(cand[1]), Lc.item(), ok,
                            st.compressed))
            if ok:
                lh, ll = cand
                st.pin_h = math.exp(lh)
                loss = Lc.item()
                g = grad(Lc, a, b)
                break
            d *= 0.5
    return {"h": math.exp(lh), "lam": math.exp(ll), "loss": loss, "n_compress": st.n_compress,
            "n_fits": st.n_fits, "history": history}
