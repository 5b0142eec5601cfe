"""Host logic of the (h, lambda) descent (autograd.tune_hyperparameters) with
the validation loss replaced by a smooth stand-in on the CPU: steps alternate
lambda / h, move against the gradient's sign, halve until the loss falls,
accept only decreases, and pin the accepted h so that lambda trials find its
compression.  The GPU test of the same loop checks the loss itself."""
import math

import torch

import paper_1803_10274_amd.autograd as ag


def _fake_loss(calls):
    def validation_loss(a, b, X, y, Xv, yv, leaf=128, opts=None, tol=1e-6, max_iter=300, prec="f32", seed=7,
                        state=None):
        st = state if state is not None else ag._State()
        h = math.exp(float(a.detach()))
        cache = st.__dict__.setdefault("hss_cache", {})
        st.compressed = h not in cache
        if st.compressed:
            st.n_compress = getattr(st, "n_compress", 0) + 1
            for k in [k for k in cache if k != getattr(st, "pin_h", None)]:
                del cache[k]
            cache[h] = object()
        st.n_fits = getattr(st, "n_fits", 0) + 1
        calls.append((h, math.exp(float(b.detach())), getattr(st, "pin_h", None)))
        # minimum at h = 2, lambda = 0.5
        return (a - math.log(2.0)) ** 2 + 0.3 * (b - math.log(0.5)) ** 2 + 0.1, st
    return validation_loss


def test_descent_alternates_halves_and_pins(monkeypatch):
    calls = []
    monkeypatch.setattr(ag, "validation_loss", _fake_loss(calls))
    X = torch.zeros(3, 2)
    res = ag.tune_hyperparameters(X, X, X, X, 0.5, 8.0, steps=12, step=0.5)
    hist = res["history"]
    assert hist[0][0] == "start" and hist[0][5]
    kinds = [e[0] for e in hist[1:]]
    # lambda first, then h, each step possibly several halved trials
    assert kinds[0] == "lambda" and "h" in kinds
    acc = [e[3] for e in hist if e[4]]
    assert all(b < a for a, b in zip(acc, acc[1:]))
    assert res["loss"] == acc[-1]
    # a rejected trial is followed by a half-size trial of the same kind
    for prev, e in zip(hist[1:], hist[2:]):
        if not prev[4] and e[0] == prev[0]:
            i = 1 if e[0] == "h" else 2
            base = [x for x in hist[:hist.index(prev)] if x[4]][-1]
            assert math.isclose(abs(math.log(e[i] / base[i])), 0.5 * abs(math.log(prev[i] / base[i])))
    # lambda trials never compress; a compression is only made for a new h
    assert all(not e[5] for e in hist if e[0] == "lambda")
    assert all(e[1] != p[1] for p, e in zip(hist, hist[1:]) if e[5])
    assert res["n_fits"] == len(hist) == len(calls)
    assert res["n_compress"] == sum(1 for e in hist if e[5])
    # every lambda trial runs with its (accepted) h pinned, so it reuses that
    # h's compression; history and calls are one per fit, in order
    for e, (h, lam, pin) in zip(hist, calls):
        if e[0] == "lambda":
            assert pin == h == e[1]
    # six steps of 0.5 per coordinate reach the stand-in's minimum (log
    # distances 1.39 in h and 2.77 in lambda from the start)
    assert abs(math.log(res["h"] / 2.0)) < 0.3 and abs(math.log(res["lam"] / 0.5)) < 0.3
