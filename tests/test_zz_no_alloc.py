"""krr_predict_noalloc against krr_predict through the C-ABI: two calls in a
row on the same device (the second with a smaller input, so the static
scratch holds the first call's contents), FP32 and FP64 entries, one and ten
right-hand sides; the scores must equal krr_predict's (same kernels, same
column splits) and the labels too.  No hipMalloc is made by the no-alloc
calls, and sizes beyond the static scratch are refused."""
import ctypes

import numpy as np
import pytest
import torch

import synthdata as sd

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _case(n, m, d, k, seed):
    Xp = sd.points(n, d, seed=seed, scale=0.5)
    Xt = sd.points(m, d, seed=seed + 1, scale=0.5)
    a = sd.vectors(n, k, seed=seed + 2)
    return _t(Xt), _t(Xp), _t(a)


@pytest.mark.parametrize("prec,k", [("f32", 1), ("f64", 1), ("f32", 10), ("f64", 10)])
def test_noalloc_matches_predict_twice(gpu_lib, prec, k):
    h = 1.1
    for n, m, d in ((20000, 3000, 8), (5000, 700, 5)):  # the second call is smaller
        Xt, Xp, a = _case(n, m, d, k, seed=n + k)
        ref_s, ref_l = gpu_lib.predict(Xt, Xp, h, a, prec=prec)
        scores = torch.full((m, k), float("nan"), dtype=torch.float64, device="cuda")
        labels = torch.full((m,), -7, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        d0, c0 = gpu_lib.alloc_counts()
        gpu_lib.predict_noalloc(Xt, Xp, h, a, scores, labels, prec=prec)
        torch.cuda.synchronize()
        assert gpu_lib.alloc_counts() == (d0, c0)
        assert torch.equal(scores, ref_s), (n, m, float((scores - ref_s).abs().max()))
        assert torch.equal(labels, ref_l)


def test_noalloc_rejects_oversize_and_aliasing(gpu_lib):
    from paper_1803_10274_amd import _lib
    L = gpu_lib.load()
    n, m = 1 << 22, 1 << 16  # the FP32 column data alone exceed 128 MiB
    Xp = torch.zeros((n, 8), dtype=torch.float32, device="cuda")
    Xt = torch.zeros((m, 8), dtype=torch.float32, device="cuda")
    a = torch.zeros((n, 1), dtype=torch.float64, device="cuda")
    s = torch.zeros((m, 1), dtype=torch.float64, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    rc = L.krr_predict_noalloc(P(Xt), m, P(Xp), n, 8, _lib.KRR_F32, 1.0, P(a), 1, P(s), None, _lib.KRR_F32, None)
    assert rc == _lib.KRR_E_INVAL and b"limit" in L.krr_last_error()
    rc = L.krr_predict_noalloc(P(Xp), n, P(Xp), n, 8, _lib.KRR_F32, 1.0, P(a), 1, P(a), None, _lib.KRR_F32, None)
    assert rc == _lib.KRR_E_INVAL and b"alias" in L.krr_last_error()
