"""Device memory of the library through a caller's allocator: with counting
callbacks registered (wrapping torch's caching allocator), a whole fit, a
prediction and the clustering orderings make no hipMalloc of their own, every
buffer they take comes from the callbacks, and every one of them is returned
once the results and handles are gone."""
import gc

import numpy as np
import torch

import synthdata as sd
import pytest

pytestmark = pytest.mark.gpu


def test_every_buffer_from_the_registered_allocator(gpu_lib):
    taken, returned = [], []

    def alloc(size, stream):
        p = torch.cuda.caching_allocator_alloc(int(size), stream=int(stream or 0))
        taken.append(p)
        return p

    def free(ptr, stream):
        returned.append(ptr)
        torch.cuda.caching_allocator_delete(int(ptr))

    p = sd.c1_two_gaussians(n=3000, m=100)
    X = torch.from_numpy(p.X.astype(np.float32)).cuda()
    y = torch.from_numpy(p.y).cuda()
    Xt = torch.from_numpy(p.Xt.astype(np.float32)).cuda()
    torch.cuda.synchronize()
    gpu_lib.set_allocator(alloc, free)
    try:
        d0, c0 = gpu_lib.alloc_counts()
        res = gpu_lib.fit(X, y, p.h, p.lam, leaf=64, opts=gpu_lib.HssOptions(rtol=1e-4, r0=64, prec="f16"))
        gpu_lib.predict(Xt, res.Xp, p.h, res.alpha_perm)
        for m in ("kd", "pca"):
            gpu_lib.cluster_order(X, 64, m)
        torch.cuda.synchronize()
        assert res.info["refine"]["converged"]
        del res
        gc.collect()
        torch.cuda.synchronize()
        d1, c1 = gpu_lib.alloc_counts()
    finally:
        gpu_lib.set_allocator()  # torch's caching allocator again
    assert d1 == d0, "the library called hipMalloc while an allocator was registered"
    assert c1 - c0 == len(taken) > 0
    assert sorted(taken) == sorted(returned)
