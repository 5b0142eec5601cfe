"""HSS compression and ULV on the 16-Gaussian distribution at n = 8192 (six
tree levels, leaf 128), with the absolute truncation used by the refined
fit: the GPU generators are compared with the oracle's randomized
construction run on the same random block, and the ULV factor with a dense
factorization of the exported matrix."""
import numpy as np
import pytest
import scipy.linalg as sla
import torch

import synthdata as sd
from oracle import cluster as oc, hss as oh, kernel as ok

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def case():
    p = sd.c2_sixteen_gaussians(n=8192, m=10)
    t = oc.cluster2mn(p.X, 128, 7)
    Xp = np.ascontiguousarray(p.X[t.perm])
    K = ok.kernel_dense(Xp, Xp, p.h)
    return p, t, Xp, K


@pytest.mark.parametrize("prec,r,atol", [("f16", 128, 1.0), ("f32", 128, 1.0), ("f16", 256, 0.3)])
def test_scale_compress_and_ulv(gpu_lib, case, prec, r, atol):
    p, t, Xp, K = case
    tree = gpu_lib.tree_from_nodes(t.nodes)
    H = gpu_lib.HSS(tree, _t(Xp), p.h, gpu_lib.HssOptions(rtol=1e-2, atol=atol, r0=r, dr=r, r_max=4 * r,
                                                          prec=prec, seed=5))
    ex = H.export()
    G = oh.HSS(nodes=t.nodes[:, :4])
    G.U, G.D, G.B, G.J = ex["U"], ex["D"], ex["B"], ex["J"]
    Kg = oh.assemble(G)
    rr = H.stats.r_final
    R = gpu_lib.random_block(5, p.n, rr).cpu().numpy().astype(np.float64)
    Ho = oh.randomized(Xp, t.nodes, p.h, 1e-2, R, atol=atol * np.sqrt(rr), K=K)
    Ko = oh.assemble(Ho)
    eg = np.linalg.norm(K - Kg)
    eo = np.linalg.norm(K - Ko)
    assert eg <= 1.5 * eo + 1e-9 * np.linalg.norm(K), (eg, eo)
    assert abs(H.stats.max_rank - Ho.max_rank()) <= 3
    lam = p.lam
    A = Kg + lam * np.eye(p.n)
    y = p.y[t.perm]
    F = gpu_lib.ULV(H, lam)
    got = F.solve(_t(y)).cpu().numpy()
    ref = sla.cho_solve(sla.cho_factor(A, lower=True), y)
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
