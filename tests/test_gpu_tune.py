"""The launch-shape autotuner: it records the fastest knob values per shape in
its JSON cache, `apply` restores them, and the kernels stay within their error
bounds at any knob value."""
import json

import numpy as np
import pytest
import torch

import synthdata as sd
from gpu_util import fp32_product_bound, leaf_ranges, mfma_sample_bound
from oracle import cluster as oc, cmath

pytestmark = pytest.mark.gpu

KNOBS = ("symmetric", "sample_rb", "mv_blocks", "sym_chunk")


@pytest.fixture
def restore(gpu_lib):
    saved = {k: gpu_lib.get_tuning(k) for k in KNOBS}
    yield
    for k, v in saved.items():
        gpu_lib.set_tuning(k, v)


def test_autotune_cache_and_apply(gpu_lib, restore, tmp_path):
    from paper_1803_10274_amd import tune
    path = str(tmp_path / "tune.json")
    entry = tune.autotune(d=8, r=64, prec="f16", n=8192, reps=1, path=path)
    assert set(entry["knobs"]) == {"sample_rb", "mv_blocks", "sym_chunk"}
    for k, v in entry["knobs"].items():
        assert v in tune.CANDIDATES[k]
    with open(path) as f:
        db = json.load(f)
    assert tune.cache_key(8, 64, "f16") in db
    for k in ("sample_rb", "mv_blocks", "sym_chunk"):
        gpu_lib.set_tuning(k, tune.CANDIDATES[k][-1])
    assert tune.apply(8, 64, "f16", path=path) == entry["knobs"]
    for k, v in entry["knobs"].items():
        assert gpu_lib.get_tuning(k) == v
    assert tune.apply(9, 64, "f16", path=path) is None or tune._width(9) == 12


@pytest.mark.parametrize("rb", [1, 2, 4, 8])
def test_sampler_any_pass_width(gpu_lib, restore, rb):
    gpu_lib.set_tuning("sample_rb", rb)
    n, h = 900, 0.75
    X = sd.c2_sixteen_gaussians(n=n, m=1).X
    t = oc.cluster2mn(X, 100, 1)
    Xp = np.ascontiguousarray(X[t.perm])
    lb, le = leaf_ranges(t.nodes, n)
    R = sd.random_block(n, 288, seed=rb)
    Xd = torch.from_numpy(Xp).cuda()
    S = gpu_lib.kernel_sample(Xd, h, torch.from_numpy(R).cuda(), torch.from_numpy(lb).cuda(),
                              torch.from_numpy(le).cuda(), prec="f16", split_terms=2).cpu().numpy()
    rows = np.arange(n)
    ref = cmath.sample_masked(Xp, R, h, lb, le, rows)
    assert np.all(np.abs(S - ref) <= mfma_sample_bound(Xp, R, h, lb, le, "f16", 2, rows))


@pytest.mark.parametrize("blocks,chunk", [(64, 64), (65536, 128), (1024, 1 << 20)])
def test_products_any_split(gpu_lib, restore, blocks, chunk):
    gpu_lib.set_tuning("mv_blocks", blocks)
    gpu_lib.set_tuning("sym_chunk", chunk)
    n, d, h = 2500, 8, 0.8
    X = sd.points(n, d, seed=3)
    W = sd.vectors(n, 2, seed=3)
    Xd = torch.from_numpy(X).cuda()
    ref = cmath.kmv(X, X, W, h)
    bound = fp32_product_bound(X, X, W, h)
    for Y in (Xd, Xd.clone()):  # symmetric and split-K forms
        out = gpu_lib.kernel_matvec(Xd, Y, h, torch.from_numpy(W).cuda(), prec="f32").cpu().numpy()
        assert np.all(np.abs(out - ref) <= bound)
