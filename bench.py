"""Benchmark: Gaussian-kernel ridge regression fit at n = 2^20, d = 8.

One step = one pass of the whole hot path on the sixteen-Gaussian workload
(n = 1,048,576 training points, d = 8, h = 0.75, lambda = 10, 100,000 test
points, synthetic data): 2MN clustering, permutation, HSS compression with
mixed-precision sampling (FP16 hi/lo split entries, FP32 accumulation), FP64
IDs and ULV factorization, solve, PCG refinement on the FP32 kernel product to
a relative residual of 1e-6, un-permutation, and prediction of the test set.

Reported: the fit time of the mixed path (value, seconds, lower is better),
the same fit with FP32 sampling (`fp32`), the two hot kernels against their
rooflines (the sampling product on the matrix cores; the refinement's kernel
product on the vector ALUs), each timed with HIP events on the stream it runs
on, the batched form (64 ragged problems) and the hyper-parameter gradient
(n = 131,072, d = 18) as extra timed legs, and the CPU oracle on a bounded
sample.

`--kernels-only` runs just one launch of each hot kernel (plus a plain copy of
known size, for counter calibration) on the same workload: the command the
hardware-counter profiles are taken with.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published dense peaks (FLOP/s)
PEAK = {"f16": 2.5e15, "bf16": 2.5e15, "f32": 157.3e12, "f64": 78.6e12}
PEAK_FP64_VECTOR = 78.6e12
PEAK_F32_VECTOR = 157.3e12
# transcendental (v_exp_f32) issue at a quarter of the lane rate: 256 CUs x 64 lanes x 2.4 GHz / 4
PEAK_EXP2 = 256 * 64 * 2.4e9 / 4

# HBM traffic per launch at n = 2^20, d = 8 (r = 256 for the sampler), from
# two hardware-counter runs of `bench.py --kernels-only` (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch), each scaled by what the counter reads for a
# plain 1 GiB device copy in the same run (FETCH_SIZE 524,314 KiB -> x2.000;
# WRITE_SIZE 1,048,576 KiB -> x1.000).  Valid only while the kernel's source
# file is unchanged (sha256 below); otherwise the bench reports null.
PMC_TRAFFIC = {
    "sampling": {"fetch_kib": 930383607.1875, "write_kib": 1048576.0, "fetch_scale": 2.0, "write_scale": 1.0,
                 "source": "paper_1803_10274_amd/csrc/sample_mfma.hip",
                 "sha256": "bcd0d5396bd1701e27d4c92645b02fded9aa6e4ae6559e2bc90a8edeb4e761b3", "n": 1 << 20, "r": 256},
    # the symmetric product's six launches: column data, FP32 weights,
    # diagonal blocks, row-block anchors, upper triangle, reduction
    "kernel_product": {"fetch_kib": 17890529.375, "write_kib": 6384645.15625, "fetch_scale": 2.0, "write_scale": 1.0,
                       "source": "paper_1803_10274_amd/csrc/matvec.hip",
                       "sha256": "a3885e9b4f9550f2388f8e28c44e3c996e5c34ab6301c944f84e4f613bd03194",
                       "n": 1 << 20, "r": None},
    # the same six launches through the negligible-tile map
    "kernel_product_mapped": {"fetch_kib": 8465179.125, "write_kib": 6115831.375, "fetch_scale": 2.0,
                              "write_scale": 1.0, "source": "paper_1803_10274_amd/csrc/matvec.hip",
                              "sha256": "a3885e9b4f9550f2388f8e28c44e3c996e5c34ab6301c944f84e4f613bd03194",
                              "n": 1 << 20, "r": None},
}

def pmc_traffic(kind, n, r=None):
    """Calibrated HBM bytes per launch, or None if the counters do not
    describe the current kernel and size."""
    import hashlib
    t = PMC_TRAFFIC.get(kind)
    if t is None or t["n"] != n or (t["r"] is not None and t["r"] != r):
        return None
    with open(os.path.join(ROOT, t["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["sha256"]:
            return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


# Executed matrix-core work per launch from hardware counters
# (SQ_INSTS_VALU_MFMA_MOPS_* count matrix-core math operations in units of
# 512; SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE give the busy share), from
# `rocprofv3 --pmc` runs of `bench.py --kernels-only`; valid only while the
# kernel's source file is unchanged (sha256), otherwise reported as null.
PMC_MFMA = {
    "sampling": {"mops": {"f16": 659243755520.0, "bf16": 274886295552.0}, "mfma_busy_frac": 0.3469,
                 "valu_busy_frac": 0.2214, "coexec_frac": 0.0445,
                 "source": "paper_1803_10274_amd/csrc/sample_mfma.hip",
                 "sha256": "bcd0d5396bd1701e27d4c92645b02fded9aa6e4ae6559e2bc90a8edeb4e761b3", "n": 1 << 20, "r": 256,
                 "profile": "profiles/k_sample_mfma_sixteen_gaussians_n1048576_r256.md"},
    "sampling_every_tile": {"mops": {"f16": 2199023255552.0, "bf16": 274886295552.0}, "mfma_busy_frac": 0.5938,
                            "valu_busy_frac": 0.3308, "coexec_frac": 0.0863,
                            "source": "paper_1803_10274_amd/csrc/sample_mfma.hip",
                            "sha256": "bcd0d5396bd1701e27d4c92645b02fded9aa6e4ae6559e2bc90a8edeb4e761b3",
                            "n": 1 << 20, "r": 256,
                            "profile": "profiles/k_sample_mfma_sixteen_gaussians_n1048576_r256.md"},
    "kernel_product": {"mops": {"bf16": 137371844608.0}, "mfma_busy_frac": 0.2973, "valu_busy_frac": 0.864,
                       "coexec_frac": 0.1303, "source": "paper_1803_10274_amd/csrc/matvec.hip",
                       "sha256": "a3885e9b4f9550f2388f8e28c44e3c996e5c34ab6301c944f84e4f613bd03194",
                       "n": 1 << 20, "r": None, "profile": "profiles/k_kmv_symb_sixteen_gaussians_n1048576.md"},
    "kernel_product_mapped": {"mops": {"bf16": 41267506944.0}, "mfma_busy_frac": 0.1974, "valu_busy_frac": 0.6788,
                              "coexec_frac": 0.0738, "source": "paper_1803_10274_amd/csrc/matvec.hip",
                              "sha256": "a3885e9b4f9550f2388f8e28c44e3c996e5c34ab6301c944f84e4f613bd03194",
                              "n": 1 << 20, "r": None,
                              "profile": "profiles/k_kmv_symb_tile_map_sixteen_gaussians_n1048576.md"},
}


def pmc_mfma(kind, n, r, launch_s):
    """Counter-based matrix-core figures for one launch, or nulls."""
    import hashlib
    t = PMC_MFMA.get(kind)
    none = {"executed_mfma_tflops": None, "executed_mfma_frac": None, "mfma_busy_frac": None}
    if t is None or t["n"] != n or (t["r"] is not None and t["r"] != r):
        return none
    with open(os.path.join(ROOT, t["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["sha256"]:
            return none
    ops = 512.0 * sum(t["mops"].values())
    peak = sum(PEAK[k] * v for k, v in t["mops"].items()) / max(sum(t["mops"].values()), 1e-30)
    return {"executed_mfma_tflops": ops / launch_s / 1e12, "executed_mfma_frac": ops / launch_s / peak,
            "mfma_busy_frac": t.get("mfma_busy_frac"), "valu_busy_frac": t.get("valu_busy_frac"),
            "mfma_valu_coexec_frac": t.get("coexec_frac"), "mfma_counters": t["profile"]}


def fp64_relres(krr, res, y, p):
    """The fitted coefficients' relative residual recomputed with the FP64
    kernel product (the library's own FP64 kernel; the CPU oracle certifies
    the same coefficients separately from a dump)."""
    import torch
    yp = krr.gather_rows(y.reshape(-1, 1).contiguous(), res.perm)
    a64 = res.alpha_perm.reshape(-1, 1).contiguous()
    r64 = yp - krr.kernel_matvec(res.Xp, res.Xp, p.h, a64, prec="f64") - p.lam * a64
    return float(torch.linalg.norm(r64) / torch.linalg.norm(yp))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--m", type=int, default=100_000)
    ap.add_argument("--prec", default="f16")
    ap.add_argument("--split", type=int, default=2)
    ap.add_argument("--rtol", type=float, default=1e-2)
    ap.add_argument("--r0", type=int, default=256)
    ap.add_argument("--atol", type=float, default=6.0)
    ap.add_argument("--r-max", type=int, default=4096, help="largest sample width adaptive growth may reach")
    ap.add_argument("--cap-policy", type=int, default=0,
                    help="at r_max: 0 fails with a rank-cap error, 1 truncates every rank")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner before the fits")
    ap.add_argument("--tune-dir", default=os.path.join(ROOT, "gpurun_out"),
                    help="where the autotuner's cache file is written")
    ap.add_argument("--dump-alpha", metavar="DIR",
                    help="write the fitted coefficients (original order) of the headline and image-like fits "
                         "to DIR for certification by the CPU oracle")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-sampling comparison fit")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-problem batched leg")
    ap.add_argument("--no-grad", action="store_true", help="skip the gradient leg")
    ap.add_argument("--no-image", action="store_true", help="skip the image-like (d = 784) leg")
    ap.add_argument("--kernels-only", action="store_true", help="one launch of each hot kernel (profiling)")
    ap.add_argument("--wide-kernels", action="store_true",
                    help="launches of the wide-point kernel products at the image-like size (profiling)")
    ap.add_argument("--reps", type=int, default=3, help="launches per kernel timing")
    ap.add_argument("--grad-kernels", action="store_true",
                    help="the fused backward's two dh launches at the gradient workload's size (profiling)")
    ap.add_argument("--orderings", action="store_true",
                    help="the Table 2 style memory / rank comparison of the orderings on 10,000-point stand-ins")
    ap.add_argument("--cpu-dense", action="store_true",
                    help="time the oracle's dense FP64 KRR fit on the host at n = 1,000, 8,192 and 32,768")
    ap.add_argument("--scaling", action="store_true",
                    help="fit the sixteen-Gaussian workload at n = 2^16 .. 2^20 and print the phase times per n")
    ap.add_argument("--summarize-trace", metavar="CSV",
                    help="print per-(kernel, grid) launch statistics of a rocprofv3 kernel-trace CSV and exit")
    return ap.parse_args()


def summarize_trace(path, top=25):
    """Launch statistics of a rocprofv3 kernel trace grouped by kernel and grid
    size (the same kernel at different sizes is listed separately)."""
    import csv
    groups = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            grid = row.get("Grid_Size") or "x".join(row.get(k, "?") for k in ("Grid_Size_X", "Grid_Size_Y",
                                                                            "Grid_Size_Z"))
            key = (row["Kernel_Name"], grid)
            dur = int(row["End_Timestamp"]) - int(row["Start_Timestamp"])
            g = groups.setdefault(key, [0, 0, None, 0])
            g[0] += 1
            g[1] += dur
            g[2] = dur if g[2] is None else min(g[2], dur)
            g[3] = max(g[3], dur)
    total = sum(g[1] for g in groups.values())
    print("| kernel | grid | calls | total ms | avg ms | min ms | max ms | % |")
    print("|---|---|---|---|---|---|---|---|")
    for (name, grid), (c, t, lo, hi) in sorted(groups.items(), key=lambda kv: -kv[1][1])[:top]:
        short = name.replace("krr::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        print(f"| {short[:70]} | {grid} | {c} | {t / 1e6:.3f} | {t / c / 1e6:.3f} | {lo / 1e6:.3f} | {hi / 1e6:.3f} | "
              f"{100.0 * t / total:.2f} |")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def leaf_arrays(nodes, n, dev):
    import numpy as np
    import torch
    lbn = np.empty(n, dtype=np.int32)
    len_ = np.empty(n, dtype=np.int32)
    for b, e in nodes[nodes[:, 2] < 0][:, :2]:
        lbn[b:e] = b
        len_[b:e] = e
    return torch.from_numpy(lbn).to(dev), torch.from_numpy(len_).to(dev)


def time_launches(fn, reps):
    """Average duration of fn() measured with HIP events on torch's current
    stream, which is the stream the library launches on."""
    import torch
    fn()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def kernels_only(args):
    """One launch each: a 1 GiB device copy, the sampling product (with the
    negligible-tile skip, then with every tile evaluated) and the refinement
    kernel product (every entry, then recording its tile map, then through
    the map), on the 16-Gaussian workload in tree order."""
    import torch

    import paper_1803_10274_amd as krr
    import synthdata as sd
    krr.load()
    dev = torch.device("cuda:0")
    p = sd.c2_sixteen_gaussians(n=args.n, m=1)
    X = torch.from_numpy(p.X).to(dev)
    perm, tree = krr.cluster_2mn(X, p.leaf, 7)
    Xp = krr.gather_rows(X, perm)
    lb, le = leaf_arrays(tree.nodes, args.n, dev)
    R = krr.random_block(1, args.n, args.r0)
    w = torch.from_numpy(sd.vectors(args.n, 1, seed=3)).to(dev)
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    log("copy 1 GiB")
    b.copy_(a)
    torch.cuda.synchronize()
    log("sampling product (negligible tiles skipped)")
    krr.kernel_sample(Xp, p.h, R, lb, le, prec=args.prec, split_terms=args.split)
    torch.cuda.synchronize()
    log("sampling product (every tile evaluated)")
    krr.set_tuning("sample_skip", 0)
    krr.kernel_sample(Xp, p.h, R, lb, le, prec=args.prec, split_terms=args.split)
    krr.set_tuning("sample_skip", 1)
    torch.cuda.synchronize()
    log("kernel product")
    krr.kernel_matvec(Xp, Xp, p.h, w, prec="f32")
    torch.cuda.synchronize()
    log("kernel product through its tile map: recording, then one product")
    tmap = krr.TileMap()
    tmap.matvec(Xp, p.h, w)
    torch.cuda.synchronize()
    tmap.matvec(Xp, p.h, w)
    torch.cuda.synchronize()
    del tmap
    print(json.dumps({"kernels_only": True, "n": args.n, "r": args.r0, "copy_bytes": 2 * a.numel() * 4}), flush=True)


def grad_kernels(args):
    """The two dh launches of the validation-loss gradient on the
    eight-Gaussian workload (n = 131,072 training, 16,384 validation, d = 18):
    K o T products of the validation rows against the training points and of
    the training points against themselves, each timed with HIP events."""
    import torch

    import paper_1803_10274_amd as krr
    import synthdata as sd
    krr.load()
    p = sd.c5_eight_gaussians()
    X = torch.from_numpy(p.X).cuda()
    Xv = torch.from_numpy(p.Xt).cuda()
    a = torch.from_numpy(sd.vectors(p.X.shape[0], 1, seed=3)).cuda()
    g = torch.from_numpy(sd.vectors(p.Xt.shape[0], 1, seed=4)).cuda()
    b = torch.from_numpy(sd.vectors(p.X.shape[0], 1, seed=5)).cuda()
    torch.cuda.synchronize()
    out = {"grad_kernels": True, "n": p.X.shape[0], "m_v": p.Xt.shape[0], "d": p.d}
    for name, fn, entries in (
            ("validation", lambda: krr.kernel_matvec_bwd(Xv, X, p.h, a, g, want=("dh",)),
             float(p.Xt.shape[0]) * p.X.shape[0]),
            ("training", lambda: krr.kernel_matvec_bwd(X, X, p.h, a, b, want=("dh",)),
             float(p.X.shape[0]) ** 2)):
        log(f"dh launch: {name}")
        t = time_launches(fn, args.reps)
        out[name] = {"s": t, "entries_per_s": entries / t, "exp2_rate_frac": entries / t / PEAK_EXP2}
    print(json.dumps(out), flush=True)


def orderings():
    """Section 4.3's comparison (Table 2's memory columns) on synthetic
    stand-ins of 10,000 training points with z-scored columns, as the paper
    normalises its data: HSS memory (the paper's metric, MB) and maximum rank
    for the natural order (NP), KD tree, PCA tree and 2MN (mean over three
    seeds, as the paper averages three runs), leaf 16, relative tolerance
    0.1, FP32 sampling from r = 128 grown as needed.  One JSON line per
    stand-in."""
    import numpy as np
    import torch

    import paper_1803_10274_amd as krr
    import synthdata as sd
    krr.load()
    cases = [("sixteen_gaussians d=8", sd.c2_sixteen_gaussians(n=10_000, m=1, d=8).X, 1.0),
             ("sixteen_gaussians d=16", sd.c2_sixteen_gaussians(n=10_000, m=1, d=16).X, 1.0),
             ("eight_gaussians d=18", sd.c5_eight_gaussians(n=10_000, m=1).X, 1.5),
             ("sixteen_gaussians d=54", sd.c2_sixteen_gaussians(n=10_000, m=1, d=54).X, 1.0),
             ("image_like d=784", sd.c3_image_like(n=10_000, m=1).X, 4.0)]
    opts = krr.HssOptions(rtol=0.1, r0=128, dr=128, r_max=4096, prec="f32")
    for name, X, h in cases:
        X = X.astype(np.float64)
        sdev = X.std(axis=0)
        Z = ((X - X.mean(axis=0)) / np.where(sdev > 0, sdev, 1.0)).astype(np.float32)
        Xt = torch.from_numpy(Z).cuda()
        mem, rank = {}, {}
        for m in ("np", "kd", "pca", "2mn"):
            b, k = [], []
            for seed in ((7, 8, 9) if m == "2mn" else (7,)):
                log(f"orderings: {name}, {m}, seed {seed}")
                perm, tree = krr.cluster_order(Xt, 16, m, seed=seed)
                H = krr.HSS(tree, krr.gather_rows(Xt, perm), h, opts)
                b.append(H.stats.bytes_paper / 1e6)
                k.append(H.stats.max_rank)
            mem[m], rank[m] = round(float(np.mean(b)), 2), int(max(k))
        print(json.dumps({"orderings": True, "workload": name, "n": 10_000, "h": h, "leaf": 16, "rtol": 0.1,
                          "memory_mb": mem, "max_rank": rank}), flush=True)


def scaling(args):
    """The headline fit at n = 2^16 .. 2^20 (same options, one warm-up fit at
    each n, then one timed), one JSON line per n: phase times, the sampling
    kernel's time, iterations and the FP64 residual.  Checks the work model:
    sampling O(n^2 r), clustering / compression / factorization / solve near
    O(n), refinement O(n^2) per iteration."""
    import torch

    import paper_1803_10274_amd as krr
    import synthdata as sd
    krr.load()
    dev = torch.device("cuda:0")
    opts = krr.HssOptions(rtol=args.rtol, atol=args.atol, r0=args.r0, dr=args.r0, r_max=args.r_max,
                          prec=args.prec, split_terms=args.split, cap_policy=args.cap_policy)
    for lg in range(16, 21):
        n = 1 << lg
        p = sd.c2_sixteen_gaussians(n=n, m=1)
        X = torch.from_numpy(p.X).to(dev)
        y = torch.from_numpy(p.y).to(dev)
        torch.cuda.synchronize()
        log(f"scaling: n = {n}")
        for rep in range(2):
            t0 = time.perf_counter()
            res = krr.fit(X, y, p.h, p.lam, leaf=p.leaf, opts=opts, tol=1e-6, max_iter=300, raise_on_fail=False)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
        out = {"scaling": True, "n": n, "fit_s": t, "phases_s": res.info["phases"],
               "t_sample_ms": res.info["hss"]["t_sample_ms"], "t_id_ms": res.info["hss"]["t_id_ms"],
               "r_final": res.info["hss"]["r_final"], "max_rank": res.info["hss"]["max_rank"],
               "bytes_paper": res.info["hss"]["bytes_paper"], "ulv_shift": res.info["ulv_shift"],
               "refine_iterations": res.info["refine"]["iterations"],
               "relres_fp64": fp64_relres(krr, res, y, p)}
        print(json.dumps(out), flush=True)
        del res, X, y


def wide_kernels(args):
    """The wide-point kernel products at the image-like size (n = 60,000,
    d = 784, ten right-hand sides): two launches with FP32 entries (BF16
    three-term exponents), one with FP64 entries."""
    import numpy as np
    import torch

    import paper_1803_10274_amd as krr
    import synthdata as sd
    krr.load()
    dev = torch.device("cuda:0")
    p = sd.c3_image_like()
    X = torch.from_numpy(np.ascontiguousarray(p.X, dtype=np.float32)).to(dev)
    W = torch.from_numpy(sd.vectors(p.n, 10, seed=3)).to(dev)
    torch.cuda.synchronize()
    for prec in ("f32", "f32", "f64"):
        log(f"wide kernel product, {prec} entries")
        krr.kernel_matvec(X, X, p.h, W, prec=prec)
        torch.cuda.synchronize()
    print(json.dumps({"wide_kernels": True, "n": p.n, "d": p.d, "nrhs": 10}), flush=True)


def main():
    args = parse()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.wide_kernels:
        wide_kernels(args)
        return
    if args.kernels_only:
        kernels_only(args)
        return
    if args.scaling:
        scaling(args)
        return
    if args.grad_kernels:
        grad_kernels(args)
        return
    if args.orderings:
        orderings()
        return
    if args.cpu_dense:
        cpu_dense()
        return
    import numpy as np
    import torch

    import paper_1803_10274_amd as krr
    import synthdata as sd

    krr.load()
    dev = torch.device("cuda:0")
    p = sd.c2_sixteen_gaussians(n=args.n, m=args.m)
    X = torch.from_numpy(p.X).to(dev)
    y = torch.from_numpy(p.y).to(dev)
    Xt = torch.from_numpy(p.Xt).to(dev)
    torch.cuda.synchronize()
    opts = krr.HssOptions(rtol=args.rtol, atol=args.atol, r0=args.r0, dr=args.r0, r_max=args.r_max,
                          prec=args.prec, split_terms=args.split, cap_policy=args.cap_policy)
    tune_cache = None
    if not args.no_tune:
        # launch shapes for this point width and sample width, chosen by the
        # autotuner at the workload's own size before anything is timed (the
        # best column chunk of the symmetric product depends on n)
        from paper_1803_10274_amd import tune
        tune_cache = os.path.join(args.tune_dir, "tune.json")
        log("autotuning launch shapes")
        tune.autotune(p.d, r=args.r0, prec=args.prec, n=args.n, split_terms=args.split, reps=2, path=tune_cache)
        log(f"tuned: {json.load(open(tune_cache))}")

    def step(o):
        res = krr.fit(X, y, p.h, p.lam, leaf=p.leaf, opts=o, tol=1e-6, max_iter=300, raise_on_fail=False,
                      tune_cache=tune_cache)
        torch.cuda.synchronize()
        t_fit = time.perf_counter()
        _, lab = krr.predict(Xt, res.Xp, p.h, res.alpha_perm)
        torch.cuda.synchronize()
        return res, lab, t_fit

    for i in range(args.warmup):
        t0 = time.perf_counter()
        res, lab, t_fit = step(opts)
        log(f"warmup {i}: fit {t_fit - t0:.3f} s, total {time.perf_counter() - t0:.3f} s, "
            f"phases {res.info['phases']}, shift {res.info['ulv_shift']}, hss {res.info['hss']}, "
            f"refine it {res.info['refine']['iterations']} relres {res.info['refine']['relres'][0]:.2e}")
    fit_times, step_times = [], []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        res, lab, t_fit = step(opts)
        fit_times.append(t_fit - t0)
        step_times.append(time.perf_counter() - t0)
        log(f"step {i}: fit {fit_times[-1]:.3f} s, step {step_times[-1]:.3f} s, phases {res.info['phases']}, "
            f"refine {res.info['refine']['iterations']} it relres {res.info['refine']['relres'][0]:.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_all
    acc = float((lab.cpu().numpy() == p.yt.astype(np.int32)).mean())
    hs = res.info["hss"]
    rf = res.info["refine"]

    # FP32-sampling comparison fit, same data, tree, lambda and tolerance
    fp32 = None
    if not args.no_fp32:
        o32 = krr.HssOptions(rtol=args.rtol, atol=args.atol, r0=args.r0, dr=args.r0, r_max=args.r_max, prec="f32",
                             cap_policy=args.cap_policy)
        t0 = time.perf_counter()
        r32, _, t_fit32 = step(o32)
        fp32 = {"fit_s": t_fit32 - t0, "phases": r32.info["phases"], "t_sample_ms": r32.info["hss"]["t_sample_ms"],
                "refine_iterations": r32.info["refine"]["iterations"],
                "relres": r32.info["refine"]["relres"][0], "r_final": r32.info["hss"]["r_final"]}
        fp32["relres_fp64"] = fp64_relres(krr, r32, y, p)
        log(f"fp32 fit: {fp32}")
        del r32

    # the two hot kernels, each timed with HIP events on the stream it runs on
    n = args.n
    r = hs["r_final"]
    R = krr.random_block(1, n, r)
    Xp = res.Xp
    lb, le = leaf_arrays(res.tree.nodes, n, dev)
    log("timing the sampling product")
    t_sample = time_launches(lambda: krr.kernel_sample(Xp, p.h, R, lb, le, prec=args.prec, split_terms=args.split),
                             args.reps)
    flops = float(n) * n * (2 * p.d + 2 * r)
    achieved = flops / t_sample
    peak = PEAK[args.prec if args.prec in PEAK else "f16"]
    roof_sample = {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                   "frac": achieved / peak, "traffic": pmc_traffic("sampling", n, r),
                   "kernel": "k_sample_mfma (sampling product S = K R)",
                   "launch_s": t_sample, "algorithmic_flops": flops,
                   "flops_basis": "n^2 (2d + 2r): one distance dot product and one row of K R per kernel entry"}
    roof_sample.update(pmc_mfma("sampling", n, r, t_sample))
    # the same launch with every tile evaluated (no entry dropped): the
    # kernel's efficiency on full tiles
    krr.set_tuning("sample_skip", 0)
    t_full = time_launches(lambda: krr.kernel_sample(Xp, p.h, R, lb, le, prec=args.prec, split_terms=args.split),
                           args.reps)
    krr.set_tuning("sample_skip", 1)
    roof_sample["every_tile"] = {"launch_s": t_full, "achieved": flops / t_full / 1e12, "frac": flops / t_full / peak}
    roof_sample["every_tile"].update(pmc_mfma("sampling_every_tile", n, r, t_full))
    del R
    # the metric's second sample width: one pass at r = 2 r0 (same points and
    # tree, tile skip on as in the fit)
    r2 = 2 * args.r0
    R2 = krr.random_block(1, n, r2)
    log(f"timing the sampling product at r = {r2}")
    t_r2 = time_launches(lambda: krr.kernel_sample(Xp, p.h, R2, lb, le, prec=args.prec, split_terms=args.split),
                         args.reps)
    flops2 = float(n) * n * (2 * p.d + 2 * r2)
    roof_sample["wider_sample"] = {"r": r2, "launch_s": t_r2, "achieved": flops2 / t_r2 / 1e12,
                                   "frac": flops2 / t_r2 / peak}
    del R2
    w = res.alpha_perm.reshape(n, -1)[:, :1].contiguous()
    log("timing the refinement kernel product (every entry)")
    t_mv = time_launches(lambda: krr.kernel_matvec(Xp, Xp, p.h, w, prec="f32"), args.reps)
    # The symmetric product evaluates each off-diagonal entry once and the
    # diagonal row blocks (512 rows at d <= 9, 8 waves x 4 row tiles x 16) in
    # full; the unit of work is an evaluated entry (2d + 2 flops for its
    # exponent, one exp2), priced against the FP32 vector peak, with the exp2
    # issue floor of the same entries beside it.
    rb = 512 if p.d <= 9 else 256
    evaluated = n * rb + (float(n) * n - n * rb) / 2
    mv_flops = evaluated * (2 * p.d + 2)
    every_entry = {"launch_s": t_mv, "achieved": mv_flops / t_mv / 1e12, "frac": mv_flops / t_mv / PEAK_F32_VECTOR,
                   "traffic": pmc_traffic("kernel_product", n),
                   "evaluated_entries": evaluated, "algorithmic_flops": mv_flops,
                   "entries_per_s": evaluated / t_mv, "exp2_floor_frac": evaluated / PEAK_EXP2 / t_mv}
    every_entry.update(pmc_mfma("kernel_product", n, None, t_mv))
    # The refinement's products after its first: through the tile map that
    # the first one recorded (tiles whose entries are all below 2^-32 left
    # out).  Evaluated entries: the diagonal blocks plus the kept tiles.
    log("timing the refinement kernel product through its tile map")
    tmap = krr.TileMap()
    tmap.matvec(Xp, p.h, w)  # records the map (every entry evaluated)
    kept, tiles, per_tile = tmap.counts()
    t_map = time_launches(lambda: tmap.matvec(Xp, p.h, w), args.reps)
    del tmap
    rb_map = per_tile // 16 * 8 if per_tile else rb  # rows of the map's row blocks (8 waves)
    evaluated_map = n * rb_map + float(kept) * per_tile
    map_flops = evaluated_map * (2 * p.d + 2)
    form = krr.get_tuning("symmetric")
    mapped = form == 4 and p.d <= 31 and kept > 0
    mv_kernel = {4: "k_kmv_symb (refinement product K w over K's upper triangle: FP32-accurate exponents from "
                    "three-term BF16 splits on the matrix cores, re-centred per row block, FP32 entries; "
                    "through the negligible-tile map the refinement's first product records; timed with its "
                    "diagonal-block, anchor and reduction launches)",
                 3: "k_kmv_symf (refinement product K w over K's upper triangle: FP32 exponents on the matrix "
                    "cores, re-centred per row block, FP32 entries; timed with its diagonal-block, anchor and "
                    "reduction launches)"}.get(form, "k_kmv_sym (refinement product K w over K's upper triangle, "
                                                    "FP64 exponent, FP32 entries; timed with its diagonal-block "
                                                    "and reduction launches)")
    if mapped:
        t_use, ev_use, fl_use = t_map, evaluated_map, map_flops
        basis = (f"(2d + 2) flops per evaluated kernel entry; evaluated entries = n x {rb_map} (the {rb_map}-row "
                 f"diagonal blocks) + the tile map's kept wave tiles x their entries ({per_tile // 16} rows x 16 "
                 "points)")
    else:
        t_use, ev_use, fl_use = t_mv, evaluated, mv_flops
        basis = (f"(2d + 2) flops per evaluated kernel entry; evaluated entries = n x {rb} + "
                 f"(n^2 - n x {rb}) / 2 (upper triangle plus full {rb}-row diagonal blocks)")
    roof_mv = {"bound": "alu", "achieved": fl_use / t_use / 1e12, "peak": PEAK_F32_VECTOR / 1e12,
               "unit": "TFLOP/s", "frac": fl_use / t_use / PEAK_F32_VECTOR,
               "traffic": pmc_traffic("kernel_product_mapped" if mapped else "kernel_product", n),
               "kernel": mv_kernel, "launch_s": t_use,
               "peak_basis": "FP32 vector peak 157.3 TFLOP/s (256 CU x 128 lanes x 2 flops x 2.4 GHz)",
               "flops_basis": basis,
               "evaluated_entries": ev_use, "evaluated_entries_frac": ev_use / (float(n) * n),
               "tile_map": {"kept_tiles": kept, "tiles": tiles, "entries_per_tile": per_tile},
               "algorithmic_flops": fl_use, "entries_per_s": ev_use / t_use,
               "exp2_floor_frac": ev_use / PEAK_EXP2 / t_use,
               "exp2_floor_basis": "one exp2 per evaluated entry at 256 CU x 64 lanes x 2.4 GHz / 4 = "
                                   "9.83e12 exp2/s",
               "every_entry": every_entry}
    roof_mv.update(pmc_mfma("kernel_product_mapped" if mapped else "kernel_product", n, None, t_use))
    relres_fp64 = fp64_relres(krr, res, y, p)
    log(f"FP64 relative residual of the fitted coefficients: {relres_fp64:.3e}")
    log(f"sampling {t_sample * 1e3:.1f} ms ({achieved / 1e12:.1f} TFLOP/s); "
        f"kernel product {t_mv * 1e3:.1f} ms ({mv_flops / t_mv / 1e12:.1f} TFLOP/s evaluated), through its tile map "
        f"{t_map * 1e3:.1f} ms ({map_flops / t_map / 1e12:.1f} TFLOP/s evaluated, {kept} of {tiles} tiles)")
    if args.dump_alpha:
        os.makedirs(args.dump_alpha, exist_ok=True)
        np.save(os.path.join(args.dump_alpha, "alpha_sixteen_gaussians.npy"), res.alpha.cpu().numpy())
    # the step's dominant kernel: the one whose phase takes longer
    ph = res.info["phases"]
    mv_dominant = ph.get("refine", 0.0) > ph.get("compress", 0.0)
    roofline = roof_mv if mv_dominant else roof_sample
    cert = {"r_final": hs["r_final"], "iterations": rf["iterations"]}
    del res

    batched = None if args.no_batched else batched_leg()
    grad = None if args.no_grad else grad_leg()
    image = None if args.no_image else image_leg(args.dump_alpha)
    cpu = None if args.no_cpu else cpu_baseline(p, cert)

    out = {
        "metric": "KRR fit s at n=1M d=8: mixed vs FP32 HSS at equal acc; sample TFLOP/s",
        "value": float(np.median(fit_times)),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{args.prec}-split{args.split}/f32/f64",
        "data": "synthetic",
        "config": {"workload": f"sixteen_gaussians n={n} d={p.d} h={p.h} lambda={p.lam} leaf={p.leaf} "
                               f"rtol={args.rtol} atol={args.atol} r0={args.r0} dr={args.r0} r_max={args.r_max} "
                               f"cap_policy={args.cap_policy} test_m={args.m}",
                   "sampling": args.prec, "split_terms": args.split, "r0": args.r0, "r_max": args.r_max,
                   "cap_policy": args.cap_policy, "autotuned": tune_cache is not None},
        "fit_s_min": float(np.min(fit_times)),
        "phases_s": ph,
        "fp32": fp32,
        "sample_tflops": achieved / 1e12,
        "relres": rf["relres"][0],
        "relres_fp64": relres_fp64,
        "refine_iterations": rf["iterations"],
        "accuracy": acc,
        "hss": {k: hs[k] for k in ("r_final", "regrowths", "max_rank", "levels", "bytes_paper",
                                   "t_sample_ms", "t_id_ms", "t_total_ms")},
        "roofline": roofline,
        "roofline_sampling": roof_sample,
        "roofline_kernel_product": roof_mv,
        "batched": batched,
        "gradient": grad,
        "image_like": image,
        "cpu_baseline": cpu,
        "fit_s_all": [float(t) for t in fit_times],
        "environment": run_environment(),
    }
    print(json.dumps(out), flush=True)


def run_environment():
    """What the run was measured on: device, ROCm and torch versions, the
    GPU clocks amd-smi reports (when it is there) and a hash of the library
    sources (the box has no git history)."""
    import hashlib
    import subprocess

    import torch
    env = {"device": torch.cuda.get_device_name(0), "torch": torch.__version__, "hip": torch.version.hip}
    try:
        with open("/opt/rocm/.info/version") as f:
            env["rocm"] = f.read().strip()
    except OSError:
        env["rocm"] = None
    try:
        r = subprocess.run(["amd-smi", "metric", "--clock", "-g", "0"], capture_output=True, text=True, timeout=20)
        lines = [l.strip() for l in r.stdout.splitlines() if "CLK" in l or "MHZ" in l.upper()]
        env["amd_smi_clock"] = lines[:12] if r.returncode == 0 else None
    except (OSError, subprocess.SubprocessError):
        env["amd_smi_clock"] = None
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1803_10274_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    env["sources_sha256"] = h.hexdigest()
    return env


def batched_leg():
    """64 ragged problems (n log-uniform in [2048, 32768], d in {8, 18, 54},
    per-problem h and lambda): one batched fit per dimension group, mixed
    sampling, refinement to 1e-6 on every problem."""
    import numpy as np
    import torch

    import paper_1803_10274_amd as krr
    import synthdata as sd
    ps = sd.c4_ragged_batch()
    probs = [(torch.from_numpy(q.X).cuda(), torch.from_numpy(q.y).cuda(), q.h, q.lam) for q in ps]
    opts = krr.HssOptions(rtol=1e-2, atol=1.0, r0=256, dr=256, r_max=256, prec="f16", cap_policy=1)
    torch.cuda.synchronize()
    krr.fit_batched(probs[:4], leaf=128, opts=opts, tol=1e-6, max_iter=300, raise_on_fail=False)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = krr.fit_batched(probs, leaf=128, opts=opts, tol=1e-6, max_iter=300, raise_on_fail=False)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    worst = max(float(np.max(rf["relres"])) for rf in res.info["refine"])
    out = {"workload": "64 ragged problems, n log-uniform in [2048, 32768], d in {8, 18, 54}",
           "sum_n": int(sum(q.X.shape[0] for q in ps)), "fit_s": t, "phases_s": res.info["phases"],
           "groups": len(res.groups), "refine_iterations": [rf["iterations"] for rf in res.info["refine"]],
           "worst_relres": worst}
    log(f"batched: {out}")
    return out


def grad_leg():
    """Validation-loss value and gradient in (log h, log lambda) at n = 131,072,
    d = 18, 16,384 validation points (forward fit + adjoint solve)."""
    import torch

    import paper_1803_10274_amd as krr
    from paper_1803_10274_amd import autograd as kag
    import synthdata as sd
    p = sd.c5_eight_gaussians()
    X, y = torch.from_numpy(p.X).cuda(), torch.from_numpy(p.y).cuda()
    Xv, yv = torch.from_numpy(p.Xt).cuda(), torch.from_numpy(p.yt).cuda()

    def once(state=None):
        lh = torch.tensor(math.log(p.h), dtype=torch.float64, device="cuda", requires_grad=True)
        ll = torch.tensor(math.log(p.lam), dtype=torch.float64, device="cuda", requires_grad=True)
        L, st = kag.validation_loss(lh, ll, X, y, Xv, yv, leaf=p.leaf, state=state)
        L.backward()
        torch.cuda.synchronize()
        return L, lh.grad, ll.grad, st

    _, _, _, st = once()
    t0 = time.perf_counter()
    L, gh, gl, _ = once(st)
    t = time.perf_counter() - t0
    out = {"workload": f"eight_gaussians n={p.X.shape[0]} d={p.d} m_v={p.Xt.shape[0]} h={p.h} lambda={p.lam}",
           "loss_and_grad_s": t, "loss": float(L.detach()), "dL_dlogh": float(gh), "dL_dloglam": float(gl)}
    log(f"gradient: {out}")
    return out


def image_leg(dump=None):
    """The image-like workload at full size (n = 60,000, d = 784, ten
    one-vs-all right-hand sides): FP16 2-term sampling on the matrix cores
    (wide-point GEMM kernel), mixed-precision refinement (FP32-entry products,
    FP64 residuals) to 1e-6, one-vs-all accuracy on 10,000 test points."""
    import numpy as np
    import torch

    import paper_1803_10274_amd as krr
    import synthdata as sd
    p = sd.c3_image_like()
    X = torch.from_numpy(p.X).cuda()
    Y = torch.from_numpy(np.ascontiguousarray(p.y)).cuda()
    opts = krr.HssOptions(rtol=1e-2, atol=0.0, r0=256, dr=256, r_max=1024, prec="f16", cap_policy=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = krr.fit(X, Y, p.h, p.lam, leaf=p.leaf, opts=opts, tol=1e-6, max_iter=300, raise_on_fail=False,
                  res_prec="f64")
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    _, lab = krr.predict(torch.from_numpy(p.Xt).cuda(), res.Xp, p.h, res.alpha_perm)
    if dump:
        os.makedirs(dump, exist_ok=True)
        np.save(os.path.join(dump, "alpha_image_like.npy"), res.alpha.cpu().numpy())
    out = {"workload": f"image_like n={p.n} d={p.d} classes=10 h={p.h} lambda={p.lam}", "fit_s": t,
           "phases_s": res.info["phases"], "refine_iterations": res.info["refine"]["iterations"],
           "relres_fp64_max": float(max(res.info["refine"]["relres"])),
           "t_sample_ms": res.info["hss"]["t_sample_ms"],
           "accuracy": float((lab.cpu().numpy() == p.yt).mean())}
    log(f"image-like: {out}")
    return out


def cpu_dense():
    """The oracle's dense FP64 KRR fit (Algorithm 1 steps 1-2: form K from
    the differences, Cholesky, solve) on the host, on the first n points of
    the sixteen-Gaussian workload: one thread and all threads at n = 1,000 and
    8,192 (SciPy LAPACK), all threads at n = 32,768 (torch's CPU Cholesky: the
    SciPy build fails to factor that size).  One JSON line per case."""
    import numpy as np
    import torch

    import synthdata as sd
    from oracle import kernel as ok
    cores, nproc, model = cpu_info()
    p = sd.c2_sixteen_gaussians(n=32768, m=1)
    from threadpoolctl import threadpool_limits
    for n, threads in ((1000, 1), (1000, cores), (8192, 1), (8192, cores), (32768, cores)):
        torch.set_num_threads(threads)
        X = p.X[:n].astype(np.float64)
        y = np.asarray(p.y[:n], dtype=np.float64)
        log(f"cpu dense: n = {n}, {threads} threads")
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            K = ok.kernel_dense(X, X, p.h)
            t1 = time.perf_counter()
            if n <= 8192:
                ok.krr_solve_dense(K, y, p.lam)
            else:
                K[np.diag_indices_from(K)] += p.lam
                L = torch.linalg.cholesky(torch.from_numpy(K))
                torch.cholesky_solve(torch.from_numpy(y).reshape(-1, 1), L)
                del L
            t2 = time.perf_counter()
        del K
        print(json.dumps({"cpu_dense": True, "n": n, "threads": threads, "form_s": t1 - t0, "solve_s": t2 - t1,
                          "nproc": nproc, "cpu_model": model}), flush=True)


def cpu_info():
    """Host cores this process may use, and the CPU model."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    # the oracle's OpenMP loops use at most OMP_NUM_THREADS threads
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        cores = min(cores, int(os.environ["OMP_NUM_THREADS"]))
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return cores, os.cpu_count(), model


def cpu_baseline(p, cert):
    """The oracle timed on the host on bounded samples of the headline
    workload, extrapolated (labelled as such) to the GPU fit's dominant work:
      - the 2MN clustering of all n points, single-threaded (measured in full);
      - the FP64 matrix-free product K w (all host cores) on 2048 rows x all n
        columns, extrapolated linearly in rows to one full product;
      - the sampling pass S = K R with r columns (all host cores) on 64 rows x
        all n columns, extrapolated linearly in rows to the whole pass.
    value = clustering + one sampling pass + one product per refinement
    iteration of the GPU fit (the same algorithm's dominant work, in seconds)."""
    import numpy as np

    import synthdata as sd
    from oracle import cluster as oc, cmath
    cores, nproc, model = cpu_info()
    log("cpu baseline: oracle 2MN")
    t0 = time.perf_counter()
    tree = oc.cluster2mn(p.X, p.leaf, 7)
    t_cluster = time.perf_counter() - t0
    Xp = np.ascontiguousarray(p.X[tree.perm], dtype=np.float64)
    n = p.n
    rows = np.arange(0, n, n // 2048)[:2048]
    w = sd.vectors(n, 1, seed=3)
    log("cpu baseline: oracle FP64 kernel product rows")
    t0 = time.perf_counter()
    cmath.kmv(Xp, Xp, w, p.h, rows=rows)
    t_rows = time.perf_counter() - t0
    t_product = t_rows * n / rows.shape[0]
    r = cert["r_final"]
    srows = np.arange(0, n, n // 64)[:64]
    R = sd.random_block(n, r, seed=1)
    lb, le = tree.leaf_ranges_per_point()
    log("cpu baseline: oracle sampling rows")
    t0 = time.perf_counter()
    cmath.sample_masked(Xp, R, p.h, lb, le, srows)
    t_srows = time.perf_counter() - t0
    t_pass = t_srows * n / srows.shape[0]
    iters = int(cert["iterations"])
    value = t_cluster + t_pass + iters * t_product
    return {"value": value, "unit": "s", "cores": cores, "kind": "oracle",
            "sample": f"oracle 2MN of all {n} points (1 thread, measured {t_cluster:.1f} s); FP64 matrix-free "
                      f"K w on {rows.shape[0]} rows x {n} columns ({cores} threads, {t_rows:.2f} s, extrapolated "
                      f"to {t_product:.0f} s per product); FP64 sample K R, r = {r}, on {srows.shape[0]} rows "
                      f"({cores} threads, {t_srows:.2f} s, extrapolated to {t_pass:.0f} s per pass); value = "
                      f"clustering + one pass + {iters} products (the GPU fit's refinement iterations), "
                      "extrapolated",
            "cluster_s": t_cluster, "product_s_extrapolated": t_product, "sampling_pass_s_extrapolated": t_pass,
            "product_entries_per_s": rows.shape[0] * float(n) / t_rows,
            "nproc": nproc, "cpu_model": model}


if __name__ == "__main__":
    main()
