"""Benchmark: Gaussian-kernel ridge regression fit at n = 2^20, d = 8.

One step = one pass of the whole hot path on the sixteen-Gaussian workload
(n = 1,048,576 training points, d = 8, h = 0.75, lambda = 10, 100,000 test
points, synthetic data): 2MN clustering, permutation, HSS compression with
mixed-precision sampling (FP16 hi/lo split entries, FP32 accumulation), FP64
IDs and ULV factorization, solve, PCG refinement on the FP32 kernel product to
a relative residual of 1e-6, un-permutation, and prediction of the test set.

Reported: the fit time of the mixed path (value, seconds, lower is better),
the same fit with FP32 sampling (`fp32_fit_s`), the sampling kernel's
throughput against the matrix-core roofline (measured with HIP events on the
stream it runs on), and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f16": 2.5e15, "bf16": 2.5e15, "f32": 157.3e12, "f64": 78.6e12}


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
    ap.add_argument("--atol", type=float, default=3.0)
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-sampling comparison fit")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--sample-reps", type=int, default=3)
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
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
    opts = krr.HssOptions(rtol=args.rtol, atol=args.atol, r0=args.r0, dr=args.r0, r_max=args.r0, prec=args.prec,
                          split_terms=args.split, cap_policy=1)

    def step(o):
        res = krr.fit(X, y, p.h, p.lam, leaf=p.leaf, opts=o, tol=1e-6, max_iter=300, raise_on_fail=False)
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
        o32 = krr.HssOptions(rtol=args.rtol, atol=args.atol, r0=args.r0, dr=args.r0, r_max=args.r0, prec="f32",
                             cap_policy=1)
        t0 = time.perf_counter()
        r32, _, t_fit32 = step(o32)
        fp32 = {"fit_s": t_fit32 - t0, "phases": r32.info["phases"], "t_sample_ms": r32.info["hss"]["t_sample_ms"],
                "refine_iterations": r32.info["refine"]["iterations"],
                "relres": r32.info["refine"]["relres"][0], "r_final": r32.info["hss"]["r_final"]}
        log(f"fp32 fit: {fp32}")
        del r32

    # dominant kernel: the sampling product, timed with HIP events on the current stream
    r = hs["r_final"]
    R = krr.random_block(1, args.n, r)
    Xp = res.Xp
    lb = torch.empty(args.n, dtype=torch.int32, device=dev)
    le = torch.empty(args.n, dtype=torch.int32, device=dev)
    nodes = res.tree.nodes
    leaves = nodes[nodes[:, 2] < 0]
    lbn = np.empty(args.n, dtype=np.int32)
    len_ = np.empty(args.n, dtype=np.int32)
    for b, e in leaves[:, :2]:
        lbn[b:e] = b
        len_[b:e] = e
    lb.copy_(torch.from_numpy(lbn))
    le.copy_(torch.from_numpy(len_))
    krr.kernel_sample(Xp, p.h, R, lb, le, prec=args.prec, split_terms=args.split)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.sample_reps):
        krr.kernel_sample(Xp, p.h, R, lb, le, prec=args.prec, split_terms=args.split)
    e1.record(stream)
    e1.synchronize()
    t_sample = e0.elapsed_time(e1) / 1e3 / args.sample_reps
    n = args.n
    flops = float(n) * n * (2 * p.d + 2 * r)
    achieved = flops / t_sample
    peak = PEAK[args.prec if args.prec in PEAK else "f16"]
    roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None, "kernel": "sampling product",
                "launch_s": t_sample, "algorithmic_flops": flops}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(p)

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
                               f"rtol={args.rtol} atol={args.atol} r={args.r0} test_m={args.m}",
                   "sampling": args.prec, "split_terms": args.split},
        "fit_s_min": float(np.min(fit_times)),
        "phases_s": res.info["phases"],
        "ulv_shift": res.info["ulv_shift"],
        "fp32": fp32,
        "sample_tflops": achieved / 1e12,
        "relres": rf["relres"][0],
        "refine_iterations": rf["iterations"],
        "accuracy": acc,
        "hss": {k: hs[k] for k in ("r_final", "regrowths", "max_rank", "levels", "bytes_paper",
                                   "t_sample_ms", "t_id_ms", "t_total_ms")},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(p):
    """The oracle on a bounded sample: dense FP64 KRR (form K, Cholesky, solve)
    at n_s = 4096 points of the same workload, timed on the host, scaled to
    n = 2^20 by the O(n^3) Cholesky cost (and its O(n^2) forming cost)."""
    import numpy as np

    from oracle import kernel as ok
    n_s = 4096
    Xs = p.X[:n_s].astype(np.float64)
    ys = p.y[:n_s]
    t0 = time.perf_counter()
    K = ok.kernel_dense(Xs, Xs, p.h)
    t1 = time.perf_counter()
    ok.krr_solve_dense(K, ys, p.lam)
    t2 = time.perf_counter()
    scale = p.n / n_s
    est = (t1 - t0) * scale ** 2 + (t2 - t1) * scale ** 3
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return {"value": est, "unit": "s", "cores": cores, "kind": "oracle",
            "sample": f"dense FP64 KRR fit (kernel_dense + Cholesky) on the first {n_s} points, "
                      f"measured form {t1 - t0:.2f} s + solve {t2 - t1:.2f} s, scaled to n={p.n} by "
                      "n^2 (forming) and n^3 (Cholesky)"}


if __name__ == "__main__":
    main()
