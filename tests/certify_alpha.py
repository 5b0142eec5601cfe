"""Certify fitted coefficients written by `bench.py --dump-alpha DIR` with the
oracle's FP64 matrix-free residual over every row (Algorithm 1 step 2: the
coefficients solve (K + lambda I) alpha = y; the residual is that definition
evaluated without forming K).

    python tests/certify_alpha.py DIR

For each dump it regenerates the seeded workload, computes
||y - (K + lambda I) alpha|| / ||y|| per right-hand side with the oracle on all
host threads, and prints one JSON line (relres, time, threads).  Not a pytest
module: at n = 2^20 it is about 10^12 kernel evaluations on the CPU."""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synthdata as sd  # noqa: E402
from oracle import cmath  # noqa: E402

WORKLOADS = {
    "alpha_sixteen_gaussians.npy": lambda: sd.c2_sixteen_gaussians(m=1),
    "alpha_image_like.npy": lambda: sd.c3_image_like(m=1),
}


def certify(path, make):
    p = make()
    alpha = np.load(path)
    y = np.asarray(p.y, dtype=np.float64)
    t0 = time.perf_counter()
    r = cmath.residual(p.X, alpha, y, p.h, p.lam)
    t = time.perf_counter() - t0
    rr = np.linalg.norm(r.reshape(r.shape[0], -1), axis=0) / np.linalg.norm(y.reshape(y.shape[0], -1), axis=0)
    return {"dump": os.path.basename(path), "n": int(p.X.shape[0]), "d": int(p.X.shape[1]),
            "relres_oracle_fp64": [float(v) for v in rr], "max_relres": float(rr.max()),
            "rows": "all", "seconds": t, "threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count())),
            "cpu_count": os.cpu_count()}


def main():
    d = sys.argv[1]
    for name, make in WORKLOADS.items():
        path = os.path.join(d, name)
        if os.path.exists(path):
            print(json.dumps(certify(path, make)), flush=True)


if __name__ == "__main__":
    main()
