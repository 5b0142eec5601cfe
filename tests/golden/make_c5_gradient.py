"""Writes c5_gradient_n32768.json: the oracle's dense FP64 validation loss and
its gradient in (log h, log lambda) on the eight-Gaussian gradient workload
reduced to n = 32,768 training and m_v = 4,096 validation points, at its
evaluation point h = 2, lambda = 1 (loss and gradient: adjoint of Algorithm 1
step 2, formulas in oracle/grad.py).  Calls only oracle/ and the seeded input
generator; about 12 GB of memory and a minute or two on 8 cores.

    python tests/golden/make_c5_gradient.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import synthdata as sd  # noqa: E402
from oracle import grad as og  # noqa: E402

N, MV = 32768, 4096


def main():
    p = sd.c5_eight_gaussians(n=N, m=MV)
    t0 = time.perf_counter()
    L, gh, gl = og.val_loss_grad_blocked(p.X.astype(np.float64), p.y, p.Xt.astype(np.float64), p.yt, p.h, p.lam)
    t = time.perf_counter() - t0
    out = {"workload": f"eight_gaussians n={N} m_v={MV} d={p.d} h={p.h} lambda={p.lam}",
           "n": N, "m_v": MV, "h": p.h, "lam": p.lam, "loss": L, "dL_dlogh": gh, "dL_dloglam": gl,
           "source": "oracle.grad.val_loss_grad_blocked (dense FP64 Cholesky)", "seconds": round(t, 1),
           "host_threads": os.cpu_count()}
    with open(os.path.join(HERE, "c5_gradient_n32768.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
