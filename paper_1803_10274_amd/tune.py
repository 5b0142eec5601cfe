"""Launch-shape autotuner for the hot kernels, with a JSON cache.

The library exposes a few process-wide launch knobs (include/krr.h,
KRR_TUNE_*): the number of 32-column blocks per pass of the sampling product,
the workgroup count the split-K kernel product aims for, and the column chunk
of the symmetric kernel product (plus the switch for that product).  None of
them changes results beyond floating-point summation order.  `autotune` times
the candidates on synthetic points of the caller's shape with HIP events and
stores the fastest per key (arch, padded width, sample width, precision) in a
JSON file; `apply` sets the knobs from that file before a fit.

Only the timing loop lives here; every launch is a libkrr kernel.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import get_tuning, kernel_matvec, kernel_sample, random_block, set_tuning

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "krr_hss", "tune.json")

CANDIDATES = {
    "sample_rb": [8, 4, 2],
    "mv_blocks": [1024, 2048, 4096],
    "sym_chunk": [4096, 8192, 16384, 32768],
}


def _width(d: int) -> int:
    """The padded point width the kernels are instantiated for."""
    for w in (4, 8, 12, 16, 20, 24, 32, 48, 56, 64):
        if d <= w:
            return w
    return d


def cache_key(d: int, r: int, prec: str) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "none"
    return f"{arch}/d{_width(d)}/r{r}/{prec}"


def _load(path):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _time(fn, reps):
    fn()
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(reps):
        fn()
    b.record(s)
    b.synchronize()
    return a.elapsed_time(b) / reps


def autotune(d: int, r: int = 256, prec: str = "f16", n: int = 1 << 17, split_terms: int = 2, reps: int = 3,
             path: str = DEFAULT_CACHE, seed: int = 0) -> dict:
    """Time each knob's candidates (the others at their current values) on n
    synthetic points of width d and record the fastest under cache_key."""
    rng = np.random.default_rng(seed)
    X = torch.from_numpy(rng.standard_normal((n, d)).astype(np.float32)).cuda()
    h = float(np.sqrt(d))
    R = random_block(seed + 1, n, r)
    w = torch.from_numpy(rng.standard_normal((n, 1))).cuda()
    chosen, timings = {}, {}
    saved = {k: get_tuning(k) for k in CANDIDATES}
    try:
        runs = {
            "sample_rb": lambda: kernel_sample(X, h, R, prec=prec, split_terms=split_terms),
            "mv_blocks": lambda: kernel_matvec(X, X.clone(), h, w, prec="f32"),  # the split-K (non-symmetric) form
            "sym_chunk": lambda: kernel_matvec(X, X, h, w, prec="f32"),
        }
        for knob, values in CANDIDATES.items():
            t = {}
            for v in values:
                set_tuning(knob, v)
                t[v] = _time(runs[knob], reps)
            best = min(t, key=t.get)
            set_tuning(knob, best)
            chosen[knob] = best
            timings[knob] = {str(k): v for k, v in t.items()}
    except Exception:
        for k, v in saved.items():
            set_tuning(k, v)
        raise
    entry = {"knobs": chosen, "ms": timings, "n": n}
    db = _load(path)
    db[cache_key(d, r, prec)] = entry
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return entry


def apply(d: int, r: int = 256, prec: str = "f16", path: str = DEFAULT_CACHE) -> dict | None:
    """Set the knobs recorded for this shape, if any; returns them."""
    entry = _load(path).get(cache_key(d, r, prec))
    if entry is None:
        return None
    for knob, value in entry["knobs"].items():
        set_tuning(knob, value)
    return entry["knobs"]
