"""Builds and loads the oracle's C part (oracle/c/oracle.c) with plain gcc.

Test infrastructure only (see the package docstring)."""
import ctypes
import os
import subprocess
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "c", "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c -> liboracle.so (FP contraction off, OpenMP on)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            _lib = ctypes.CDLL(build())
            i64, i32, u64, vp, dbl = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                      ctypes.c_void_p, ctypes.c_double)
            _lib.oracle_cluster2mn.restype = i64
            _lib.oracle_cluster2mn.argtypes = [vp, i64, i32, i32, i32, u64, vp, vp, vp]
            _lib.oracle_kmv.restype = None
            _lib.oracle_kmv.argtypes = [vp, vp, i64, i32, dbl, vp, i32, vp, i64, vp]
            _lib.oracle_sample_masked.restype = None
            _lib.oracle_sample_masked.argtypes = [vp, i64, i32, dbl, vp, i32, vp, vp, vp, i64, vp]
            _lib.oracle_order.restype = i64
            _lib.oracle_order.argtypes = [vp, i64, i32, i32, i32, vp, vp, vp]
            _lib.oracle_seeds.restype = ctypes.c_int
            _lib.oracle_seeds.argtypes = [vp, i64, i32, i64, i64, u64, vp, vp]
            _lib.oracle_node_draw.restype = u64
            _lib.oracle_node_draw.argtypes = [u64, i64, i64, u64]
            _lib.oracle_sm_step.restype = u64
            _lib.oracle_sm_step.argtypes = [u64]
            _lib.oracle_isqrt64.restype = u64
            _lib.oracle_isqrt64.argtypes = [u64]
        return _lib
