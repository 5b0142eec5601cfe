"""The C ABI library loads on a machine without a GPU, exports every entry
point include/krr.h declares, and rejects invalid arguments before touching a
device (no compute calls are made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "krr.h")
LIB = os.path.join(ROOT, "paper_1803_10274_amd", "libkrr.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import paper_1803_10274_amd.build as b
        b.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("krr_cluster_2mn", "hss_compress", "hss_ulv_factor", "hss_solve", "kernel_matvec",
                 "kernel_matvec_bwd", "krr_refine", "krr_predict", "hss_export", "krr_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []


def test_binding_declares_every_symbol():
    from paper_1803_10274_amd import _lib
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_validation_before_device(lib):
    from paper_1803_10274_amd import _lib
    L = _lib.load(LIB)
    # nrhs out of range
    rc = L.kernel_matvec(None, 10, None, 10, 3, _lib.KRR_F32, 1.0, None, 0, 0.0, None, _lib.KRR_F32, None)
    assert rc == _lib.KRR_E_INVAL
    assert b"nrhs" in L.krr_last_error()
    # non-positive h
    rc = L.kernel_matvec(None, 10, None, 10, 3, _lib.KRR_F32, -1.0, None, 1, 0.0, None, _lib.KRR_F32, None)
    assert rc == _lib.KRR_E_INVAL
    # NULL out handle
    rc = L.hss_ulv_factor(None, 1.0, None, None)
    assert rc == _lib.KRR_E_INVAL
    # bad point dtype
    opts = _lib.ClusterOpts(16, 100, 1)
    h = ctypes.c_void_p()
    rc = L.krr_cluster_2mn(None, 7, 10, 2, ctypes.byref(opts), None, None, ctypes.byref(h))
    assert rc == _lib.KRR_E_INVAL and not h.value
    # a malformed tree table is rejected on the host
    import numpy as np
    bad = np.array([[0, 5, -1, -1, 2], [5, 10, -1, -1, 2], [0, 9, 0, 1, -1]], dtype=np.int64)
    rc = L.krr_tree_from_host(bad.ctypes.data_as(ctypes.c_void_p), 3, ctypes.byref(h))
    assert rc == _lib.KRR_E_INVAL and b"split" in L.krr_last_error()
    good = np.array([[0, 5, -1, -1, 2], [5, 10, -1, -1, 2], [0, 10, 0, 1, -1]], dtype=np.int64)
    assert L.krr_tree_from_host(good.ctypes.data_as(ctypes.c_void_p), 3, ctypes.byref(h)) == 0
    n, nn = ctypes.c_int64(), ctypes.c_int64()
    assert L.krr_tree_size(h, ctypes.byref(n), ctypes.byref(nn)) == 0 and (n.value, nn.value) == (10, 3)
    L.krr_tree_destroy(h)


def test_no_device_reported(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1803_10274_amd import _lib
    L = _lib.load(LIB)
    assert L.krr_device_count() == 0
    R = ctypes.c_void_p(1)
    assert L.krr_random_block(1, 4, 4, 0, R, None) == _lib.KRR_E_NODEVICE
