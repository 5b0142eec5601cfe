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


def _bad_calls(L, _lib):
    """One invalid call per entry point: (name, thunk, message fragment).  Every
    pointer the library only tests for NULL is a fake non-NULL address; host
    arrays it reads (offsets, h, lambda, options, tree tables) are real."""
    import numpy as np
    P = ctypes.c_void_p(64)  # never dereferenced before the device check
    i64p = ctypes.POINTER(ctypes.c_int64)
    dblp = ctypes.POINTER(ctypes.c_double)
    keep = []

    def arr(a, dt, ptr):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data_as(ptr)

    nodes = np.array([[0, 5, -1, -1, 2], [5, 10, -1, -1, 2], [0, 10, 0, 1, -1]], dtype=np.int64)
    tree = ctypes.c_void_p()
    assert L.krr_tree_from_host(nodes.ctypes.data_as(ctypes.c_void_p), 3, ctypes.byref(tree)) == 0
    keep.append(tree)
    good = _lib.HssOpts(1e-2, 0.0, 64, 32, 256, 10, _lib.KRR_F64, 1, 0, 1)
    bad_r0 = _lib.HssOpts(1e-2, 0.0, 40, 32, 256, 10, _lib.KRR_F64, 1, 0, 1)
    out = ctypes.c_void_p(99)
    copts = _lib.ClusterOpts(16, 100, 1)
    F32, F64 = _lib.KRR_F32, _lib.KRR_F64
    off_empty = arr([0, 5, 5], np.int64, i64p)
    off_bad0 = arr([1, 5], np.int64, i64p)
    off_ok = arr([0, 5], np.int64, i64p)
    h_neg = arr([-1.0], np.float64, dblp)
    h_ok = arr([1.0], np.float64, dblp)
    return keep, tree, out, [
        ("krr_gather_rows", lambda: L.krr_gather_rows(P, F32, 4, 0, P, P, None), "bad sizes"),
        ("krr_scatter_rows", lambda: L.krr_scatter_rows(P, F32, -1, 2, P, P, None), "bad sizes"),
        ("kernel_sample r", lambda: L.kernel_sample(P, 10, 3, F32, 1.0, P, 48, None, None, P, F32, 1, None),
         "multiple of 32"),
        ("kernel_sample leaf", lambda: L.kernel_sample(P, 10, 3, F32, 1.0, P, 32, P, None, P, F32, 1, None),
         "both leaf arrays"),
        ("krr_random_block", lambda: L.krr_random_block(1, -1, 4, 0, P, None), "bad arguments"),
        ("kernel_matvec_bwd", lambda: L.kernel_matvec_bwd(P, 3, P, 4, 2, F32, 0.0, P, P, 1, P, P, P, P, F32, None),
         "h must be positive"),
        ("hss_compress", lambda: L.hss_compress(tree, P, F64, 2, 1.0, ctypes.byref(bad_r0), None, ctypes.byref(out),
                                                None), "r0"),
        ("hss_matvec", lambda: L.hss_matvec(None, P, 1, P, None), "bad arguments"),
        ("hss_export_sizes", lambda: L.hss_export_sizes(None, None, None, None), "NULL handle"),
        ("hss_export", lambda: L.hss_export(None, P, P, P, None), "NULL argument"),
        ("hss_ulv_factor_spd", lambda: L.hss_ulv_factor_spd(P, 1.0, 0.0, None, ctypes.byref(out), None),
         "pivot_floor"),
        ("hss_ulv_factor_shifted", lambda: L.hss_ulv_factor_shifted(P, 0.0, None, ctypes.byref(out), None),
         "lambda must be > 0"),
        ("hss_ulv_use_graph", lambda: L.hss_ulv_use_graph(None, 1), "NULL factor"),
        ("hss_solve", lambda: L.hss_solve(P, P, 0, P, None), "nrhs"),
        ("krr_refine", lambda: L.krr_refine(None, P, 10, F32, 2, 1.0, 1.0, P, 1, P, 1e-6, 10, 7, F64, None, None),
         "mv_prec"),
        ("krr_predict", lambda: L.krr_predict(P, 3, P, 4, 2, F32, 1.0, P, 65, P, P, F32, None), "bad sizes"),
        ("krr_set_tuning knob", lambda: L.krr_set_tuning(99, 1), "unknown knob"),
        ("krr_set_tuning value", lambda: L.krr_set_tuning(0, 5), "0 to 4"),
        ("krr_set_tuning sym skip", lambda: L.krr_set_tuning(_lib.KRR_TUNE_SYM_SKIP, 3), "0, 1 or 2"),
        ("krr_tile_map_create", lambda: L.krr_tile_map_create(None), "NULL pointer"),
        ("krr_tile_map_destroy", lambda: L.krr_tile_map_destroy(None), "NULL handle"),
        ("kernel_matvec_mapped", lambda: L.kernel_matvec_mapped(P, 10, 3, F32, 1.0, P, 1, 0.0, P, None, None),
         "NULL map"),
        ("krr_tile_map_counts", lambda: L.krr_tile_map_counts(None, None, None), "NULL pointer"),
        ("krr_get_tuning", lambda: L.krr_get_tuning(0, None), "bad arguments"),
        ("krr_dot_columns", lambda: L.krr_dot_columns(P, P, 5, 0, P, None), "bad arguments"),
        ("krr_tree_size", lambda: L.krr_tree_size(None, None, None), "NULL tree"),
        ("krr_tree_export", lambda: L.krr_tree_export(None, None, None), "NULL tree"),
        ("krr_tree_roots", lambda: L.krr_tree_roots(None, None, None), "NULL tree"),
        ("krr_cluster_2mn_batched", lambda: L.krr_cluster_2mn_batched(P, F32, off_empty, 2, 3, ctypes.byref(copts),
                                                                      None, P, ctypes.byref(out)), "problem 1 is empty"),
        ("hss_compress_batched", lambda: L.hss_compress_batched(tree, P, F64, 2, h_neg, ctypes.byref(good), None,
                                                                ctypes.byref(out), None), "h[0] must be > 0"),
        ("hss_num_problems", lambda: L.hss_num_problems(None, None), "NULL argument"),
        ("hss_ulv_factor_batched", lambda: L.hss_ulv_factor_batched(P, None, 0, None, ctypes.byref(out), None),
         "NULL argument"),
        ("kernel_sample_batched", lambda: L.kernel_sample_batched(P, F32, off_bad0, 1, 3, h_ok, P, 32, None, None, P,
                                                                  F32, 1, None), "offsets[0] must be 0"),
        ("kernel_matvec_batched", lambda: L.kernel_matvec_batched(P, F32, off_ok, 1, 3, h_neg, P, 1, P, F32, None),
         "h[0] must be positive"),
        ("krr_refine_batched", lambda: L.krr_refine_batched(None, P, F32, off_ok, 1, 3, h_ok, None, P, 1, P, 1e-6, 10,
                                                            F32, F64, None, None, None), "NULL lambda"),
        ("krr_cluster_order method", lambda: L.krr_cluster_order(P, F32, 10, 2, 7, None, 0, ctypes.byref(copts), None,
                                                                 P, ctypes.byref(out)), "unknown method"),
        ("krr_cluster_order offsets", lambda: L.krr_cluster_order(P, F32, 10, 2, 2, off_ok, 1, ctypes.byref(copts),
                                                                  None, P, ctypes.byref(out)), "offsets[np]"),
        ("krr_val_residual", lambda: L.krr_val_residual(P, P, 0, 1, P, P, None), "m >= 1"),
        ("krr_set_allocator", lambda: L.krr_set_allocator(P, None, None), "both functions or neither"),
        ("krr_predict_noalloc", lambda: L.krr_predict_noalloc(P, 3, P, 4, 65, F32, 1.0, P, 1, P, P, F32, None),
         "d = 65 > 64"),
        ("krr_alloc_counts", lambda: L.krr_alloc_counts(None, None), "NULL argument"),
        ("krr_val_grad_finish", lambda: L.krr_val_grad_finish(P, P, P, None, 1.0, -1.0, P, None), "positive"),
    ]


def test_every_entry_point_validates_before_device(lib):
    # each call is invalid on the host: the library must answer KRR_E_INVAL
    # with a message naming the fault, before any device call (on a machine
    # without a GPU a late check would answer KRR_E_NODEVICE instead), and
    # leave an out-handle NULL
    from paper_1803_10274_amd import _lib
    L = _lib.load(LIB)
    before = ctypes.c_int()
    assert L.krr_get_tuning(0, ctypes.byref(before)) == 0
    keep, tree, out, calls = _bad_calls(L, _lib)
    try:
        for name, call, frag in calls:
            out.value = 99
            rc = call()
            assert rc == _lib.KRR_E_INVAL, (name, rc, L.krr_last_error())
            assert frag.encode() in L.krr_last_error(), (name, L.krr_last_error())
            if "hss_ulv_factor" in name or "compress" in name or "cluster" in name:
                assert not out.value, name
    finally:
        L.krr_tree_destroy(tree)
    # a rejected tuning value leaves the knob as it was
    after = ctypes.c_int()
    assert L.krr_get_tuning(0, ctypes.byref(after)) == 0 and after.value == before.value
