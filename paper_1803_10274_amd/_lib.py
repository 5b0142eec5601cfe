"""ctypes declarations of libkrr (include/krr.h).  Loads the in-tree
libkrr.so; there is no fallback: without the library every call raises."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkrr.so")

KRR_OK, KRR_E_INVAL, KRR_E_NOMEM, KRR_E_HIP = 0, -1, -2, -3
KRR_E_RANK_CAP, KRR_E_NUMERIC, KRR_E_NOT_CONVERGED, KRR_E_NODEVICE = -4, -5, -6, -7
KRR_F64, KRR_F32, KRR_F16_SPLIT, KRR_BF16_SPLIT = 0, 1, 2, 3
KRR_TUNE_SYMMETRIC, KRR_TUNE_SAMPLE_RB, KRR_TUNE_MV_BLOCKS, KRR_TUNE_SYM_CHUNK, KRR_TUNE_SAMPLE_SKIP = 0, 1, 2, 3, 4
KRR_TUNE_SYM_SKIP = 5

_CODES = {KRR_E_INVAL: "KRR_E_INVAL", KRR_E_NOMEM: "KRR_E_NOMEM", KRR_E_HIP: "KRR_E_HIP",
          KRR_E_RANK_CAP: "KRR_E_RANK_CAP", KRR_E_NUMERIC: "KRR_E_NUMERIC",
          KRR_E_NOT_CONVERGED: "KRR_E_NOT_CONVERGED", KRR_E_NODEVICE: "KRR_E_NODEVICE"}


class KrrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class ClusterOpts(ctypes.Structure):
    _fields_ = [("leaf_size", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class HssOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("atol", ctypes.c_double), ("r0", ctypes.c_int32),
                ("dr", ctypes.c_int32), ("r_max", ctypes.c_int32), ("oversample", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("split_terms", ctypes.c_int32), ("cap_policy", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class HssStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_nodes", ctypes.c_int64), ("levels", ctypes.c_int64),
                ("r_final", ctypes.c_int32), ("regrowths", ctypes.c_int32), ("max_rank", ctypes.c_int32),
                ("truncated", ctypes.c_int32), ("bytes_paper", ctypes.c_int64), ("bytes_stored", ctypes.c_int64),
                ("t_sample_ms", ctypes.c_double), ("t_id_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class RefineStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("matvecs", ctypes.c_int32),
                ("relres", ctypes.c_double * 64), ("t_ms", ctypes.c_double)]


_vp, _i32, _i64, _u64, _dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
_P = ctypes.POINTER

# name: (restype, argtypes)
SIGNATURES = {
    "krr_last_error": (ctypes.c_char_p, []),
    "krr_device_count": (ctypes.c_int, []),
    "krr_set_allocator": (ctypes.c_int, [_vp, _vp, _vp]),
    "krr_alloc_counts": (ctypes.c_int, [_P(_i64), _P(_i64)]),
    "krr_cluster_2mn": (ctypes.c_int, [_vp, _i32, _i64, _i32, _P(ClusterOpts), _vp, _vp, _P(_vp)]),
    "krr_cluster_order": (ctypes.c_int, [_vp, _i32, _i64, _i32, _i32, _vp, _i32, _P(ClusterOpts), _vp, _vp,
                                         _P(_vp)]),
    "krr_tree_from_host": (ctypes.c_int, [_vp, _i64, _P(_vp)]),
    "krr_val_residual": (ctypes.c_int, [_vp, _vp, _i64, _i32, _vp, _vp, _vp]),
    "krr_val_grad_finish": (ctypes.c_int, [_vp, _vp, _vp, _vp, _dbl, _dbl, _vp, _vp]),
    "krr_tree_size": (ctypes.c_int, [_vp, _P(_i64), _P(_i64)]),
    "krr_tree_export": (ctypes.c_int, [_vp, _vp, _vp]),
    "krr_tree_destroy": (None, [_vp]),
    "krr_gather_rows": (ctypes.c_int, [_vp, _i32, _i64, _i32, _vp, _vp, _vp]),
    "krr_scatter_rows": (ctypes.c_int, [_vp, _i32, _i64, _i32, _vp, _vp, _vp]),
    "kernel_matvec": (ctypes.c_int, [_vp, _i64, _vp, _i64, _i32, _i32, _dbl, _vp, _i32, _dbl, _vp, _i32, _vp]),
    "krr_tile_map_create": (ctypes.c_int, [_P(_vp)]),
    "krr_tile_map_destroy": (ctypes.c_int, [_vp]),
    "kernel_matvec_mapped": (ctypes.c_int, [_vp, _i64, _i32, _i32, _dbl, _vp, _i32, _dbl, _vp, _vp, _vp]),
    "krr_tile_map_counts": (ctypes.c_int, [_vp, _P(_i64), _vp]),
    "kernel_sample": (ctypes.c_int, [_vp, _i64, _i32, _i32, _dbl, _vp, _i32, _vp, _vp, _vp, _i32, _i32, _vp]),
    "krr_random_block": (ctypes.c_int, [_u64, _i64, _i32, _i32, _vp, _vp]),
    "kernel_matvec_bwd": (ctypes.c_int, [_vp, _i64, _vp, _i64, _i32, _i32, _dbl, _vp, _vp, _i32, _vp, _vp, _vp,
                                         _vp, _i32, _vp]),
    "hss_compress": (ctypes.c_int, [_vp, _vp, _i32, _i32, _dbl, _P(HssOpts), _vp, _P(_vp), _P(HssStats)]),
    "hss_destroy": (None, [_vp]),
    "hss_matvec": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp]),
    "hss_export_sizes": (ctypes.c_int, [_vp, _P(_i64), _P(_i64), _P(_i64)]),
    "hss_export": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "hss_ulv_factor": (ctypes.c_int, [_vp, _dbl, _vp, _P(_vp)]),
    "hss_ulv_factor_spd": (ctypes.c_int, [_vp, _dbl, _dbl, _vp, _P(_vp), _P(_i64)]),
    "hss_ulv_factor_shifted": (ctypes.c_int, [_vp, _dbl, _vp, _P(_vp), _P(_dbl)]),
    "hss_ulv_destroy": (None, [_vp]),
    "hss_ulv_use_graph": (ctypes.c_int, [_vp, _i32]),
    "hss_solve": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp]),
    "krr_refine": (ctypes.c_int, [_vp, _vp, _i64, _i32, _i32, _dbl, _dbl, _vp, _i32, _vp, _dbl, _i32, _i32, _i32,
                                  _vp, _P(RefineStats)]),
    "krr_predict": (ctypes.c_int, [_vp, _i64, _vp, _i64, _i32, _i32, _dbl, _vp, _i32, _vp, _vp, _i32, _vp]),
    "krr_predict_noalloc": (ctypes.c_int, [_vp, _i64, _vp, _i64, _i32, _i32, _dbl, _vp, _i32, _vp, _vp, _i32, _vp]),
    "krr_dot_columns": (ctypes.c_int, [_vp, _vp, _i64, _i32, _vp, _vp]),
    "krr_set_tuning": (ctypes.c_int, [_i32, _i32]),
    "krr_get_tuning": (ctypes.c_int, [_i32, _P(_i32)]),
    # batched form
    "krr_cluster_2mn_batched": (ctypes.c_int, [_vp, _i32, _P(_i64), _i32, _i32, _P(ClusterOpts), _vp, _vp,
                                               _P(_vp)]),
    "krr_tree_roots": (ctypes.c_int, [_vp, _P(_i64), _P(_i32)]),
    "hss_compress_batched": (ctypes.c_int, [_vp, _vp, _i32, _i32, _P(_dbl), _P(HssOpts), _vp, _P(_vp),
                                            _P(HssStats)]),
    "hss_num_problems": (ctypes.c_int, [_vp, _P(_i32)]),
    "hss_ulv_factor_batched": (ctypes.c_int, [_vp, _P(_dbl), _i32, _vp, _P(_vp), _P(_dbl)]),
    "kernel_sample_batched": (ctypes.c_int, [_vp, _i32, _P(_i64), _i32, _i32, _P(_dbl), _vp, _i32, _vp, _vp, _vp,
                                             _i32, _i32, _vp]),
    "kernel_matvec_batched": (ctypes.c_int, [_vp, _i32, _P(_i64), _i32, _i32, _P(_dbl), _vp, _i32, _vp, _i32,
                                             _vp]),
    "krr_refine_batched": (ctypes.c_int, [_vp, _vp, _i32, _P(_i64), _i32, _i32, _P(_dbl), _P(_dbl), _vp, _i32,
                                          _vp, _dbl, _i32, _i32, _i32, _vp, _P(RefineStats), _P(_dbl)]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libkrr.so and declare every entry point (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"libkrr.so not built ({path}); run __graft_entry__.build() or "
                              "python paper_1803_10274_amd/build.py")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(rc):
    if rc != KRR_OK:
        raise KrrError(rc, load().krr_last_error().decode(errors="replace"))
    return rc
