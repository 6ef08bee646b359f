"""ctypes declarations of librnamg (include/rnamg.h).

Argument marshalling only.  Importing this module loads the in-tree
librnamg.so and fails loudly when it is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librnamg.so")

RN_OK, RN_EINVAL, RN_ENOMEM, RN_ESINGULAR, RN_EBREAKDOWN, RN_ENONFINITE, RN_EHIP, RN_ELIMIT = range(8)
RN_CG, RN_GMRES, RN_PCG_JACOBI, RN_CGNR = 0, 1, 2, 3
RN_FP64, RN_FP32_MIXED = 0, 1
RN_OPT_PERSISTENT_PRODUCT, RN_OPT_PADDED_PATTERN, RN_OPT_FUSED_SETUP, RN_OPT_PRODUCT_LANES, RN_OPT_METRICS, \
    RN_OPT_FUSED_CG, RN_OPT_TAPE_INTERVAL = range(7)
# rn_set_allocator callbacks: void *alloc(size_t bytes, void *user); void release(void *ptr, void *user)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
# bytes of the allocation-free entry point's scratch array per GPU
NOALLOC_SCRATCH_BYTES = 64 << 20
STATUS_NAMES = {0: "RN_OK", 1: "RN_EINVAL", 2: "RN_ENOMEM", 3: "RN_ESINGULAR", 4: "RN_EBREAKDOWN",
                5: "RN_ENONFINITE", 6: "RN_EHIP", 7: "RN_ELIMIT"}


class rn_matrix(C.Structure):
    _fields_ = [("n", C.c_int32), ("block_m", C.c_int32), ("nnz", C.c_int64),
                ("rowptr", C.c_void_p), ("colind", C.c_void_p), ("vals", C.c_void_p)]


class rn_emin_stats(C.Structure):
    _fields_ = [("iters_done", C.c_int32), ("rank_deficient_rows", C.c_int32),
                ("status_code", C.c_int32), ("fused_cg", C.c_int32),
                ("first", C.c_double), ("last", C.c_double),
                ("spgemm_bytes", C.c_double), ("spgemm_flops", C.c_double),
                ("work_units", C.c_double), ("energy", C.c_double), ("proj_residual", C.c_double),
                ("constraint_residual", C.c_double)]


class rn_setup_view(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_cols", C.c_int32), ("nB", C.c_int32), ("rank_deficient", C.c_int32),
                ("nnz_S", C.c_int64), ("nnz_N", C.c_int64),
                ("S_rowptr", C.c_void_p), ("S_colind", C.c_void_p),
                ("N_rowptr", C.c_void_p), ("N_colind", C.c_void_p), ("is_root", C.c_void_p),
                ("T", C.c_void_p), ("Bc", C.c_void_p), ("P", C.c_void_p),
                ("That", C.c_void_p), ("Bchat", C.c_void_p), ("RT", C.c_void_p),
                ("plan", C.c_void_p), ("plan_T", C.c_void_p)]


class rn_level_view(C.Structure):
    _fields_ = [("n", C.c_int32), ("block_m", C.c_int32), ("nnz_A", C.c_int64),
                ("A_rowptr", C.c_void_p), ("A_colind", C.c_void_p), ("A_vals", C.c_void_p), ("B", C.c_void_p),
                ("nB", C.c_int32), ("n_agg", C.c_int32), ("agg", C.c_void_p), ("roots", C.c_void_p),
                ("setup", C.c_void_p), ("stats", rn_emin_stats), ("stats_RT", rn_emin_stats)]


# name -> (restype, argtypes); every declaration of include/rnamg.h
_vp, _i32, _i64, _d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
_pi32, _pi64 = C.POINTER(C.c_int32), C.POINTER(C.c_int64)
SIGNATURES = {
    "rn_create": (_i32, [C.POINTER(C.c_void_p), _vp]),
    "rn_destroy": (None, [_vp]),
    "rn_set_stream": (_i32, [_vp, _vp]),
    "rn_set_allocator": (_i32, [_vp, _vp, _vp, _vp]),
    "rn_set_option": (_i32, [_vp, _i32, _i32]),
    "rn_last_error": (C.c_char_p, [_vp]),
    "rn_version": (C.c_char_p, []),
    "rn_strength": (_i32, [_vp, C.POINTER(rn_matrix), _d, _vp, _vp, _pi64]),
    "rn_strength_values": (_i32, [_vp, C.POINTER(rn_matrix), _d, _vp, _vp, _i64, _vp]),
    "rn_pattern_values": (_i32, [_vp, _i32, _vp, _vp, _vp, _i64, _vp, _i32, _i32, _vp, _vp, _vp, _pi64]),
    "rn_pattern_dofs": (_i32, [_vp, _i32, _vp, _vp, _i64, _vp, _vp, _i32, _i32, _vp, _vp, _vp, _pi64]),
    "rn_aggregate_host": (_i32, [_i32, _vp, _vp, _vp, _vp, _pi32]),
    "rn_pattern": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _i32, _i32, _i32, _vp, _vp, _vp, _pi64]),
    "rn_smooth_candidates": (_i32, [_vp, C.POINTER(rn_matrix), _vp, _i32, _i32, _d]),
    "rn_tentative": (_i32, [_vp, _i32, _i32, _vp, _vp, _i64, _vp, _vp, _vp, _i32, _vp, _i32, _vp, _vp, _pi32]),
    "rn_filter": (_i32, [_vp, _i32, _i32, _vp, _vp, _i64, _vp, _vp, _vp, _i32, _d, _vp, _vp, _vp, _pi64]),
    "rn_enforce": (_i32, [_vp, _i32, _i32, _vp, _vp, _i64, _vp, _vp, _vp, _i32, _vp, _pi32]),
    "rn_spgemm": (_i32, [_vp, _i32, _i32, _i32, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _pi64]),
    "rn_galerkin": (_i32, [_vp, C.POINTER(rn_matrix), _i32, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _pi64]),
    "rn_transpose": (_i32, [_vp, C.POINTER(rn_matrix), _vp, _vp, _vp, _vp]),
    "rn_plan_create": (_i32, [_vp, C.POINTER(rn_matrix), _i32, _vp, _vp, _i64, _vp, _vp, _i32,
                              C.POINTER(C.c_void_p)]),
    "rn_plan_destroy": (None, [_vp]),
    "rn_plan_bytes": (C.c_size_t, [_vp]),
    "rn_masked_product": (_i32, [_vp, _vp, _vp, _i32, _vp, _i32, _i32, _vp]),
    "rn_energy_min": (_i32, [_vp, _vp, _vp, _i32, _vp, _i32, _i32, _i32, _vp, _vp,
                             C.POINTER(rn_emin_stats), _vp]),
    "rn_energy_min_noalloc": (_i32, [_vp, _vp, _vp, _i32, _vp, _i32, _i32, _i32, _vp, _vp,
                                     C.POINTER(rn_emin_stats)]),
    "rn_energy": (_i32, [_vp, _vp, _vp, _vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "rn_constraint_residual": (_i32, [_vp, _i32, _i32, _vp, _vp, _i64, _vp, _vp, _vp, _i32,
                                      C.POINTER(C.c_double)]),
    "rn_tape_create": (_i32, [_vp, _vp, _i32, _i32, C.POINTER(C.c_void_p)]),
    "rn_tape_destroy": (None, [_vp]),
    "rn_energy_min_bwd": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "rn_setup": (_i32, [_vp, C.POINTER(rn_matrix), _vp, _vp, _i32, _vp, _vp, _i32, _i32, _i32, _d, _i32, _i32,
                        C.POINTER(C.c_void_p), C.POINTER(rn_emin_stats), C.POINTER(rn_emin_stats)]),
    "rn_setup_view_get": (_i32, [_vp, C.POINTER(rn_setup_view)]),
    "rn_setup_destroy": (None, [_vp]),
    "rn_hierarchy_build": (_i32, [_vp, C.POINTER(rn_matrix), _vp, _i32, _i32, _i32, _d, _i32, _i32, _i32, _i32,
                                  C.POINTER(C.c_void_p)]),
    "rn_hierarchy_levels": (_i32, [_vp]),
    "rn_hierarchy_level": (_i32, [_vp, _i32, C.POINTER(rn_level_view)]),
    "rn_hierarchy_destroy": (None, [_vp]),
}

_lib = None


def lib():
    """The loaded library; raises ImportError when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              f"`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib
