"""ctypes declarations of liblap's C ABI (include/lap.h).  Argument
marshalling only: every computation runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblap.so")

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_double = ctypes.c_double
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p
c_char_p = ctypes.c_char_p

LAP_OK, LAP_EINVAL, LAP_ENOMEM, LAP_ENOTCONV, LAP_EDIVERGED, LAP_EHIP = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "LAP_OK", -1: "LAP_EINVAL", -2: "LAP_ENOMEM", -3: "LAP_ENOTCONV",
                -4: "LAP_EDIVERGED", -5: "LAP_EHIP"}
LAP_SOR_RB, LAP_ADI, LAP_MG = 1, 2, 3
LAP_JACOBI, LAP_SOR_LEX, LAP_SLOR_LEX, LAP_ADI_LEX = 4, 5, 6, 7
LAP_FP64, LAP_MIXED = 0, 1
LAP_STOP_REL_L2, LAP_STOP_RES_INF, LAP_STOP_DELTA = 0, 1, 2
LAP_ADI_RELAX_AFTER, LAP_ADI_RELAX_INSIDE = 0, 1
LAP_SMOOTH_RB, LAP_SMOOTH_ZEBRA = 0, 1
LAP_ALLOC_FP64, LAP_ALLOC_MIXED, LAP_ALLOC_ADI, LAP_ALLOC_ALL = 1, 2, 4, 7

# kernel classes of lap_ctx_kernel_stats
KC_SWEEP, KC_SWEEP_PROLONG, KC_RESTRICT, KC_DEFECT, KC_COARSE, KC_FINALIZE, KC_ADI_ROWS, KC_ADI_COLS, \
    KC_RESIDUAL, KC_SUBTREE, KC_PRE, KC_TWO, KC_TWO_PLAIN, KC_PAPER, KC_FOUR = range(15)


class LapInfo(ctypes.Structure):
    _fields_ = [("iterations", c_int32), ("status", c_int32), ("rel_res_l2", c_double),
                ("res_l2", c_double), ("res_linf", c_double), ("res0_l2", c_double),
                ("seconds", c_double), ("monitor", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LapOpts(ctypes.Structure):
    _fields_ = [("method", c_int32), ("precision", c_int32), ("omega", c_double), ("tol", c_double),
                ("max_iter", c_int32), ("stop", c_int32), ("nu1", c_int32), ("nu2", c_int32),
                ("check_every", c_int32), ("adi_form", c_int32), ("use_graph", c_int32), ("smoother", c_int32),
                ("fmg", c_int32), ("inner", c_int32)]


_P = c_void_p
_S = c_int32      # lap_status
_PS = ctypes.POINTER

SIGNATURES = {
    "lap_opts_default": (None, [_PS(LapOpts)]),
    "lap_ctx_create": (_S, [_P, c_size_t, _P, _PS(_P)]),
    "lap_ctx_destroy": (_S, [_P]),
    "lap_ctx_usage": (_S, [_P, _PS(c_size_t), _PS(c_size_t)]),
    "lap_ctx_set_timing": (_S, [_P, c_int32]),
    "lap_ctx_kernel_stats": (_S, [_P, c_int32, c_int32, _PS(c_int64), _PS(c_double), _PS(c_double)]),
    "lap_ctx_reset_stats": (_S, [_P]),
    "lap_grid_footprint": (c_size_t, [c_int32, c_int32, c_int32]),
    "lap_grid_create": (_S, [_P, c_int32, c_int32, c_double, c_double, _P, _P, _PS(_P)]),
    "lap_grid_create_ex": (_S, [_P, c_int32, c_int32, c_double, c_double, _P, _P, c_int32, _PS(_P)]),
    "lap_grid_destroy": (_S, [_P]),
    "lap_grid_read": (_S, [_P, _P]),
    "lap_grid_write": (_S, [_P, _P]),
    "lap_grid_levels": (_S, [_P, _PS(c_int32)]),
    "lap_grid_level_shape": (_S, [_P, c_int32, _PS(c_int32), _PS(c_int32)]),
    "lap_solve": (_S, [_P, c_int32, c_double, c_double, c_int32, c_int32, _PS(LapInfo)]),
    "lap_solve_ex": (_S, [_P, _PS(LapOpts), _PS(LapInfo)]),
    "lap_residual": (_S, [_P, _PS(c_double), _PS(c_double)]),
    "lap_residual_ex": (_S, [_P, _PS(c_double), _PS(c_double)]),
    "lap_solve_batch": (_S, [_P, _PS(_P), c_int32, _PS(LapOpts), _PS(LapInfo)]),
    "lap_batch_step": (_S, [_P, _PS(_P), c_int32, c_int32, c_int32, _PS(c_int32), _PS(LapInfo)]),
    "lap_grid_set_tol": (_S, [_P, c_double]),
    "lap_grid_set_omega": (_S, [_P, c_double]),
    "lap_grid_reset": (_S, [_P]),
    "lap_op_rb_sweep": (_S, [c_int32, c_int32, c_int32, c_int32, c_double, c_double, c_double,
                             _P, _P, _P, c_int32, _P, _P]),
    "lap_op_residual": (_S, [c_int32, c_int32, c_int32, c_int32, c_double, c_double, _P, _P, _P, _P, _P, _P]),
    "lap_op_residual_static": (_S, [c_int32, c_int32, c_int32, c_int32, c_double, c_double, _P, _P, _P, _P, _P]),
    "lap_op_work_bytes": (c_size_t, [c_int32, c_int32]),
    "lap_op_restrict": (_S, [c_int32, c_int32, c_int32, c_int32, c_double, c_double, _P, _P, _P, c_int32, _P]),
    "lap_op_adi_half": (_S, [c_int32, c_int32, c_int32, c_int32, c_double, c_double, c_double, c_int32,
                             c_int32, _P, _P, _P, _P]),
    "lap_size_class": (c_int32, [c_int32, c_int32]),
    "lap_ctx_set_tiling": (_S, [_P, c_int32, c_int32, c_int32, c_int32, c_int32, c_int32]),
    "lap_ctx_get_tiling": (_S, [_P, c_int32, c_int32, c_int32, _PS(c_int32), _PS(c_int32), _PS(c_int32)]),
    "lap_ctx_set_subtree": (_S, [_P, c_int64]),
    "lap_ctx_set_fusion": (_S, [_P, c_int32]),
    "lap_ctx_get_fusion": (_S, [_P, _PS(c_int32)]),
    "lap_ctx_get_subtree": (_S, [_P, _PS(c_int64), _PS(c_int32)]),
    "lap_autotune": (_S, [_P, c_int32, c_int32, c_int32, c_char_p, c_size_t]),
    "lap_op_stream_copy": (_S, [_P, _P, c_size_t, c_int32, _P]),
    "lap_last_error": (c_char_p, []),
    "lap_version": (c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load liblap.so and declare every entry point; raises if it is missing
    (there is no fallback implementation)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() "
                           "(or python paper_2208_02427_amd/build.py)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
