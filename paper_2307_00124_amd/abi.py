"""ctypes mirror of include/bfpmg.h and the loader of libbfpmg.so.

The library is required: importing this module raises if the shared object
is missing (build it with ``python paper_2307_00124_amd/build.py``). There is
no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbfpmg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bfpmg.h")

BFP_OK, BFP_EINVAL, BFP_EWIDTH, BFP_ESHAPE, BFP_ENONFINITE = 0, -1, -2, -3, -4
BFP_ENOMEM, BFP_EHIP, BFP_EBUSY, BFP_ENOTFOUND, BFP_PENDING = -5, -6, -7, -8, 1
BFP_NORMALIZE, BFP_SATURATE = 0, 1
BFP_STENCIL_A, BFP_STENCIL_R, BFP_STENCIL_P = 0, 1, 2
BFP_GAMMA_NORM, BFP_GAMMA_SUM, BFP_GAMMA_EXPLICIT = 1, 2, 3
BFP_META_SLOTS = 288
MG_DIAG_SITES = 8
MG_DIAG_BINS = 64
MG_DIAG_GAP_BINS = 61
BFP_META_EXP, BFP_META_MAX, BFP_META_MIN, BFP_META_SAT, BFP_META_MU, BFP_META_FLAGS = range(6)
MG_POLICY_Q, MG_POLICY_NN, MG_POLICY_NN_IR_FIRST_Q, MG_POLICY_NN_IR_FIRST2_Q, MG_POLICY_NN_IR_Q = range(5)
MG_MAX_LEVELS = 16
MG_NOALLOC_BYTES = 32 << 20


class bfp_vec(C.Structure):
    _fields_ = [("mant", C.c_void_p), ("meta", C.c_void_p), ("w", C.c_int32),
                ("storage_bits", C.c_int32), ("ndim", C.c_int32), ("n", C.c_int32),
                ("pitch", C.c_int64)]


class bfp_scalar(C.Structure):
    _fields_ = [("m", C.c_int64), ("exp", C.c_int64), ("w", C.c_int32)]


class bfp_stencil(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("kind", C.c_int32), ("exp", C.c_int64),
                ("w", C.c_int32), ("taps", C.c_int32 * 27)]


class bfp_tiles(C.Structure):
    _fields_ = [("mant", C.c_void_p), ("exps", C.c_void_p), ("w", C.c_int32),
                ("storage_bits", C.c_int32), ("ndim", C.c_int32), ("n", C.c_int32),
                ("T", C.c_int32), ("pitch", C.c_int64)]


class fe_rational_band(C.Structure):
    _fields_ = [("nrows", C.c_int32), ("ncols", C.c_int32), ("band", C.c_int32),
                ("col0", C.c_void_p), ("num", C.c_void_p), ("den", C.c_void_p)]


class fe_params(C.Structure):
    _fields_ = [("m", C.c_int32), ("L", C.c_int32), ("N", C.c_int32), ("eta_num", C.c_int32),
                ("eta_den", C.c_int32), ("w_check", C.c_int32 * 17), ("w_work", C.c_int32 * 17),
                ("w_inner", C.c_int32 * 17)]


class bfp_gamma(C.Structure):
    _fields_ = [("rule", C.c_int32), ("a_meta", C.c_void_p), ("b_meta", C.c_void_p),
                ("c", bfp_scalar)]


_W = C.c_int32 * (MG_MAX_LEVELS + 1)


class mg_params(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("L", C.c_int32), ("nu1", C.c_int32), ("nu2", C.c_int32),
                ("N", C.c_int32), ("policy", C.c_int32), ("min_storage_bits", C.c_int32),
                ("w_check", _W), ("w_work", _W), ("w_inner", _W),
                ("c1", bfp_scalar), ("c2", bfp_scalar), ("c1_gamma", bfp_scalar)]


class mg_prec_est_result(C.Structure):
    _fields_ = [("q_check", C.c_int32), ("q_inner", C.c_int32), ("rho_ref", C.c_double),
                ("rho", C.c_double), ("rates", C.c_int32)]


_LF = C.c_float * (MG_MAX_LEVELS + 1)


class mg_tune_report(C.Structure):
    _fields_ = [("first_level", C.c_int32), ("last_level", C.c_int32),
                ("star_rows", _W), ("transfer_rows", _W),
                ("star_us", _LF), ("star_default_us", _LF),
                ("transfer_us", _LF), ("transfer_default_us", _LF)]


class mg_server_cfg(C.Structure):
    _fields_ = [("max_slots", C.c_int32), ("max_queue", C.c_int32),
                ("exec_max_points", C.c_int32)]


class mg_request(C.Structure):
    _fields_ = [("prm", mg_params), ("rhs_dev", C.c_void_p * MG_MAX_LEVELS),
                ("x_out_dev", C.c_void_p)]


class mg_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("gpu_ms", C.c_float)]


P = C.POINTER
VP = C.c_void_p
I = C.c_int
I64 = C.c_int64

# name -> (restype, argtypes); the exported C-ABI
SIGNATURES = {
    "bfp_layout": (I, [I, I, I, P(I64), P(C.c_size_t)]),
    "bfp_vec_init": (I, [P(bfp_vec), VP]),
    "bfp_meta_reset": (I, [VP, VP]),
    "bfp_vec_assign": (I, [P(bfp_vec), I64, VP]),
    "bfp_vec_from_f64": (I, [VP, I64, P(bfp_vec), VP]),
    "bfp_vec_to_f64": (I, [P(bfp_vec), VP, VP]),
    "bfp_vec_check": (I, [P(bfp_vec), VP]),
    "bfp_stencil_apply": (I, [P(bfp_stencil), P(bfp_vec), P(bfp_scalar), P(bfp_scalar),
                              P(bfp_vec), I, I, P(bfp_gamma), P(bfp_vec), VP]),
    "bfp_residual": (I, [P(bfp_stencil), P(bfp_vec), P(bfp_vec), I, I, P(bfp_gamma),
                         P(bfp_vec), VP]),
    "bfp_axpy": (I, [P(bfp_scalar), P(bfp_vec), P(bfp_scalar), P(bfp_vec), I, I,
                     P(bfp_gamma), P(bfp_vec), VP]),
    "bfp_sub": (I, [P(bfp_vec), P(bfp_vec), I, I, P(bfp_gamma), P(bfp_vec), VP]),
    "bfp_dot": (I, [P(bfp_vec), P(bfp_vec), VP, VP]),
    "bfp_stream_copy": (I, [VP, VP, C.c_int64, I, VP]),
    "bfp_normalize": (I, [P(bfp_vec), I, P(bfp_vec), VP]),
    "bfp_saturate_truncate": (I, [P(bfp_vec), I, P(bfp_gamma), P(bfp_vec), VP]),
    "bfp_cheby_coeffs": (I, [I64, I64, I64, I64, I64, I64, I, P(bfp_scalar), P(bfp_scalar)]),
    "mg_params_init": (I, [I, I, I, I, I, I, I, I, I, P(mg_params)]),
    "bfp_energy_norm": (I, [P(C.c_double), I, I, P(C.c_double)]),
    "mg_conv_rate_bytes": (C.c_size_t, [P(mg_params)]),
    "mg_error_propagation": (I, [P(mg_params), VP, C.c_size_t, VP, P(C.c_double)]),
    "mg_conv_rate": (I, [P(mg_params), VP, C.c_size_t, VP, P(C.c_double)]),
    "mg_params_apply_estimate": (I, [P(mg_params), I, I, I, I]),
    "mg_prec_est": (I, [P(mg_params), I, C.c_double, I, I, VP, C.c_size_t, VP,
                        P(mg_prec_est_result)]),
    "mg_eta_scan": (I, [P(mg_params), I, I, VP, C.c_size_t, VP, P(I), P(C.c_double),
                        P(C.c_double)]),
    "mg_hierarchy_bytes": (C.c_size_t, [P(mg_params)]),
    "mg_hierarchy_create": (I, [P(mg_params), VP, C.c_size_t, VP, P(VP)]),
    "mg_hierarchy_destroy": (I, [VP]),
    "mg_set_rhs": (I, [VP, I, VP, VP]),
    "mg_set_x": (I, [VP, I, VP, VP]),
    "mg_fmg": (I, [VP, VP]),
    "mg_fmg_f64": (I, [VP, VP, VP]),
    "mg_diag_read": (I, [VP, VP, I, VP]),
    "mg_ir_safe": (I, [VP, I, I, I, I, I, P(I), VP]),
    "mg_ir": (I, [VP, I, I, VP]),
    "mg_vcycle": (I, [VP, I, P(bfp_vec), P(bfp_vec), VP]),
    "mg_get_vec": (I, [VP, I, I, P(bfp_vec)]),
    "mg_counters": (I, [VP, P(C.c_double), P(I64)]),
    "mg_batch_bytes": (C.c_size_t, [P(mg_params), I]),
    "mg_batch_create": (I, [P(mg_params), I, VP, C.c_size_t, VP, P(VP)]),
    "mg_batch_destroy": (I, [VP]),
    "mg_solve_batch": (I, [VP, VP, VP]),
    "mg_batch_get_vec": (I, [VP, I, I, I, P(bfp_vec)]),
    "mg_batch_counters": (I, [VP, P(C.c_double), P(I64)]),
    "mg_server_create": (I, [P(mg_server_cfg), VP, C.c_size_t, P(VP)]),
    "mg_server_submit": (I, [VP, P(mg_request), P(C.c_uint64)]),
    "mg_server_poll": (I, [VP, C.c_uint64, P(mg_result)]),
    "mg_server_stats": (I, [VP, P(I), P(I), P(C.c_size_t)]),
    "mg_server_collect": (I, [VP, P(C.c_uint64), P(mg_result), I, P(I)]),
    "mg_server_destroy": (I, [VP]),
    "mg_fmg_f64_noalloc": (I, [P(mg_params), VP, VP, VP]),
    "mg_autotune": (I, [VP, I, VP, P(mg_tune_report)]),
    "mg_autotune_solve": (I, [VP, I, VP, P(mg_tune_report)]),
    "fp64_mg_bytes": (C.c_size_t, [I, I]),
    "fp64_mg_create": (I, [I, I, I, I, I, C.c_double, C.c_double, VP, C.c_size_t, VP, P(VP)]),
    "fp64_mg_fmg": (I, [VP, VP, VP, VP]),
    "fp64_mg_destroy": (I, [VP]),
    "bfp_tiles_layout": (I, [I, I, I, I, P(I64), P(C.c_size_t), P(C.c_size_t)]),
    "bfp_tiles_init": (I, [P(bfp_tiles), VP]),
    "bfp_tiles_from_f64": (I, [VP, P(bfp_tiles), VP, VP]),
    "bfp_tiles_to_f64": (I, [P(bfp_tiles), VP, VP]),
    "bfp_tiles_stencil_apply": (I, [P(bfp_stencil), P(bfp_tiles), P(bfp_scalar), P(bfp_scalar),
                                    P(bfp_tiles), P(bfp_tiles), VP, VP]),
    "bfp_tiles_axpby": (I, [P(bfp_scalar), P(bfp_tiles), P(bfp_scalar), P(bfp_tiles),
                            P(bfp_tiles), VP, VP]),
    "fe_hierarchy_create": (I, [P(fe_params), VP, VP, VP, VP, P(VP)]),
    "fe_fmg": (I, [VP, VP]),
    "fe_get": (I, [VP, I, I, VP, P(I64), P(I)]),
    "fe_coefficients": (I, [VP, P(bfp_scalar), P(bfp_scalar)]),
    "fe_counters": (I, [VP, P(C.c_double), P(I64)]),
    "fe_hierarchy_destroy": (I, [VP]),
    "bfp_tuning_set": (I, [C.c_char_p, I]),
    "bfp_tuning_get": (I, [C.c_char_p, C.POINTER(I)]),
    "bfp_last_error": (C.c_char_p, []),
}


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python paper_2307_00124_amd/build.py` (there is no fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = load()


class BFPError(RuntimeError):
    def __init__(self, code: int, fn: str):
        msg = lib.bfp_last_error().decode()
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


def check(rc: int, fn: str) -> int:
    if rc < 0:
        raise BFPError(rc, fn)
    return rc
