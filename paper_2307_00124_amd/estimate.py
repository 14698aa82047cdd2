"""A priori estimation of the BFP precisions (Section 6.2, Algorithm
bfp-prec-est) and of the Chebyshev parameter eta (Section 5): bindings of
the library's mg_error_propagation, mg_conv_rate, mg_prec_est, mg_eta_scan
and mg_params_apply_estimate (argument marshalling only; the searches, the
device solves and the energy norm run in the library)."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import abi, check, lib, mg_params_init, MG_POLICY_NN_IR_FIRST_Q


def _copy(p: abi.mg_params) -> abi.mg_params:
    q = abi.mg_params()
    C.memmove(C.addressof(q), C.addressof(p), C.sizeof(p))
    return q


class _Arena:
    """A 256-byte aligned device arena sized by mg_conv_rate_bytes."""

    def __init__(self, params: abi.mg_params, device="cuda"):
        n = lib.mg_conv_rate_bytes(C.byref(params))
        if n == 0:
            check(abi.BFP_EINVAL, "mg_conv_rate_bytes")
        buf = torch.empty(n + 256, dtype=torch.uint8, device=device)
        off = (-buf.data_ptr()) % 256
        self.buf = buf[off:off + n]
        self.ptr = C.c_void_p(self.buf.data_ptr())
        self.bytes = n


def base_params(ndim: int, j: int, nu=(1, 0), eta_percent: int = 23,
                policy: int = MG_POLICY_NN_IR_FIRST_Q) -> abi.mg_params:
    """Parameters of the estimation level j: the solver's working widths
    w_j = min(32, 2j + 8), cycle nu, policy and eta; check and inner widths
    are set by the width rules of each evaluation."""
    return mg_params_init(ndim, j, 32, True, nu[0], nu[1], 2, policy, eta_percent)


def apply_estimate(params: abi.mg_params, q_check: int, q_inner: int, m: int = 1,
                   k: int = 2) -> abi.mg_params:
    """A copy of params with the check and inner width rules of
    bfp-prec-est applied (mg_params_apply_estimate)."""
    p = _copy(params)
    check(lib.mg_params_apply_estimate(C.byref(p), q_check, q_inner, m, k),
          "mg_params_apply_estimate")
    return p


def widths(params: abi.mg_params) -> tuple[dict, dict, dict]:
    L = params.L
    return ({j: params.w_check[j] for j in range(1, L + 1)},
            {j: params.w_work[j] for j in range(1, L + 1)},
            {j: params.w_inner[j] for j in range(1, L + 1)})


def error_propagation(params: abi.mg_params) -> np.ndarray:
    """E (N x N, E[:, k] = one IR-V iteration applied to e_k) on level
    params.L, from the device."""
    ar = _Arena(params)
    N = ((1 << params.L) - 1) ** params.ndim
    E = np.zeros(N * N, dtype=np.float64)
    check(lib.mg_error_propagation(C.byref(params), ar.ptr, ar.bytes, None,
                                   E.ctypes.data_as(C.POINTER(C.c_double))),
          "mg_error_propagation")
    return E.reshape(N, N).T.copy()


def energy_norm(E: np.ndarray, ndim: int, j: int) -> float:
    """||E||_A for the scaled operator of level j (bfp_energy_norm)."""
    Ec = np.ascontiguousarray(np.asarray(E, dtype=np.float64).T)
    rho = C.c_double()
    check(lib.bfp_energy_norm(Ec.ctypes.data_as(C.POINTER(C.c_double)), ndim, j,
                              C.byref(rho)), "bfp_energy_norm")
    return rho.value


def conv_rate(params: abi.mg_params) -> float:
    ar = _Arena(params)
    rho = C.c_double()
    check(lib.mg_conv_rate(C.byref(params), ar.ptr, ar.bytes, None, C.byref(rho)), "mg_conv_rate")
    return rho.value


def bfp_prec_est(params: abi.mg_params, q_max: int = 64, rho_thresh: float = 1.05,
                 m: int = 1, k: int = 2) -> dict:
    """Algorithm bfp-prec-est on level params.L (mg_prec_est)."""
    ar = _Arena(apply_estimate(params, q_max, q_max, m, k))
    r = abi.mg_prec_est_result()
    check(lib.mg_prec_est(C.byref(params), q_max, float(rho_thresh), m, k, ar.ptr, ar.bytes,
                          None, C.byref(r)), "mg_prec_est")
    return {"q_check": r.q_check, "q_inner": r.q_inner, "rho_ref": r.rho_ref, "rho": r.rho,
            "rates_evaluated": r.rates}


def eta_scan(params: abi.mg_params, lo: int = 1, hi: int = 99) -> tuple[int, float, list]:
    """eta = i / 100 in lo..hi minimizing rho_v on level params.L
    (mg_eta_scan): (i, its rate, every rate)."""
    ar = _Arena(params)
    best = C.c_int()
    rho = C.c_double()
    rates = (C.c_double * (hi - lo + 1))()
    check(lib.mg_eta_scan(C.byref(params), lo, hi, ar.ptr, ar.bytes, None, C.byref(best),
                          C.byref(rho), rates), "mg_eta_scan")
    return best.value, rho.value, list(rates)
