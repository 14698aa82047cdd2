"""A priori estimation of the BFP precisions (Section 6.2, Algorithm
bfp-prec-est), driven by the library's BFP V-cycles on the device.

conv-rate-v-cycle: rho_v = ||E||_A on a coarse level j, E the error
propagation matrix of one BFP IR-V iteration (b = 0, so the new iterate is
the propagated error), built column by column by running the iteration on
the canonical basis vectors; rho_v is the square root of the largest
generalized eigenvalue of E^T A E x = lambda A x (a dense host eigenproblem,
LAPACK through scipy, on at most a few thousand unknowns).

bfp-prec-est: with the width rules check_j(q) = j (m + k) + q and
inner_j(q) = j m + q (m = 1 and k = 2 for the 5- and 7-point Poisson
problems), the smallest q (binary search over 1..q_max) whose rate stays
within rho_thresh of the rate at q_max, first for the check width and then,
with that check width, for the inner width. Every width is capped at the
32-bit mantissa storage, the inner width at the working width (check >=
working >= inner), and the working widths are the solver's
w_j = min(32, 2j + 8).
"""
from __future__ import annotations

import numpy as np
import torch
from scipy.linalg import eigh

from . import Hierarchy, MG_POLICY_NN_IR_FIRST_Q, bfp_vec_to_f64, mg_params_init


def width_rules(j: int, q_check: int, q_inner: int, m: int = 1, k: int = 2, cap: int = 32):
    """(check, work, inner) widths of levels 1..j, as dicts."""
    work = {l: min(cap, 2 * l + 8) for l in range(1, j + 1)}
    check = {l: max(work[l], min(cap, l * (m + k) + q_check)) for l in range(1, j + 1)}
    inner = {l: min(work[l], l * m + q_inner) for l in range(1, j + 1)}
    return check, work, inner


def dense_A(j: int, ndim: int) -> np.ndarray:
    """The scaled operator of level j on the interior: 5-point [1; -1/4] in
    2D, 7-point [3/4; -1/8] in 3D."""
    n = (1 << j) - 1
    centre, off = (1.0, -0.25) if ndim == 2 else (0.75, -0.125)
    idx = np.arange(n ** ndim).reshape((n,) * ndim)
    A = np.diag(np.full(n ** ndim, centre))
    for ax in range(ndim):
        lo = [slice(None)] * ndim
        hi = [slice(None)] * ndim
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        a, b = idx[tuple(lo)].ravel(), idx[tuple(hi)].ravel()
        A[a, b] = off
        A[b, a] = off
    return A


def error_propagation(ndim: int, j: int, widths, policy: int = MG_POLICY_NN_IR_FIRST_Q,
                      nu=(1, 0), eta: int = 23, stream=None) -> np.ndarray:
    """E with E[:, k] = one BFP IR-V iteration on level j applied to e_k."""
    check, work, inner = widths
    p = mg_params_init(ndim, j, 32, True, nu[0], nu[1], 2, policy, eta)
    for l in range(1, j + 1):
        p.w_check[l], p.w_work[l], p.w_inner[l] = check[l], work[l], inner[l]
    H = Hierarchy(p, stream=stream)
    for l in range(1, j + 1):
        H.set_rhs(l, torch.zeros(((1 << l) + 1,) * ndim, dtype=torch.float64, device="cuda"),
                  stream)
    n = (1 << j) - 1
    N = n ** ndim
    side = (1 << j) + 1
    e = torch.zeros((side,) * ndim, dtype=torch.float64, device="cuda")
    cols = torch.empty((N, N), dtype=torch.float64, device="cuda")
    inner_view = (slice(1, -1),) * ndim
    for k in range(N):
        pos = tuple(int(c) + 1 for c in np.unravel_index(k, (n,) * ndim))
        e.zero_()
        e[pos] = 1.0
        H.set_x(j, e, stream)
        H.ir(j, 1, stream)
        cols[:, k] = bfp_vec_to_f64(H.get_vec(j, 0))[inner_view].reshape(-1)
    return cols.cpu().numpy()


def energy_rate(E: np.ndarray, A: np.ndarray) -> float:
    """||E||_A = sqrt(max lambda of E^T A E x = lambda A x)."""
    return float(np.sqrt(max(eigh(E.T @ A @ E, A, eigvals_only=True).max(), 0.0)))


def conv_rate_v_cycle(ndim: int, j: int, widths, **kw) -> float:
    return energy_rate(error_propagation(ndim, j, widths, **kw), dense_A(j, ndim))


def _min_q(ok, q_max: int) -> int:
    lo, hi = 1, q_max
    while lo < hi:
        mid = (lo + hi) // 2
        if ok(mid):
            hi = mid
        else:
            lo = mid + 1
    return lo


def bfp_prec_est(ndim: int, j_c: int, q_max: int, rho_thresh: float, **kw) -> dict:
    """Algorithm bfp-prec-est on level j_c: the constants of the check and
    inner width rules, the reference rate and the rate they reach."""
    cache = {}

    def rate(q_c, q_i):
        if (q_c, q_i) not in cache:
            cache[(q_c, q_i)] = conv_rate_v_cycle(ndim, j_c, width_rules(j_c, q_c, q_i), **kw)
        return cache[(q_c, q_i)]

    ref = rate(q_max, q_max)
    q_check = _min_q(lambda q: rate(q, q_max) / ref < rho_thresh, q_max)
    q_inner = _min_q(lambda q: rate(q_check, q) / ref < rho_thresh, q_max)
    return {"rho_ref": ref, "q_check": q_check, "q_inner": q_inner,
            "rho": rate(q_check, q_inner), "rates_evaluated": len(cache)}


def argmin_unimodal(f, lo: int, hi: int) -> int:
    """Smallest minimizer of f over the integers lo..hi, by ternary search
    (f taken as unimodal there), evaluating f at most once per point."""
    cache = {}

    def F(i):
        if i not in cache:
            cache[i] = f(i)
        return cache[i]

    while hi - lo > 2:
        m1 = lo + (hi - lo) // 3
        m2 = hi - (hi - lo) // 3
        if F(m1) <= F(m2):
            hi = m2
        else:
            lo = m1
    return min(range(lo, hi + 1), key=lambda i: (F(i), i))


def estimate_eta(ndim: int, j: int, widths, nu=(1, 0), lo: int = 1, hi: int = 99,
                 **kw) -> tuple[int, float]:
    """The Chebyshev smoother's parameter eta = i / 100 (the library's
    integer percent) with the smallest V-cycle rate rho_v on level j: the
    bfp-prec-est machinery applied to the eta the paper fixes empirically.
    Returns (i, rho_v)."""
    rate = lambda i: conv_rate_v_cycle(ndim, j, widths, nu=nu, eta=i, **kw)
    i = argmin_unimodal(rate, lo, hi)
    return i, rate(i)
