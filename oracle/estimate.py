"""A priori estimation of the BFP precisions (Section 6.2, Algorithm
bfp-prec-est). Test infrastructure: the plain reference the device-driven
estimation is checked against.

conv-rate-v-cycle: rho_v = ||E||_A, the square root of the largest
generalized eigenvalue of E^T A E x = lambda A x, where E is the error
propagation matrix of one BFP IR-V iteration on level j (b = 0, so the new
iterate is the propagated error) built column by column from the canonical
basis vectors, A the scaled operator of the level (scaling A does not change
the eigenvalues).

bfp-prec-est: with the width rules check_j(q) = j (m + k) + q and
inner_j(q) = j m + q (m = 1, k = 2 for the 5- and 7-point Poisson problems),
rho_ref = rho_v(check(q_max), inner(q_max)), then the smallest q with
rho_v(check(q), inner(q_max)) / rho_ref < rho_thresh, then the smallest q'
with rho_v(check(q), inner(q')) / rho_ref < rho_thresh (binary searches over
1..q_max). Readings: widths are capped at 32 bits (the mantissa storage) and
the inner width at the working width (the order check >= working >= inner);
the working widths are the solver's w_j = min(32, 2j + 8).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
from scipy.linalg import eigh

from . import fd, mg
from .bfp import from_f64


def width_rules(j: int, q_check: int, q_inner: int, m: int = 1, k: int = 2,
                cap: int = 32) -> mg.Widths:
    """Widths of levels 1..j under the rules of bfp-prec-est."""
    work = {l: min(cap, 2 * l + 8) for l in range(1, j + 1)}
    check = {l: max(work[l], min(cap, l * (m + k) + q_check)) for l in range(1, j + 1)}
    inner = {l: min(work[l], l * m + q_inner) for l in range(1, j + 1)}
    return mg.Widths(check, work, inner)


def dense_A(j: int, ndim: int) -> np.ndarray:
    """The scaled operator of level j as a dense matrix on the interior."""
    n = (1 << j) - 1
    N = n ** ndim
    taps = {o: float(t) * 2.0 ** fd.scaled_A(j, ndim).e for o, t in fd.scaled_A(j, ndim).taps.items()}
    A = np.zeros((N, N))
    idx = np.arange(N).reshape((n,) * ndim)
    for p in np.ndindex(*(n,) * ndim):
        for o, t in taps.items():
            q = tuple(a + b for a, b in zip(p, o[-ndim:]))
            if all(0 <= c < n for c in q):
                A[idx[p], idx[q]] += t
    return A


def error_propagation(ndim: int, j: int, widths: mg.Widths, policy: str = "nn_ir_first_q",
                      nu=(1, 0), eta: Fraction = Fraction(23, 100)) -> np.ndarray:
    """E with E[:, k] = one BFP IR-V iteration applied to e_k (b = 0)."""
    n = (1 << j) - 1
    zeros = {l: np.zeros(((1 << l) + 1,) * ndim) for l in range(1, j + 1)}
    H = mg.build_hierarchy(zeros, ndim, j, widths, mg.make_smoother(ndim, eta),
                           policy=policy, nu1=nu[0], nu2=nu[1])
    cols = []
    for k in range(n ** ndim):
        e = np.zeros(((1 << j) + 1,) * ndim)
        e[tuple(c + 1 for c in np.unravel_index(k, (n,) * ndim))] = 1.0
        x1, _ = mg.ir_iteration(H, j, from_f64(e, widths.work[j]), None, first=True)
        cols.append(x1.to_f64()[(slice(1, -1),) * ndim].ravel())
    return np.stack(cols, axis=1)


def energy_rate(E: np.ndarray, A: np.ndarray) -> float:
    """||E||_A = sqrt(max lambda of E^T A E x = lambda A x)."""
    return float(np.sqrt(max(eigh(E.T @ A @ E, A, eigvals_only=True).max(), 0.0)))


def conv_rate_v_cycle(ndim: int, j: int, widths: mg.Widths, **kw) -> float:
    return energy_rate(error_propagation(ndim, j, widths, **kw), dense_A(j, ndim))


def _min_q(ok, q_max: int) -> int:
    """Smallest q in 1..q_max with ok(q), by binary search (ok is taken as
    monotone in q); q_max when none."""
    lo, hi = 1, q_max
    while lo < hi:
        mid = (lo + hi) // 2
        if ok(mid):
            hi = mid
        else:
            lo = mid + 1
    return lo


def bfp_prec_est(ndim: int, j_c: int, q_max: int, rho_thresh: float, rate=None,
                 **kw) -> dict:
    """Algorithm bfp-prec-est; `rate(widths)` gives rho_v on level j_c (the
    oracle's by default). Returns the constants and the rates met."""
    if rate is None:
        rate = lambda wd: conv_rate_v_cycle(ndim, j_c, wd, **kw)
    ref = rate(width_rules(j_c, q_max, q_max))
    q_check = _min_q(lambda q: rate(width_rules(j_c, q, q_max)) / ref < rho_thresh, q_max)
    q_inner = _min_q(lambda q: rate(width_rules(j_c, q_check, q)) / ref < rho_thresh, q_max)
    return {"rho_ref": ref, "q_check": q_check, "q_inner": q_inner,
            "rho": rate(width_rules(j_c, q_check, q_inner))}


def estimate_eta(ndim: int, j: int, widths: mg.Widths, nu=(1, 0), lo: int = 1, hi: int = 99,
                 **kw) -> tuple[int, float]:
    """The Chebyshev smoother's parameter: Section 5 minimizes the V-cycle
    convergence rate over eta = i / 100; every i in lo..hi is evaluated
    (i = 0 and 100 are excluded since 0 < eta < 1), ties go to the smaller
    i. Returns (i, rho_v)."""
    best = None
    for i in range(lo, hi + 1):
        r = conv_rate_v_cycle(ndim, j, widths, nu=nu, eta=Fraction(i, 100), **kw)
        if best is None or r < best[1]:
            best = (i, r)
    return best
