"""The empirical Chebyshev parameter eta (paper Section 5 and Section 6.2).

The V-cycle convergence rate rho_v = ||E||_A is the square root of the largest
generalized eigenvalue of E^T A E x = lambda A x, where E = I - M A is the
error propagation matrix of one IR-V iteration and M (the V-cycle as a linear
map) is built by applying the V-cycle to the canonical basis vectors. eta is
chosen on the estimation level by minimizing rho_v over eta = i/100; the
open interval 0 < eta < 1 required by ChebyshevNodes leaves i = 1..99. Ties go
to the smallest i. Everything here is FP64, as a setup computation.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import scipy.linalg

from .fp64 import FP64MG, apply_f64
from .mg import cheby_nodes


def _interior_dense(mg: FP64MG, l: int, fn) -> np.ndarray:
    d = mg.ndim
    n = (1 << l) - 1
    N = n ** d
    out = np.empty((N, N))
    e = np.zeros(((n + 2),) * d)
    inner = (slice(1, -1),) * d
    for k in range(N):
        e[...] = 0.0
        e[inner].flat[k] = 1.0
        out[:, k] = fn(e)[inner].reshape(-1)
    return out


def vcycle_rate(ndim: int, l: int, c1: float, c2: float, nu1: int = 1,
                nu2: int = 0, a_c: float = 1.0) -> float:
    """rho_v of IR-V(nu1, nu2) on level l with exact (unquantized) c1, c2
    for D^-1 A; a_c rescales them to the stored operator."""
    f = {j: np.zeros(((1 << j) + 1,) * ndim) for j in range(1, l + 1)}
    mg = FP64MG(f, ndim, l, c1 / a_c, c2 / (a_c * a_c), nu1, nu2)
    A = _interior_dense(mg, l, lambda v: apply_f64(mg.A[l], v))
    M = _interior_dense(mg, l, lambda v: mg.vcycle(l, v))
    E = np.eye(A.shape[0]) - M @ A
    lam = scipy.linalg.eigh(E.T @ A @ E, A, eigvals_only=True)
    return float(np.sqrt(max(lam.max(), 0.0)))


def eta_search(ndim: int, l_est: int, nu1: int = 1, nu2: int = 0,
               rho: Fraction = Fraction(2), grid=range(1, 100)) -> tuple[Fraction, float]:
    a_c = 1.0 if ndim == 2 else 0.75
    best = None
    for i in grid:
        eta = Fraction(i, 100)
        c1, c2 = cheby_nodes(rho, eta)
        r = vcycle_rate(ndim, l_est, float(c1), float(c2), nu1, nu2, a_c)
        if best is None or r < best[1]:
            best = (eta, r)
    return best
