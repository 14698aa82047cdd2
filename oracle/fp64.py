"""FP64 multigrid with the structure of the BFP solver, closed-form discrete
solutions and error norms.

The FP64 solver applies the same scaled operators (oracle.fd), the same
Chebyshev relaxation and the same IR / V(nu1, nu2) / FMG recursion as
oracle.mg, in IEEE double arithmetic. It is the floating-point comparator of
the paper's Figure 4 discussion and, iterated to algebraic convergence, it
reproduces the discrete solution u_h, whose closed form is known here because
sine modes are eigenvectors of the 5- and 7-point operators:
  -Laplace_h prod_k sin(k_k pi x_k) = (4/h^2) sum_k sin^2(k_k pi h / 2) * (same).
"""
from __future__ import annotations

import math

import numpy as np

from .fd import Stencil, level_scale, prolongation, scaled_A, scaled_R


def stencil_f64(st: Stencil) -> dict:
    return {o: float(t) * 2.0 ** st.e for o, t in st.taps.items()}


def apply_f64(st: Stencil, x: np.ndarray) -> np.ndarray:
    taps = stencil_f64(st)
    d = st.ndim
    nin = x.shape[0]
    if st.kind == "A":
        nout, src, step = nin, x, 1
    elif st.kind == "R":
        nout, src, step = (nin - 1) // 2 + 1, x, 2
    else:
        nout = 2 * (nin - 1) + 1
        src = np.zeros((nout,) * d)
        src[(slice(None, None, 2),) * d] = x
        step = 1
    out = np.zeros((nout,) * d)
    ni = nout - 2
    if ni <= 0:
        return out
    acc = np.zeros((ni,) * d)
    for o, t in taps.items():
        sl = tuple(slice(step + c, step + c + step * (ni - 1) + 1, step) for c in o)
        acc += t * src[sl]
    out[(slice(1, -1),) * d] = acc
    return out


class FP64MG:
    """IR / V(nu1, nu2) / FMG in FP64 on the scaled system A' u = b'."""

    def __init__(self, f_levels: dict, ndim: int, L: int, c1: float, c2: float,
                 nu1: int = 1, nu2: int = 0):
        self.ndim, self.L, self.c1, self.c2 = ndim, L, float(c1), float(c2)
        self.nu1, self.nu2 = nu1, nu2
        self.A = {j: scaled_A(j, ndim) for j in range(1, L + 1)}
        self.R = {j: scaled_R(j, ndim) for j in range(2, L + 1)}
        self.P = prolongation(ndim)
        self.b = {j: np.asarray(f_levels[j], dtype=np.float64) / float(level_scale(j, ndim))
                  for j in range(1, L + 1)}

    def relax0(self, l, r):
        return self.c2 * apply_f64(self.A[l], r) + self.c1 * r

    def vcycle(self, l: int, r: np.ndarray) -> np.ndarray:
        A = self.A[l]
        y = self.relax0(l, r)
        for _ in range(1, self.nu1):
            s = apply_f64(A, y) - r
            y = y - self.relax0(l, s)
        if l > 1:
            rv = apply_f64(A, y) - r
            d = self.vcycle(l - 1, apply_f64(self.R[l], rv))
            y = y - apply_f64(self.P, d)
        for _ in range(self.nu2):
            s = apply_f64(A, y) - r
            y = y - self.relax0(l, s)
        return y

    def ir(self, l: int, x: np.ndarray) -> np.ndarray:
        r = apply_f64(self.A[l], x) - self.b[l]
        return x - self.vcycle(l, r)

    def fmg(self, N: int, L: int | None = None) -> np.ndarray:
        L = self.L if L is None else L
        x = np.zeros((3,) * self.ndim)
        for l in range(1, L + 1):
            if l > 1:
                x = apply_f64(self.P, x)
            for _ in range(N):
                x = self.ir(l, x)
        return x

    def solve(self, tol: float = 1e-15, max_iter: int = 200, N: int = 2) -> np.ndarray:
        """FMG followed by IR-V iterations to algebraic convergence."""
        x = self.fmg(N)
        for _ in range(max_iter):
            xn = self.ir(self.L, x)
            if np.max(np.abs(xn - x)) <= tol * max(1.0, np.max(np.abs(xn))):
                return xn
            x = xn
        return x


def kappa_h(j: int) -> float:
    """u_h = kappa_h u* for the manufactured single-mode problems."""
    h = 2.0 ** -j
    return (math.pi * h) ** 2 / (4.0 * math.sin(math.pi * h / 2.0) ** 2)


def discrete_solution_manufactured(u_star: np.ndarray, j: int) -> np.ndarray:
    return kappa_h(j) * u_star


def discrete_solution_modes(j: int, modes, coords: np.ndarray) -> np.ndarray:
    """u_h = sum_i a_i / lambda_h(k_i) prod sin(k pi x) with
    lambda_h = (4/h^2) sum_k sin^2(k pi h / 2)."""
    h = 2.0 ** -j
    d = modes.ndim
    out = np.zeros((coords.size,) * d)
    for i in range(modes.k.shape[0]):
        lam = (4.0 / h ** 2) * sum(math.sin(float(kk) * math.pi * h / 2.0) ** 2
                                   for kk in modes.k[i])
        parts = []
        for kk in modes.k[i]:
            s = np.sin(math.pi * float(kk) * coords)
            s[0] = 0.0
            s[-1] = 0.0
            parts.append(s)
        t = parts[0]
        for p in parts[1:]:
            t = np.multiply.outer(p, t)
        out += (modes.a[i] / lam) * t
    return out


def l2_error(u: np.ndarray, ref: np.ndarray, j: int) -> float:
    """Discrete L2 norm over interior nodes: sqrt(h^d sum (u - ref)^2)."""
    d = u.ndim
    inner = (slice(1, -1),) * d
    e = (np.asarray(u, dtype=np.float64) - np.asarray(ref, dtype=np.float64))[inner]
    return math.sqrt((2.0 ** -j) ** d * float(np.sum(e * e)))
