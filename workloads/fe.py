"""The paper's finite-element model problems (Section 6), as problem data.

1D Poisson -u'' = f (m = 1) and the biharmonic u'''' = f (m = 2) on (0, 1)
with homogeneous Dirichlet conditions imposed strongly (u = 0, and u' = 0
for the biharmonic), discretized by Rayleigh-Ritz with B-splines of degree p
on a uniform mesh of M = 2^j elements (open knot vector: p + 1 knots at each
end). Level j has M + p basis functions, of which the first and last c are
removed by the boundary conditions (c = m), leaving n_j = M + p - 2m
unknowns.

This module is shared by the oracle, the tests and the benchmark as the
definition of the discrete problems. Everything is on the reference mesh of
unit spacing (knots 0, 1, ..., M), the physical mesh size h = 1/M entering
only as the factor h^(1-2m) of the stiffness matrix and h of the load
vector:
  * the stiffness matrix K_hat = int B_i^(m) B_k^(m) (exact rationals,
    piecewise polynomial integration),
  * the prolongation P from level j-1 to level j (the coarse B-splines as
    combinations of the fine ones, exact rationals by the Oslo algorithm),
  * the load vector F_hat_i = int f(h x) B_i(x) dx (FP64, Gauss-Legendre
    with p + 1 nodes per element, as the paper does).
It holds none of the BFP method's arithmetic: no set-up scaling, no
quantization.

Manufactured solutions (the paper only says "smooth functions with
trigonometric components"): u = sin(pi x) for Poisson, u = sin(pi x)^2 for
the biharmonic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from fractions import Fraction
from functools import lru_cache

import numpy as np

__all__ = ["Band", "knots", "n_unknowns", "stiffness", "prolongation", "load_vector",
           "manufactured", "PAPER_N", "element_basis", "solution_values",
           "discrete_solution", "l2_error"]

# IR-V iterations per FMG level from the paper's Figure 5 caption
PAPER_N = {("poisson", p): n for p, n in zip(range(1, 7), (2, 1, 1, 3, 7, 15))}
PAPER_N.update({("biharmonic", p): n for p, n in zip(range(3, 7), (2, 1, 2, 4))})


@dataclass
class Band:
    """A banded matrix: row i holds vals[i][t] at column col0[i] + t."""
    nrows: int
    ncols: int
    col0: list
    vals: list

    def dense(self) -> list:
        out = [[Fraction(0)] * self.ncols for _ in range(self.nrows)]
        for i in range(self.nrows):
            for t, v in enumerate(self.vals[i]):
                out[i][self.col0[i] + t] = Fraction(v)
        return out


def knots(M: int, p: int) -> tuple:
    return tuple([0] * (p + 1) + list(range(1, M)) + [M] * (p + 1))


def n_unknowns(j: int, p: int, m: int) -> int:
    return (1 << j) + p - 2 * m


# ---------------------------------------------------- piecewise polynomials

def _pmul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        if x:
            for k, y in enumerate(b):
                out[i + k] += x * y
    return out


def _padd(a, b):
    n = max(len(a), len(b))
    return [(a[i] if i < len(a) else 0) + (b[i] if i < len(b) else 0) for i in range(n)]


def _pderiv(a, k=1):
    for _ in range(k):
        a = [i * a[i] for i in range(1, len(a))] or [Fraction(0)]
    return a


def _pint01(a) -> Fraction:
    """int_0^1 of a polynomial in the local variable."""
    return sum((c / (i + 1) for i, c in enumerate(a)), Fraction(0))


@lru_cache(maxsize=None)
def _local_basis(window: tuple, p: int) -> tuple:
    """Polynomials (in the local variable s = x - e, ascending coefficients)
    of the p + 1 B-splines nonzero on the element [e, e + 1], from the
    knots window = t[mu - p .. mu + p + 1] - e (mu = e + p) by the Cox-de
    Boor recursion."""
    t = [Fraction(v) for v in window]
    # N[i] for i = 0..p: the basis function with knots t[i .. i + r + 1]
    # at recursion depth r, restricted to the element (t[p], t[p + 1])
    N = [[Fraction(0)] for _ in range(p + 1)]
    N[p] = [Fraction(1)]
    for r in range(1, p + 1):
        new = [[Fraction(0)] for _ in range(p + 1)]
        for i in range(p - r, p + 1):
            acc = [Fraction(0)]
            d1 = t[i + r] - t[i]
            if d1 != 0:   # (s - t_i) / (t_{i+r} - t_i) N_{i, r-1}
                acc = _padd(acc, _pmul([-t[i] / d1, 1 / d1], N[i]))
            if i + 1 <= p:
                d2 = t[i + r + 1] - t[i + 1]
                if d2 != 0:   # (t_{i+r+1} - s) / (t_{i+r+1} - t_{i+1}) N_{i+1, r-1}
                    acc = _padd(acc, _pmul([t[i + r + 1] / d2, -1 / d2], N[i + 1]))
            new[i] = acc
        N = new
    return tuple(tuple(v) for v in N)


def element_basis(M: int, p: int, e: int) -> tuple:
    """(first basis index, polynomials) of the B-splines nonzero on element
    e of the level with M elements."""
    t = knots(M, p)
    mu = e + p
    window = tuple(t[k] - e for k in range(mu - p, mu + p + 2))
    return e, _local_basis(window, p)


@lru_cache(maxsize=None)
def _element_matrix(window: tuple, p: int, m: int) -> tuple:
    B = _local_basis(window, p)
    D = [_pderiv(list(b), m) for b in B]
    return tuple(tuple(_pint01(_pmul(D[a], D[b])) for b in range(p + 1))
                 for a in range(p + 1))


@lru_cache(maxsize=None)
def stiffness(j: int, p: int, m: int) -> Band:
    """K_hat on the unknowns of level j (reference mesh), banded."""
    M = 1 << j
    t = knots(M, p)
    nb = M + p
    rows = [dict() for _ in range(nb)]
    for e in range(M):
        mu = e + p
        window = tuple(t[k] - e for k in range(mu - p, mu + p + 2))
        Ke = _element_matrix(window, p, m)
        for a in range(p + 1):
            for b in range(p + 1):
                if Ke[a][b]:
                    rows[e + a][e + b] = rows[e + a].get(e + b, Fraction(0)) + Ke[a][b]
    keep = range(m, nb - m)
    n = len(keep)
    col0, vals = [], []
    for i in keep:
        cols = [k - m for k in rows[i] if m <= k < nb - m]
        lo, hi = min(cols), max(cols)
        col0.append(lo)
        vals.append([rows[i].get(lo + m + q, Fraction(0)) for q in range(hi - lo + 1)])
    return Band(n, n, col0, vals)


@lru_cache(maxsize=None)
def _oslo(t: tuple, tau: tuple, p: int) -> Fraction:
    """alpha with B[t] = sum_k alpha_k B[tau_k] for one coarse B-spline with
    knots t (p + 2 of them) and one fine B-spline with knots tau (p + 2):
    the Oslo algorithm's discrete B-spline recurrence,
      alpha_(i,0) = [t_i <= tau_0 < t_(i+1)],
      alpha_(i,r) = (tau_r - t_i)/(t_(i+r) - t_i) alpha_(i,r-1)
                    + (t_(i+r+1) - tau_r)/(t_(i+r+1) - t_(i+1)) alpha_(i+1,r-1)
    (terms with a zero denominator dropped). Knots are relative (exact
    integers), so translated configurations share one computation."""
    memo = {}

    def alpha(i, r):
        if (i, r) in memo:
            return memo[(i, r)]
        if r == 0:
            v = Fraction(1) if t[i] <= tau[0] < t[i + 1] else Fraction(0)
        else:
            v = Fraction(0)
            d1 = t[i + r] - t[i]
            if d1:
                v += Fraction(tau[r] - t[i], d1) * alpha(i, r - 1)
            d2 = t[i + r + 1] - t[i + 1]
            if d2:
                v += Fraction(t[i + r + 1] - tau[r], d2) * alpha(i + 1, r - 1)
        memo[(i, r)] = v
        return v
    return alpha(0, p)


@lru_cache(maxsize=None)
def prolongation(j: int, p: int, m: int) -> Band:
    """P from level j - 1 to level j on the unknowns (fine rows, coarse
    columns): coarse basis function l = sum_k P[k][l] fine basis function k,
    in fine reference units (coarse knots are the even fine knots)."""
    Mc, Mf = 1 << (j - 1), 1 << j
    tc = tuple(2 * v for v in knots(Mc, p))
    tf = knots(Mf, p)
    nbc, nbf = Mc + p, Mf + p
    rows = [dict() for _ in range(nbf)]
    for l in range(nbc):
        lo, hi = tc[l], tc[l + p + 1]
        cw = tuple(v - lo for v in tc[l: l + p + 2])
        # fine functions whose support lies inside the coarse one
        for k in range(max(0, lo), min(nbf, hi + p + 1)):
            if tf[k] < lo or tf[k + p + 1] > hi:
                continue
            a = _oslo(cw, tuple(v - lo for v in tf[k: k + p + 2]), p)
            if a:
                rows[k][l] = a
    keep_f = range(m, nbf - m)
    col0, vals = [], []
    for i in keep_f:
        cols = [l - m for l in rows[i] if m <= l < nbc - m]
        if not cols:
            col0.append(0)
            vals.append([])
            continue
        lo, hi = min(cols), max(cols)
        col0.append(lo)
        vals.append([rows[i].get(lo + m + q, Fraction(0)) for q in range(hi - lo + 1)])
    return Band(len(keep_f), nbc - 2 * m, col0, vals)


# ------------------------------------------------------------- problems ---

def manufactured(kind: str):
    """(u, f) as FP64 callables: Poisson u = sin(pi x); biharmonic
    u = sin(pi x)^2 (u = u' = 0 at both ends), f = u''''."""
    if kind == "poisson":
        return (lambda x: np.sin(np.pi * x), lambda x: np.pi ** 2 * np.sin(np.pi * x))
    if kind == "biharmonic":
        return (lambda x: np.sin(np.pi * x) ** 2,
                lambda x: -8.0 * np.pi ** 4 * np.cos(2.0 * np.pi * x))
    raise ValueError(kind)


def load_vector(kind: str, j: int, p: int) -> np.ndarray:
    """F_hat_i = int_0^M f(h x) B_i(x) dx on the unknowns of level j, FP64,
    Gauss-Legendre with p + 1 nodes per element."""
    m = 1 if kind == "poisson" else 2
    M = 1 << j
    h = 1.0 / M
    _, f = manufactured(kind)
    gx, gw = np.polynomial.legendre.leggauss(p + 1)
    s = 0.5 * (gx + 1.0)
    wq = 0.5 * gw
    F = np.zeros(M + p)
    for e in range(M):
        first, B = element_basis(M, p, e)
        fv = f(h * (e + s))
        for a, poly in enumerate(B):
            c = np.array([float(v) for v in poly])
            bv = np.polyval(c[::-1], s)
            F[first + a] += float(np.dot(wq, fv * bv))
    return F[m: M + p - m].copy()


def solution_values(coef: np.ndarray, kind: str, j: int, p: int, x: np.ndarray) -> np.ndarray:
    """u_h(x) = sum_i c_i B_i(x) for coefficients of the unknowns (FP64)."""
    m = 1 if kind == "poisson" else 2
    M = 1 << j
    full = np.zeros(M + p)
    full[m: M + p - m] = coef
    out = np.zeros_like(x)
    X = x * M
    e = np.minimum(np.floor(X).astype(int), M - 1)
    for idx in range(x.size):
        first, B = element_basis(M, p, int(e[idx]))
        s = X[idx] - e[idx]
        out[idx] = sum(full[first + a] * float(sum(float(c) * s ** q for q, c in enumerate(poly)))
                       for a, poly in enumerate(B))
    return out


# ------------------------------------ reference solutions (FP64) --

def discrete_solution(kind: str, p: int, j: int, iters: int = 40) -> np.ndarray:
    """The coefficients of the exact discrete solution K_hat c = h^(2m) F_hat,
    to FP64 accuracy: banded FP64 solves refined with exactly computed
    residuals (the stiffness entries are exact rationals)."""
    from scipy.linalg import solve_banded
    m = 1 if kind == "poisson" else 2
    K = stiffness(j, p, m)
    rhs = [Fraction(float(v)) * Fraction(2) ** (-2 * m * j) for v in load_vector(kind, j, p)]
    n = K.nrows
    bw = max(max(i - K.col0[i], K.col0[i] + len(K.vals[i]) - 1 - i) for i in range(n))
    ab = np.zeros((2 * bw + 1, n))
    for i in range(n):
        for t, v in enumerate(K.vals[i]):
            k = K.col0[i] + t
            ab[bw + i - k, k] = float(v)
    c = np.zeros(n)
    for _ in range(iters):
        cf = [Fraction(float(v)) for v in c]
        r = [rhs[i] - sum((K.vals[i][t] * cf[K.col0[i] + t] for t in range(len(K.vals[i]))),
                          Fraction(0)) for i in range(n)]
        rf = np.array([float(v) for v in r])
        if not np.any(rf):
            break
        c = c + solve_banded((bw, bw), ab, rf)
    return c


def l2_error(kind: str, p: int, j: int, coef: np.ndarray) -> float:
    """||u - u_h|| in L2(0, 1) for the coefficients of the unknowns, by
    Gauss-Legendre with p + 3 nodes per element."""
    m = 1 if kind == "poisson" else 2
    M = 1 << j
    u, _ = manufactured(kind)
    full = np.zeros(M + p)
    full[m: M + p - m] = coef
    gx, gw = np.polynomial.legendre.leggauss(p + 3)
    s = 0.5 * (gx + 1.0)
    err = 0.0
    for e in range(M):
        first, B = element_basis(M, p, e)
        uh = np.zeros_like(s)
        for a, poly in enumerate(B):
            c = np.array([float(v) for v in poly])
            uh += full[first + a] * np.polyval(c[::-1], s)
        d = u((e + s) / M) - uh
        err += float(np.dot(0.5 * gw, d * d)) / M
    return math.sqrt(err)
