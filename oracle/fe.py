"""BFP multigrid on the paper's finite-element model problems (Section 6).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the bench's
CPU baseline; the product never imports, links or runs anything here.

Set-up S (Appendix C, Algorithm "Setup S to ensure that D = I") applied in
exact rational arithmetic to the stiffness matrices and prolongations of
workloads.fe (K_j = h_j^(1-2m) K_hat_j, F_j = h_j F_hat_j, D_j = diag K_j):
  A_j = D_j^-1 K_j = D_hat_j^-1 K_hat_j,
  b_j = D_j^-1 F_j = 2^(-2mj) F_hat / diag(K_hat_j),
  R_j = D_(j-1)^-1 P_j^T D_j = 2^(2m-1) D_hat_(j-1)^-1 P_j^T D_hat_j.
Unlike the finite-difference operators, these are not dyadic: every call
site quantizes its operator on entry, as Algorithms IR, V and FMG do (A at
the check width in the IR residual; A, P and R at the inner width inside
the V-cycle; P at the working width for the FMG prolongation), each a
normalized floor quantization Q_w of the exact matrix (one exponent for the
whole matrix). The solver is oracle.mg's IR / V / FMG, unchanged.

Readings (listed in the design notes):
  * rho for the Chebyshev coefficients is the Gershgorin bound of A on the
    estimation level min(5, L) — an upper bound of the largest generalized
    eigenvalue (Algorithm Setup S asks for one), exact, computed alike by
    every implementation; eta = 0.23 as for the finite-difference V(1,0);
  * c1, c2 floor-quantized to 16 bits; D = I holds exactly (diag A_j = 1),
    so the stored-operator constants are c1, c2 themselves.
Vectors are 1D blocks of the n_j unknowns with a zero entry at each end
(the padded layout of the other problems).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

from workloads import fe as W

from . import mg
from .bfp import BFP, floor_div_pow2, msb, nu, quantize, scalar_from_fraction


@dataclass
class BandOp:
    """A BFP banded matrix (one exponent e, integer taps): row i holds
    taps[i][t] at column col0[i] + t. apply() maps a padded input block
    (ncols + 2) to a padded output block (nrows + 2) of exact row sums."""
    kind: str
    e: int
    w: int
    m_A: int
    nrows: int
    ncols: int
    col0: list
    taps: list

    def apply(self, xm: np.ndarray) -> np.ndarray:
        if xm.shape != (self.ncols + 2,):
            raise ValueError("input block does not match the matrix")
        out = np.zeros(self.nrows + 2, dtype=object)
        for i in range(self.nrows):
            c = self.col0[i]
            out[i + 1] = sum((t * int(xm[1 + c + k]) for k, t in enumerate(self.taps[i])), 0)
        return out

    def norm_inf(self) -> Fraction:
        return max((Fraction(sum(abs(t) for t in row)) for row in self.taps),
                   default=Fraction(0)) * Fraction(2) ** self.e

    def values(self) -> list:
        s = Fraction(2) ** self.e
        return [[Fraction(t) * s for t in row] for row in self.taps]


def quantize_band(B: W.Band, w: int, kind: str) -> BandOp:
    """Q_w of a banded matrix of exact rationals: e = max nu(entry) - w over
    the nonzero entries, taps = floor(entry / 2^e)."""
    nz = [Fraction(v) for row in B.vals for v in row if v != 0]
    e = (max(nu_rational(v) for v in nz) - w) if nz else 1 - w
    taps = [[floor_div_pow2(Fraction(v), e) for v in row] for row in B.vals]
    wq = max((msb(t) for row in taps for t in row), default=1)
    m_A = max((sum(1 for t in row if t) for row in taps), default=1)
    return BandOp(kind, e, wq, max(m_A, 1), B.nrows, B.ncols, list(B.col0), taps)


def nu_rational(q: Fraction) -> int:
    """Smallest b with -2^(b-1) <= q < 2^(b-1) for a rational q != 0."""
    q = Fraction(q)
    b = math.floor(math.log2(abs(q))) - 2 if q != 0 else 0
    while not (-Fraction(2) ** (b - 1) <= q < Fraction(2) ** (b - 1)):
        b += 1
    return b


def m_of(kind: str) -> int:
    return 1 if kind == "poisson" else 2


def scaled_operators(kind: str, p: int, L: int) -> tuple[dict, dict, dict, dict]:
    """Exact A_j, R_j (j >= 2), P_j (j >= 2) as banded matrices of
    Fractions, and diag(K_hat_j), per Set-up S."""
    m = m_of(kind)
    A, R, P, dg = {}, {}, {}, {}
    for j in range(1, L + 1):
        K = W.stiffness(j, p, m)
        d = [K.vals[i][i - K.col0[i]] for i in range(K.nrows)]
        dg[j] = d
        A[j] = W.Band(K.nrows, K.ncols, list(K.col0),
                      [[v / d[i] for v in K.vals[i]] for i in range(K.nrows)])
    for j in range(2, L + 1):
        Pj = W.prolongation(j, p, m)
        P[j] = Pj
        # R = 2^(2m-1) Dc^-1 P^T Df: row l of R is column l of P, scaled
        cols = [dict() for _ in range(Pj.ncols)]
        for k in range(Pj.nrows):
            for t, v in enumerate(Pj.vals[k]):
                if v:
                    cols[Pj.col0[k] + t][k] = v
        col0, vals = [], []
        scale = Fraction(2) ** (2 * m - 1)
        for l in range(Pj.ncols):
            ks = sorted(cols[l])
            lo, hi = ks[0], ks[-1]
            col0.append(lo)
            vals.append([scale * cols[l].get(k, Fraction(0)) * dg[j][k] / dg[j - 1][l]
                         for k in range(lo, hi + 1)])
        R[j] = W.Band(Pj.ncols, Pj.nrows, col0, vals)
    return A, R, P, dg


def rhs_block(kind: str, p: int, j: int, w: int, diag: list) -> BFP:
    """b_j = Q_w(2^(-2mj) F_hat_i / diag(K_hat_j)_i), the FP64 load vector
    taken as exact dyadics."""
    m = m_of(kind)
    F = W.load_vector(kind, j, p)
    vals = np.zeros(len(F) + 2, dtype=object)
    s = Fraction(2) ** (-2 * m * j)
    for i, v in enumerate(F):
        vals[i + 1] = Fraction(float(v)) * s / diag[i]
    nz = [v for v in vals if v != 0]
    e = (max(nu_rational(v) for v in nz) - w) if nz else 1 - w
    out = np.zeros(len(vals), dtype=object)
    out[:] = [floor_div_pow2(v, e) for v in vals]
    return BFP(e, out, w)


def gershgorin(A: W.Band) -> Fraction:
    return max(sum(abs(v) for v in row) for row in A.vals)


def smoother(kind: str, p: int, L: int, eta: Fraction = Fraction(23, 100)) -> mg.Smoother:
    A, _, _, _ = scaled_operators(kind, p, min(5, L))
    rho = gershgorin(A[min(5, L)])
    c1, c2 = mg.cheby_nodes(rho, eta)
    return mg.Smoother(scalar_from_fraction(c1, 16), scalar_from_fraction(c2, 16),
                       scalar_from_fraction(c1, 16))


class FEHierarchy(mg.Hierarchy):
    """oracle.mg's hierarchy on the finite-element operators, quantized per
    call site."""

    def __post_init__(self) -> None:
        if self.policy not in mg.POLICIES:
            raise ValueError(self.policy)
        self._cache = {}

    def _q(self, which: str, l: int, w: int) -> BandOp:
        key = (which, l, w)
        if key not in self._cache:
            src = {"A": self.Aex, "R": self.Rex, "P": self.Pex}[which][l]
            self._cache[key] = quantize_band(src, w, which)
        return self._cache[key]

    def op_A(self, l: int, site: str) -> BandOp:
        w = self.widths.check[l] if site.startswith("ir_res") else self.widths.inner[l]
        return self._q("A", l, w)

    def op_R(self, l: int) -> BandOp:
        return self._q("R", l, self.widths.inner[l])

    def op_P(self, l: int, site: str) -> BandOp:
        w = self.widths.work[l] if site == "fmg_prol" else self.widths.inner[l]
        return self._q("P", l, w)

    def zero(self, l: int, w: int) -> BFP:
        return BFP(1 - w, np.zeros(self.n[l] + 2, dtype=object), w)


def build(kind: str, p: int, L: int, widths: mg.Widths, policy: str = "q",
          eta: Fraction = Fraction(23, 100)) -> FEHierarchy:
    A, R, P, dg = scaled_operators(kind, p, L)
    b = {j: rhs_block(kind, p, j, widths.check[j], dg[j]) for j in range(1, L + 1)}
    H = FEHierarchy(1, L, widths, smoother(kind, p, L, eta), b, policy=policy)
    H.Aex, H.Rex, H.Pex = A, R, P
    H.n = {j: A[j].nrows for j in range(1, L + 1)}
    return H


def fmg(H: FEHierarchy, N: int) -> BFP:
    return mg.fmg(H, N)
