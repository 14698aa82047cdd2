"""BFP multigrid: iterative refinement, V-cycle and full multigrid (paper
Section 5 and Appendix C), with the Table 1 estimates gamma / w_add.

Structure (with D = I after setup S, see oracle.fd):
  IR      r <- qgemv(A, x, b, 1, -1) at the inner width;  y <- V(r);
          x <- qsub(x, y) at the working width.
  V       y <- qgemv(A, r, r, c2, c1)      (two Chebyshev steps from y = 0)
          if l > 1: r_v <- qgemv(A, y, r, 1, -1); r_c <- qspmv(R, r_v);
                    d <- V(l - 1, r_c);  y <- qgemv(P, d, y, -1, 1)
          all outputs of V on level l at the inner width of level l.
  FMG     x <- 0 on level 1, x <- qspmv(P, x_coarse) at the working width on
          finer levels, then N IR-V iterations per level.

Readings where the paper is silent or the configurations ask for more:
  * V(nu1, nu2): pre-sweep 1 is the zero-start relaxation above; every other
    sweep is s <- qgemv(A, y, r, 1, -1); z <- qgemv(A, s, s, c2, c1);
    y <- qsub(y, z), each step quantized on its own. Estimates for the added
    steps: the residual uses the V-residual rule before the coarse
    correction and the most recent residual of the cycle after it, the
    increment the relaxation rule, the update the V-correction rule.
  * The FMG calls IR once per iteration (the goto loop with tol = -1 is read
    as "one IR-V iteration per call", N calls per level).
  * The i = 1 IR residual estimate ||r_{l-1}^(N)|| is the last residual
    computed on the next coarser FMG level; on level 1 (x = 0) it is ||b||.
  * Estimates that do not exist (IR from a given initial guess, first
    iteration) make that call use qcomp.
  * Widths: fixed (one w for everything) or progressive: working
    w_j = min(32, 2j + 8), inner w_j = min(working, max(5, w - (L - j)))
    with w the finest inner width, A and b at 32 bits.
  * c1, c2 floor-quantized to 16 bits; rho = 2 (the Gershgorin bound for
    diag-scaled 5- and 7-point operators, valid on every level).

Diagnostics (Section 4's window and Table 2; Section 6.4's saturation): per
recursion level (the input's level for a restriction, the output's
otherwise) and call site, 64 counters. A qcomp call with an estimate gamma
counts its window gap d = mu_tmp - mu*, mu_tmp = nu(gamma) - e_z* the top
of the window the estimate gives and mu* the exact result's leading bit:
bin 0 for d < 0, bin 1 + min(d, 59) otherwise. Algorithm 1 with
w_tmp = w_out + w_add recomputes exactly when d < 0 (overflow) or
d > w_add (underflow), so one histogram answers every w_add of a Table 2
sweep. An nnqcomp call counts in bin 61, its saturated entries in bin 62,
and in bin 63 if it saturated any.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction
from typing import Callable

import numpy as np

from . import blas
from .bfp import BFP, Scalar, as_block, nu, quantize, scalar_from_fraction
from .fd import Stencil, prolongation, rhs_log2_scale, scaled_A, scaled_R

ONE = Scalar(1, 0, 2)
MINUS_ONE = Scalar(-1, 0, 1)

# call sites, in the order of the diagnostics rows
SITES = ("ir_res_first", "ir_res", "ir_corr", "relax", "v_res", "restrict", "v_corr",
         "fmg_prol")
DIAG_BINS, DIAG_GAP_BINS = 64, 61
DIAG_NN_CALLS, DIAG_NN_SAT, DIAG_NN_SAT_CALLS = 61, 62, 63


def gap_bin(d: int) -> int:
    """Diagnostics bin of a qcomp window gap d = mu_tmp - mu*."""
    return 0 if d < 0 else 1 + min(d, DIAG_GAP_BINS - 2)


def recomputations(row, w_add: int) -> int:
    """Calls of a diagnostics row that Algorithm 1 with w_tmp = w_out + w_add
    recomputes: overflow (d < 0) or underflow (d > w_add)."""
    return int(row[0]) + sum(int(row[1 + d]) for d in range(w_add + 1, DIAG_GAP_BINS - 1))


# Table 1: extra window bits w_add per call site (used by qcomp's window).
W_ADD = {
    "ir_res_first": 5, "ir_res": 4, "ir_corr": 0, "relax": 2, "v_res": 4,
    "restrict": 6, "v_corr": 1, "fmg_prol": 0,
}


# ------------------------------------------------------------ parameters --

def cheby_nodes(rho: Fraction, eta: Fraction) -> tuple[Fraction, Fraction]:
    """Coefficients for two Chebyshev iterations (Appendix C), exact."""
    rho = Fraction(rho)
    eta = Fraction(eta)
    if not (0 < eta < 1):
        raise ValueError("need 0 < eta < 1")
    alpha = (1 + eta) * rho / 2
    c = (1 - eta) * rho / 2
    beta = alpha - c * c / (2 * alpha)
    return 2 / beta, -1 / (alpha * beta)


@dataclass(frozen=True)
class Smoother:
    """Quantized relaxation constants. (c1, c2) multiply r and A r in the
    relaxation qgemv; ``c1_gamma`` is the D-scaled c1 used in the V-residual
    estimate (2 c1 + 1)/4, ``vres`` that estimate's exact constant."""
    c1: Scalar
    c2: Scalar
    c1_gamma: Scalar

    @property
    def vres(self) -> Fraction:
        return (2 * self.c1_gamma.value + 1) / 4


def make_smoother(ndim: int, eta: Fraction, rho: Fraction = Fraction(2),
                  w_c: int = 16) -> Smoother:
    """c1, c2 from ChebyshevNodes for D^-1 A, rescaled to the operator
    actually stored (A' = a_c D^-1 A with a_c = diag(A') = 1 in 2D, 3/4 in 3D
    gives c1' = c1 / a_c, c2' = c2 / a_c^2), each floor-quantized to w_c bits."""
    c1, c2 = cheby_nodes(rho, eta)
    a_c = Fraction(1) if ndim == 2 else Fraction(3, 4)
    return Smoother(scalar_from_fraction(c1 / a_c, w_c),
                    scalar_from_fraction(c2 / (a_c * a_c), w_c),
                    scalar_from_fraction(c1, w_c))


@dataclass(frozen=True)
class Widths:
    """Per-level mantissa widths: check (A, b), work (x), inner (V-cycle)."""
    check: dict
    work: dict
    inner: dict


def widths_fixed(L: int, w: int) -> Widths:
    d = {j: w for j in range(1, L + 1)}
    return Widths(dict(d), dict(d), dict(d))


def widths_progressive(L: int, w: int, k: int = 2, c: int = 8, floor: int = 5,
                       cap: int = 32, check: int = 32) -> Widths:
    """Working widths grow by k bits per level, inner widths by one bit per
    level (m = 1), ordered check >= work >= inner as the three precisions
    are (Section 5)."""
    work = {j: min(cap, k * j + c) for j in range(1, L + 1)}
    inner = {j: min(work[j], max(floor, w - (L - j))) for j in range(1, L + 1)}
    return Widths({j: check for j in range(1, L + 1)}, work, inner)


# --------------------------------------------------------------- policies --

# q               qcomp for every call
# nn              nnqcomp for every call (Section 6.4 as printed)
# nn_ir_first_q   qcomp for the first IR residual of every level (each FMG
#                 level and the first IR-V iteration of a plain solve)
# nn_ir_first2_q  qcomp for the first two IR residuals of a plain IR-V solve
#                 (Remark on skipping normalization in IR-V) and for the
#                 first IR residual of each FMG level
# nn_ir_q         qcomp for every IR residual
POLICIES = ("q", "nn", "nn_ir_first_q", "nn_ir_first2_q", "nn_ir_q")


@dataclass
class Stats:
    calls: int = 0
    q_calls: int = 0
    recomputations: int = 0
    saturations: int = 0
    per_site: dict = field(default_factory=dict)
    diag: dict = field(default_factory=dict)     # (level, site index) -> 64 counters

    def diag_row(self, level: int, site: str) -> list:
        key = (level, SITES.index(site))
        if key not in self.diag:
            self.diag[key] = [0] * DIAG_BINS
        return self.diag[key]

    def diag_array(self, max_level: int = 16) -> np.ndarray:
        """The counters as [level 0..max_level][site][bin] (row 0 unused)."""
        a = np.zeros((max_level + 1, len(SITES), DIAG_BINS), dtype=np.int64)
        for (level, k), row in self.diag.items():
            a[level, k] = row
        return a

    last_saturated: int = 0      # entries the most recent call saturated

    def add(self, site: str, info: blas.QInfo) -> None:
        self.last_saturated = info.saturated
        self.calls += 1
        self.per_site[site] = self.per_site.get(site, 0) + 1
        if info.mode == "q":
            self.q_calls += 1
        self.recomputations += int(info.recomputed)
        self.saturations += info.saturated


@dataclass
class Hierarchy:
    """Everything the solver needs for levels 1..L of one problem."""
    ndim: int
    L: int
    widths: Widths
    smoother: Smoother
    b: dict                    # level -> BFP right-hand side at check width
    policy: str = "nn"
    nu1: int = 1
    nu2: int = 0
    window: bool = True        # qcomp with the Table 1 window (else plain)
    ir_res_saturated: int = 0  # entries the last IR residual saturated
    stats: Stats = field(default_factory=Stats)
    A: dict = field(default_factory=dict)
    R: dict = field(default_factory=dict)
    P: Stencil | None = None

    def __post_init__(self) -> None:
        for j in range(1, self.L + 1):
            self.A[j] = scaled_A(j, self.ndim)
            if j > 1:
                self.R[j] = scaled_R(j, self.ndim)
        self.P = prolongation(self.ndim)
        if self.policy not in POLICIES:
            raise ValueError(self.policy)


def rhs_block(f: np.ndarray, j: int, ndim: int, w: int) -> BFP:
    """b'_j = quant(f / s_j) at w bits: the exact FP64 samples of f scaled by
    the power of two 1/s_j, then normalized floor quantization."""
    x = np.asarray(f, dtype=np.float64)
    k = rhs_log2_scale(j, ndim)
    vals = np.empty(x.shape, dtype=object)
    vals.flat[:] = [Fraction(float(v)) * Fraction(2) ** k for v in x.flat]
    return quantize(vals, w)


def build_hierarchy(f_levels: dict, ndim: int, L: int, widths: Widths,
                    smoother: Smoother, **kw) -> Hierarchy:
    b = {j: rhs_block(f_levels[j], j, ndim, widths.check[j]) for j in range(1, L + 1)}
    return Hierarchy(ndim, L, widths, smoother, b, **kw)


def zero_block(j: int, ndim: int, w: int) -> BFP:
    n = (1 << j) + 1
    return BFP(1 - w, np.zeros((n,) * ndim, dtype=object), w)


# ---------------------------------------------------------------- solver --

def _quantize_op(H: Hierarchy, site: str, op: blas.Exact, w_out: int,
                 gamma: Fraction | None, force_q: bool = False) -> BFP:
    """Quantize one exact result by the hierarchy's policy: nnqcomp with the
    site's gamma, or qcomp (windowed with Table 1's w_add when an estimate
    exists, the plain definition otherwise — both give the same block)."""
    use_q = (force_q or H.policy == "q" or gamma is None
             or (site == "ir_res_first" and H.policy in ("nn_ir_first_q", "nn_ir_first2_q"))
             or (site.startswith("ir_res") and H.policy == "nn_ir_q"))
    if use_q:
        if H.window and gamma is not None and gamma > 0:
            base = "ir_res" if site.startswith("ir_res") else site
            w_add = W_ADD.get(site, W_ADD.get(base, 0))
            out, info = blas.qcomp(op, w_out, w_out + w_add, gamma)
        else:
            out, info = blas.qcomp_plain(op, w_out)
    else:
        out, info = blas.nnqcomp(op, w_out, gamma)
    H.stats.add(site, info)
    # diagnostics, on the recursion level of the call
    j = (out.m.shape[0] - 1).bit_length() - 1
    row = H.stats.diag_row(j + 1 if site == "restrict" else j, site)
    if use_q:
        if gamma is not None and gamma > 0:
            row[gap_bin(nu(Fraction(gamma)) - op.e - info.mu_star)] += 1
    else:
        row[DIAG_NN_CALLS] += 1
        row[DIAG_NN_SAT] += info.saturated
        row[DIAG_NN_SAT_CALLS] += int(info.saturated > 0)
    return out


def relax_sweep_from_zero(H: Hierarchy, l: int, r: BFP) -> BFP:
    s = H.smoother
    return _quantize_op(H, "relax", blas.gemv(H.A[l], r, r, s.c2, s.c1),
                        H.widths.inner[l], s.c1.value * r.norm_inf())


def vcycle(H: Hierarchy, l: int, r: BFP) -> BFP:
    """V(nu1, nu2) correction scheme on level l for A y = r (nu1 >= 1)."""
    w = H.widths.inner[l]
    s = H.smoother
    A = H.A[l]
    y = relax_sweep_from_zero(H, l, r)
    last_res = None
    for _ in range(1, H.nu1):
        sres = _quantize_op(H, "v_res", blas.gemv(A, y, r, ONE, MINUS_ONE), w,
                            s.vres * r.norm_inf())
        z = _quantize_op(H, "relax", blas.gemv(A, sres, sres, s.c2, s.c1), w,
                         s.c1.value * sres.norm_inf())
        y = _quantize_op(H, "v_corr", blas.sub(y, z), w, y.norm_inf() + z.norm_inf())
        last_res = sres
    if l > 1:
        rv = _quantize_op(H, "v_res", blas.gemv(A, y, r, ONE, MINUS_ONE), w,
                          s.vres * r.norm_inf())
        rc = _quantize_op(H, "restrict", blas.spmv(H.R[l], rv), w,
                          H.R[l].norm_inf() * rv.norm_inf())
        d = vcycle(H, l - 1, rc)
        y = _quantize_op(H, "v_corr", blas.gemv(H.P, d, y, MINUS_ONE, ONE), w,
                         y.norm_inf() + d.norm_inf())
        last_res = rv
    for _ in range(H.nu2):
        g = last_res.norm_inf() if last_res is not None else s.vres * r.norm_inf()
        sres = _quantize_op(H, "v_res", blas.gemv(A, y, r, ONE, MINUS_ONE), w, g)
        z = _quantize_op(H, "relax", blas.gemv(A, sres, sres, s.c2, s.c1), w,
                         s.c1.value * sres.norm_inf())
        y = _quantize_op(H, "v_corr", blas.sub(y, z), w, y.norm_inf() + z.norm_inf())
        last_res = sres
    return y


def ir_iteration(H: Hierarchy, l: int, x: BFP, gamma_res: Fraction | None,
                 force_q: bool = False, first: bool = False) -> tuple[BFP, BFP]:
    """One IR-V iteration on level l: returns (new x, the residual)."""
    r = _quantize_op(H, "ir_res_first" if first else "ir_res",
                     blas.gemv(H.A[l], x, H.b[l], ONE, MINUS_ONE),
                     H.widths.inner[l], gamma_res, force_q=force_q)
    H.ir_res_saturated = H.stats.last_saturated
    y = vcycle(H, l, r)
    xn = _quantize_op(H, "ir_corr", blas.sub(x, y), H.widths.work[l],
                      x.norm_inf() + y.norm_inf())
    return xn, r


def fmg(H: Hierarchy, N: int) -> BFP:
    """FMG(nu1, nu2): coarse-to-fine with N IR-V iterations per level."""
    x = zero_block(1, H.ndim, H.widths.work[1])
    r_last = None
    for l in range(1, H.L + 1):
        if l > 1:
            x = _quantize_op(H, "fmg_prol", blas.spmv(H.P, x), H.widths.work[l],
                             x.norm_inf())
            g_first = r_last.norm_inf()
        else:
            g_first = H.b[1].norm_inf()
        r = None
        for i in range(1, N + 1):
            g = g_first if i == 1 else r.norm_inf()
            x, r = ir_iteration(H, l, x, g, first=(i == 1))
        r_last = r
    return x


def ir_solve_safe(H: Hierarchy, x0: BFP, iters: int, q_iters: int = 2,
                  theta: Fraction = Fraction(1)) -> tuple[BFP, list, int]:
    """IR-V with the safety mechanism of Section 6.4: an iterative solver that
    skips normalization watches the residual, and when convergence stalls it
    runs Algorithm 1 (qcomp) for some operations during some iterations.
    Here: after an iteration whose IR residual saturated (nnqcomp's estimate
    was too small) or whose residual norm exceeds theta times the previous
    one, the IR residuals of the next q_iters iterations use qcomp. Returns
    (x, residual history, iterations that ran the fallback)."""
    x = x0
    r = None
    history = []
    force = 0
    switched = 0
    prev = None
    for i in range(1, iters + 1):
        g = None if r is None else r.norm_inf()
        fallback = force > 0
        force_q = fallback or (H.policy == "nn_ir_first2_q" and i <= 2)
        x, r = ir_iteration(H, H.L, x, g, force_q=force_q, first=(i == 1))
        if fallback:
            switched += 1
            force -= 1
        n = r.norm_inf()
        if H.ir_res_saturated > 0 or (prev is not None and n > Fraction(theta) * prev):
            force = q_iters
        prev = n
        history.append(r)
    return x, history, switched


def ir_solve(H: Hierarchy, x0: BFP, iters: int) -> tuple[BFP, list]:
    """IR-V(nu1, nu2) on the finest level from a given initial guess. The
    first two residuals use qcomp under the 'nn_ir_first2_q' policy (Remark
    on skipping normalization in IR-V); the first has no estimate."""
    x = x0
    r = None
    history = []
    for i in range(1, iters + 1):
        g = None if r is None else r.norm_inf()
        force_q = H.policy == "nn_ir_first2_q" and i <= 2
        x, r = ir_iteration(H, H.L, x, g, force_q=force_q, first=(i == 1))
        history.append(r)
    return x, history
