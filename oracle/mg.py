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
    trace: list | None = None  # per call: site, level, gamma, exact and output norms
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

    # The operator each call site uses. The finite-difference operators are
    # exact at their minimal width, so quantizing them to a site's width
    # (Algorithms IR, V and FMG quantize A, P and R on entry) changes
    # nothing and one object serves every site; hierarchies whose operators
    # are not exact (oracle.fe) return the site's quantized operator.
    def op_A(self, l: int, site: str):
        return self.A[l]

    def op_R(self, l: int):
        return self.R[l]

    def op_P(self, l: int, site: str):
        return self.P

    def zero(self, l: int, w: int) -> BFP:
        return zero_block(l, self.ndim, w)


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
    if H.trace is not None:
        zm = op.rows()
        exact = Fraction(max((abs(int(v)) for v in zm.flat), default=0)) * Fraction(2) ** op.e
        H.trace.append({"site": site, "level": j + 1 if site == "restrict" else j,
                        "gamma": None if gamma is None else Fraction(gamma),
                        "exact_norm": exact, "out": out,
                        "mode": info.mode, "saturated": info.saturated})
    row = H.stats.diag_row(j + 1 if site == "restrict" else j, site)
    if use_q:
        if gamma is not None and gamma > 0:
            row[gap_bin(nu(Fraction(gamma)) - op.e - info.mu_star)] += 1
    else:
        row[DIAG_NN_CALLS] += 1
        row[DIAG_NN_SAT] += info.saturated
        row[DIAG_NN_SAT_CALLS] += int(info.saturated > 0)
    return out


# One function per call site of Table 1: each forms the exact result of its
# line of Algorithm IR, V or FMG and quantizes it with that row's estimate.

def relaxation(H: Hierarchy, l: int, r: BFP) -> BFP:
    """V relaxation y = c2 A r + c1 r (two Chebyshev steps from y = 0);
    gamma = c1 ||r||, since 0 <= D^-1 A <= 2I bounds ||y|| / ||r|| below c1."""
    s = H.smoother
    return _quantize_op(H, "relax", blas.gemv(H.op_A(l, "relax"), r, r, s.c2, s.c1),
                        H.widths.inner[l], s.c1.value * r.norm_inf())


def v_residual_gamma(H: Hierarchy, r: BFP) -> Fraction:
    """(1/4)(2 c1 + 1) ||r||: the bound 2 c1 + 1 on ||A y - r|| / ||r|| after
    the relaxation, scaled by the empirical 1/4."""
    return H.smoother.vres * r.norm_inf()


def v_residual(H: Hierarchy, l: int, y: BFP, r: BFP, gamma: Fraction) -> BFP:
    """V residual r_v = A y - r at the inner width (gamma from the caller:
    v_residual_gamma before the coarse correction, the latest residual of
    the cycle after it)."""
    return _quantize_op(H, "v_res", blas.gemv(H.op_A(l, "v_res"), y, r, ONE, MINUS_ONE),
                        H.widths.inner[l], gamma)


def restriction(H: Hierarchy, l: int, rv: BFP) -> BFP:
    """Coarse residual R r_v on level l - 1; gamma = ||R|| ||r_v|| (triangle
    inequality). Its width is the inner width of level l, the recursion
    level of the call."""
    return _quantize_op(H, "restrict", blas.spmv(H.op_R(l), rv), H.widths.inner[l],
                        H.op_R(l).norm_inf() * rv.norm_inf())


def v_correction(H: Hierarchy, l: int, y: BFP, d: BFP) -> BFP:
    """y - P d; gamma = ||y|| + ||d|| (nodal interpolation keeps
    ||P d|| = ||d||, then the triangle inequality)."""
    return _quantize_op(H, "v_corr", blas.gemv(H.op_P(l, "v_corr"), d, y, MINUS_ONE, ONE),
                        H.widths.inner[l], y.norm_inf() + d.norm_inf())


def v_update(H: Hierarchy, l: int, y: BFP, z: BFP) -> BFP:
    """y - z of an added smoothing sweep, with the correction's estimate."""
    return _quantize_op(H, "v_corr", blas.sub(y, z), H.widths.inner[l],
                        y.norm_inf() + z.norm_inf())


def ir_residual(H: Hierarchy, l: int, x: BFP, gamma: Fraction | None, first: bool,
                force_q: bool = False) -> BFP:
    """IR residual A x - b at the inner width; gamma is the norm of the
    previous residual (the assumption that the residual does not grow)."""
    r = _quantize_op(H, "ir_res_first" if first else "ir_res",
                     blas.gemv(H.op_A(l, "ir_res"), x, H.b[l], ONE, MINUS_ONE),
                     H.widths.inner[l], gamma, force_q=force_q)
    H.ir_res_saturated = H.stats.last_saturated
    return r


def ir_correction(H: Hierarchy, l: int, x: BFP, y: BFP) -> BFP:
    """x - y at the working width; gamma = ||x|| + ||y|| (triangle
    inequality)."""
    return _quantize_op(H, "ir_corr", blas.sub(x, y), H.widths.work[l],
                        x.norm_inf() + y.norm_inf())


def fmg_prolongation(H: Hierarchy, l: int, x: BFP) -> BFP:
    """P x_(l-1) at the working width of level l; gamma = ||x|| (nodal
    interpolation: ||P x|| = ||x||)."""
    return _quantize_op(H, "fmg_prol", blas.spmv(H.op_P(l, "fmg_prol"), x), H.widths.work[l],
                        x.norm_inf())


def _sweep(H: Hierarchy, l: int, y: BFP, r: BFP, gamma: Fraction) -> tuple[BFP, BFP]:
    """One added smoothing sweep: s = A y - r, z = c2 A s + c1 s, y - z."""
    sres = v_residual(H, l, y, r, gamma)
    z = relaxation(H, l, sres)
    return v_update(H, l, y, z), sres


def vcycle(H: Hierarchy, l: int, r: BFP) -> BFP:
    """V(nu1, nu2) correction scheme on level l for A y = r (nu1 >= 1)."""
    y = relaxation(H, l, r)
    last_res = None
    for _ in range(1, H.nu1):
        y, last_res = _sweep(H, l, y, r, v_residual_gamma(H, r))
    if l > 1:
        rv = v_residual(H, l, y, r, v_residual_gamma(H, r))
        d = vcycle(H, l - 1, restriction(H, l, rv))
        y = v_correction(H, l, y, d)
        last_res = rv
    for _ in range(H.nu2):
        g = last_res.norm_inf() if last_res is not None else v_residual_gamma(H, r)
        y, last_res = _sweep(H, l, y, r, g)
    return y


def ir_iteration(H: Hierarchy, l: int, x: BFP, gamma_res: Fraction | None,
                 force_q: bool = False, first: bool = False) -> tuple[BFP, BFP]:
    """One IR-V iteration on level l: returns (new x, the residual)."""
    r = ir_residual(H, l, x, gamma_res, first, force_q)
    y = vcycle(H, l, r)
    return ir_correction(H, l, x, y), r


def fmg(H: Hierarchy, N: int) -> BFP:
    """FMG(nu1, nu2): coarse-to-fine with N IR-V iterations per level."""
    x = H.zero(1, H.widths.work[1])
    r_last = None
    for l in range(1, H.L + 1):
        if l > 1:
            x = fmg_prolongation(H, l, x)
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
