"""Exact BFP vector and matrix-vector operations (paper Section 4, Appendix B).

Every routine first forms the exact integer result z* (a block with exponent
e_z* and width bound w_z*) through a pair of callbacks — a *setup* giving
(e_z*, w_z*) and a *rows* function giving all mantissas of z* (the parallel
loop over i) — and then quantizes it to w_out bits with either

  qcomp   (Algorithm 1): a normalized, floor-truncated result, exact up to
          w_out bits; ``qcomp`` follows the algorithm with its estimated bit
          window (gamma, w_tmp) and recomputation, ``qcomp_plain`` is the
          result it must reach: e_out = e_z* + mu* - w_out,
          m_i = floor(z*_i / 2^(mu* - w_out)), mu* = max(1, max_i msb(z*_i));
  nnqcomp (Algorithm 3): no normalization — the output exponent comes from the
          estimate gamma alone, entries are floor-shifted and saturated to
          X_w_out.

Operands are BFP blocks (oracle.bfp.BFP) and BFP scalars (oracle.bfp.Scalar);
gamma is an exact rational (Fraction).

Readings taken where the paper is silent (each listed in the design notes):
  * a zero gamma in nnqcomp gives mu_out = 1, i.e. the exponent qcomp gives a
    zero result (e_z* + 1 - w_out); nonzero entries then saturate;
  * qcomp with gamma = 0 (no estimate) takes the plain definition, which is
    what Algorithm 1 returns for every gamma > 0 anyway;
  * ``sub`` (z = x - y) is the axpby row with alpha = 1, beta = -1 written
    out: e_z* = min(e_x, e_y), the operand with the larger exponent is
    shifted left.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from fractions import Fraction
from typing import Callable

import numpy as np

from .bfp import (BFP, Scalar, block_clamp, block_shr, block_wrap, max_msb,
                  nu, xw_range)


def ceil_log2(m: int) -> int:
    return 0 if m <= 1 else (m - 1).bit_length()


@dataclass
class Exact:
    """An exact result waiting to be quantized: exponent e_z*, width bound
    w_z* and the callback computing all rows of its mantissa block."""
    e: int
    w: int
    rows: Callable[[], np.ndarray]


# ------------------------------------------------------------- Appendix B --

def eaxpby_setup(wx: int, ex: int, wy: int, ey: int, alpha: Scalar, beta: Scalar):
    """Exact axpby setup: widths/exponents of alpha*x and beta*y, their
    exponent difference d, and (e_z*, w_z*) of the sum."""
    wa = alpha.w + wx
    wb = beta.w + wy
    ea = alpha.e + ex
    eb = beta.e + ey
    d = ea - eb
    if d < 0:
        wz = max(wa, wb + abs(d)) + 1
    else:
        wz = max(wb, wa + abs(d)) + 1
    return min(ea, eb), wz, d


def eaxpby_rows(xm: np.ndarray, ym: np.ndarray, alpha: Scalar, beta: Scalar,
                d: int) -> np.ndarray:
    """Exact axpby rows: the two exact products, the one with the larger
    exponent shifted left by |d|, then added."""
    a = alpha.m * xm
    b = beta.m * ym
    if d < 0:
        b = b * (1 << -d)
    else:
        a = a * (1 << d)
    return a + b


def axpby(alpha: Scalar, x: BFP, beta: Scalar, y: BFP) -> Exact:
    if x.m.shape != y.m.shape:
        raise ValueError("axpby operands differ in layout")
    ez, wz, d = eaxpby_setup(x.w, x.e, y.w, y.e, alpha, beta)
    return Exact(ez, wz, lambda: eaxpby_rows(x.m, y.m, alpha, beta, d))


def sub(x: BFP, y: BFP) -> Exact:
    """z = x - y: align at min(e_x, e_y) by left-shifting the other operand."""
    if x.m.shape != y.m.shape:
        raise ValueError("sub operands differ in layout")
    d = x.e - y.e
    wz = (max(y.w, x.w + d) if d >= 0 else max(x.w, y.w - d)) + 1

    def rows():
        if d >= 0:
            return x.m * (1 << d) - y.m
        return x.m - y.m * (1 << -d)
    return Exact(min(x.e, y.e), wz, rows)


def spmv(A, x: BFP) -> Exact:
    """Exact SpMV: w_z* = w_A + w_x + ceil(log2 m_A), e_z* = e_A + e_x; row i
    is the exact integer sum over the nonzeros of row i of A."""
    return Exact(A.e + x.e, A.w + x.w + ceil_log2(A.m_A), lambda: A.apply(x.m))


def gemv(A, x: BFP, y: BFP, alpha: Scalar, beta: Scalar) -> Exact:
    """Exact gemv: alpha*A*x + beta*y, composed of the spmv and axpby setups
    and rows exactly as Appendix B composes them."""
    eg = A.e + x.e
    wg = A.w + x.w + ceil_log2(A.m_A)
    ez, wz, d = eaxpby_setup(wg, eg, y.w, y.e, alpha, beta)

    def rows():
        g = A.apply(x.m)
        if g.shape != y.m.shape:
            raise ValueError("gemv: y does not match the output layout of A")
        return eaxpby_rows(g, y.m, alpha, beta, d)
    return Exact(ez, wz, rows)


def identity(x: BFP) -> Exact:
    """The exact 'result' of a copy: used to express normalize and
    saturate/truncate of an existing block through qcomp / nnqcomp."""
    return Exact(x.e, x.w, lambda: x.m.copy())


# ------------------------------------------------- quantizing drivers --

@dataclass
class QInfo:
    """What a quantizing call did: qcomp's overflow / underflow flags and
    recomputation, nnqcomp's number of saturated entries."""
    mode: str
    recomputed: bool = False
    overflow: bool = False
    underflow: bool = False
    saturated: int = 0
    mu_star: int | None = None


def qcomp(op: Exact, w_out: int, w_tmp: int, gamma: Fraction) -> tuple[BFP, QInfo]:
    """Algorithm 1, step by step: estimated window [lambda_tmp, mu_tmp) from
    gamma and w_tmp, one pass storing the windowed temporary (cast to w_tmp
    bits) while tracking mu*, then either a shift of the temporary or, on
    overflow / underflow, a recomputation shifted by lambda_out."""
    if not (0 < w_out <= w_tmp):
        raise ValueError("qcomp needs 0 < w_out <= w_tmp")
    gamma = Fraction(gamma)
    if gamma <= 0:
        raise ValueError("qcomp needs gamma > 0")
    mu_tmp = nu(gamma) - op.e
    lam_tmp = mu_tmp - w_tmp
    zm = op.rows()
    mu_star = max_msb(zm)
    tmp = block_wrap(block_shr(zm, lam_tmp), w_tmp)
    lam_out = mu_star - w_out
    e_out = op.e + lam_out
    overflow = mu_tmp < mu_star
    underflow = lam_out < lam_tmp
    if overflow or underflow:
        zm = op.rows()
        out = block_wrap(block_shr(zm, lam_out), w_out)
    else:
        out = block_wrap(block_shr(tmp, lam_out - lam_tmp), w_out)
    return (BFP(e_out, out, w_out),
            QInfo("q", overflow or underflow, overflow, underflow, 0, mu_star))


def qcomp_plain(op: Exact, w_out: int) -> tuple[BFP, QInfo]:
    """The result Algorithm 1 returns for any gamma and w_tmp: the exact block
    normalized and floor-truncated to w_out bits."""
    if w_out < 1:
        raise ValueError("w_out must be >= 1")
    zm = op.rows()
    mu_star = max_msb(zm)
    lam_out = mu_star - w_out
    return (BFP(op.e + lam_out, block_shr(zm, lam_out), w_out),
            QInfo("q", mu_star=mu_star))


def nnqcomp(op: Exact, w_out: int, gamma: Fraction) -> tuple[BFP, QInfo]:
    """Algorithm 3: mu_out from gamma alone, floor shift, saturation to
    X_w_out; one pass, no maximum over the block."""
    if w_out < 1:
        raise ValueError("w_out must be >= 1")
    gamma = Fraction(gamma)
    if gamma < 0:
        raise ValueError("gamma must be >= 0")
    mu_out = (nu(gamma) - op.e) if gamma != 0 else 1
    lam_out = mu_out - w_out
    zm = block_shr(op.rows(), lam_out)
    lo, hi = xw_range(w_out)
    nsat = sum(1 for v in zm.flat if v < lo or v > hi)
    out = block_clamp(zm, w_out)
    return BFP(op.e + lam_out, out, w_out), QInfo("nn", saturated=nsat)


def nnqcomp_plain(op: Exact, w_out: int, gamma: Fraction) -> BFP:
    """Definition of the nnqcomp result for gamma > 0: e_out =
    floor(log2 gamma) + 2 - w_out, m_i = clamp(floor(value_i / 2^e_out))."""
    gamma = Fraction(gamma)
    e_out = math.floor(math.log2(gamma)) + 2 - w_out
    # correct a possible float rounding of log2 on exact powers of two
    while Fraction(2) ** (e_out + w_out - 2) > gamma:
        e_out -= 1
    while Fraction(2) ** (e_out + w_out - 1) <= gamma:
        e_out += 1
    zm = op.rows()
    lo, hi = xw_range(w_out)
    out = np.empty(zm.shape, dtype=object)
    scale = Fraction(2) ** op.e
    for idx, v in enumerate(zm.flat):
        q = Fraction(int(v)) * scale
        num, den = q.numerator, q.denominator
        if e_out >= 0:
            f = num // (den << e_out)
        else:
            f = (num << -e_out) // den
        out.flat[idx] = min(max(f, lo), hi)
    return BFP(e_out, out, w_out)


# --------------------------------------------------------- other routines --

@dataclass
class DotResult:
    """Exact BFP^1 dot product: mantissa (an arbitrary integer), exponent and
    the width bound w_x + w_y + ceil(log2 n)."""
    m: int
    e: int
    w: int

    @property
    def value(self) -> Fraction:
        return Fraction(self.m) * Fraction(2) ** self.e


def dot(x: BFP, y: BFP) -> DotResult:
    """Exact BFP dot product (Section 2 remark): no alignment shifts, one
    exponent e_x + e_y, an accumulator growing with log2 of the length."""
    if x.m.shape != y.m.shape:
        raise ValueError("dot operands differ in layout")
    s = sum((int(a) * int(b) for a, b in zip(x.m.flat, y.m.flat)), 0)
    return DotResult(s, x.e + y.e, x.w + y.w + ceil_log2(max(1, x.m.size)))


def normalize(x: BFP, w_out: int) -> BFP:
    """Normalized floor re-quantization of a block to w_out bits (qcomp of the
    copy); a zero block gets exponent e_x + 1 - w_out."""
    return qcomp_plain(identity(x), w_out)[0]


def saturate_truncate(x: BFP, w_out: int, gamma: Fraction) -> tuple[BFP, QInfo]:
    """nnqcomp of the copy: exponent from gamma, floor shift, saturation."""
    return nnqcomp(identity(x), w_out, gamma)
