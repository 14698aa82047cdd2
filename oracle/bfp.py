"""The BFP format and its integer primitives (paper Section 2).

A BFP block is the tuple (e, m, w, d): one shared integer exponent e, a block
m of w-bit two's-complement integer mantissas in X_w = [-2^(w-1), 2^(w-1)-1],
laid out as d. It represents the rationals 2^e * m. Right shifts truncate
toward minus infinity (Section 2). Everything here is exact: mantissas are
Python integers (numpy object arrays for blocks), rationals are Fractions.

Parity: pinned by the Figure 2 worked example and the bit-string example of
Section 4 (tests/test_oracle_bfp.py), brute force over small integers and
exact Fraction round trips.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from fractions import Fraction
from typing import Iterable

import numpy as np


# ---------------------------------------------------------------- integers --

def xw_range(w: int) -> tuple[int, int]:
    """Bounds of X_w = [-2^(w-1), 2^(w-1) - 1] (Section 2)."""
    if w < 1:
        raise ValueError("width must be >= 1")
    return -(1 << (w - 1)), (1 << (w - 1)) - 1


def msb(v: int) -> int:
    """Index left of the most significant bit of a two's-complement integer:
    the smallest b >= 1 with v in X_b. msb(0) = msb(-1) = 1; msb(23) = 6 as in
    Figure 2 (bits 0000010111, leading 0 at index 5 is the sign bit)."""
    v = int(v)
    return (v if v >= 0 else ~v).bit_length() + 1


def shr(v: int, k: int) -> int:
    """Arithmetic shift v >> k with floor rounding; a negative k is the exact
    left shift v << -k."""
    v = int(v)
    return v >> k if k >= 0 else v << (-k)


def wrap(v: int, w: int) -> int:
    """decr: keep the w rightmost bits of v and read them as a w-bit
    two's-complement integer (cast to a narrower type). incr (sign
    extension) is the identity on values and needs no function."""
    half = 1 << (w - 1)
    return ((int(v) + half) % (1 << w)) - half


def clamp(v: int, w: int) -> int:
    """Saturate v to X_w."""
    lo, hi = xw_range(w)
    return lo if v < lo else hi if v > hi else int(v)


# ------------------------------------------------------------------ blocks --

def as_block(values: Iterable[int] | np.ndarray) -> np.ndarray:
    """Object array of Python ints (keeps the shape of numpy input)."""
    a = np.asarray(values)
    out = np.empty(a.shape, dtype=object)
    out.flat[:] = [int(x) for x in a.flat]
    return out


_msb_v = np.frompyfunc(msb, 1, 1)
_wrap_v = np.frompyfunc(wrap, 2, 1)
_clamp_v = np.frompyfunc(clamp, 2, 1)
_shr_v = np.frompyfunc(shr, 2, 1)


def block_msb(m: np.ndarray) -> np.ndarray:
    return _msb_v(m) if m.size else np.empty(m.shape, dtype=object)


def block_shr(m: np.ndarray, k: int) -> np.ndarray:
    return _shr_v(m, k) if m.size else m.copy()


def block_wrap(m: np.ndarray, w: int) -> np.ndarray:
    return _wrap_v(m, w) if m.size else m.copy()


def block_clamp(m: np.ndarray, w: int) -> np.ndarray:
    return _clamp_v(m, w) if m.size else m.copy()


def max_msb(m: np.ndarray) -> int:
    """max_i msb(m_i), initialised at 1 as the qcomp loop does (Algorithm 1)."""
    if m.size == 0:
        return 1
    return max(1, int(max(block_msb(m).flat)))


@dataclass
class BFP:
    """BFP block (e, m, w): value = m * 2**e. ``m`` is an object ndarray of
    Python ints whose shape is the layout d."""
    e: int
    m: np.ndarray
    w: int

    def __post_init__(self) -> None:
        self.e = int(self.e)
        self.w = int(self.w)
        if self.m.dtype != object:
            self.m = as_block(self.m)

    def fits(self) -> bool:
        lo, hi = xw_range(self.w)
        return all(lo <= int(v) <= hi for v in self.m.flat)

    def values(self) -> np.ndarray:
        """Exact values as an object array of Fractions."""
        s = Fraction(2) ** self.e
        out = np.empty(self.m.shape, dtype=object)
        out.flat[:] = [Fraction(int(v)) * s for v in self.m.flat]
        return out

    def to_f64(self) -> np.ndarray:
        return np.vectorize(float, otypes=[np.float64])(self.values()) \
            if self.m.size else np.zeros(self.m.shape)

    def norm_inf(self) -> Fraction:
        """||x||_inf = max_i |m_i| * 2^e, exact."""
        if self.m.size == 0:
            return Fraction(0)
        mx = max(abs(int(v)) for v in self.m.flat)
        return Fraction(mx) * Fraction(2) ** self.e

    def copy(self) -> "BFP":
        return BFP(self.e, self.m.copy(), self.w)


@dataclass(frozen=True)
class Scalar:
    """A BFP block of size one (alpha, beta, c1, c2, gamma): value m * 2**e."""
    m: int
    e: int
    w: int

    @property
    def value(self) -> Fraction:
        return Fraction(self.m) * Fraction(2) ** self.e


# ------------------------------------------------------- rationals and nu --

def dyadic_parts(q: Fraction) -> tuple[int, int]:
    """Write a dyadic rational as z * 2**e with integer z (q = n / 2^k)."""
    q = Fraction(q)
    den = q.denominator
    k = den.bit_length() - 1
    if den != 1 << k:
        raise ValueError(f"{q} is not dyadic")
    return q.numerator, -k


def nu(q: Fraction) -> int:
    """Smallest b with -2^(b-1) <= q < 2^(b-1) for a nonzero dyadic q; equals
    msb(z) + e for q = z * 2**e. For q > 0 this is floor(log2 q) + 2."""
    if q == 0:
        raise ValueError("nu(0) is unbounded")
    z, e = dyadic_parts(q)
    return msb(z) + e


def floor_div_pow2(q: Fraction, e: int) -> int:
    """floor(q / 2**e) for a rational q."""
    q = Fraction(q)
    num, den = q.numerator, q.denominator
    if e >= 0:
        den <<= e
    else:
        num <<= -e
    return num // den


def quantize(values: np.ndarray, w: int) -> BFP:
    """Normalized floor quantization Q_w of a block of exact dyadic values:
    e = max_i nu(q_i) - w (minimal exponent, Section 2), m_i = floor(q_i / 2^e).
    An all-zero block gets e = 1 - w (the exponent of a zero result of
    qcomp, which keeps msb(0) = 1)."""
    vals = np.asarray(values, dtype=object)
    nz = [Fraction(v) for v in vals.flat if Fraction(v) != 0]
    e = (max(nu(v) for v in nz) - w) if nz else 1 - w
    out = np.empty(vals.shape, dtype=object)
    out.flat[:] = [floor_div_pow2(Fraction(v), e) for v in vals.flat]
    return BFP(e, out, w)


def from_f64(x: np.ndarray, w: int) -> BFP:
    """quant of FP64 data to w bits (IR / V-cycle / FMG 'quant' with floor
    rounding, Section 2). FP64 values are exact dyadics, so this is Q_w of
    their exact values. Non-finite input is an error."""
    x = np.asarray(x, dtype=np.float64)
    if not np.all(np.isfinite(x)):
        raise ValueError("non-finite FP64 input")
    vals = np.empty(x.shape, dtype=object)
    vals.flat[:] = [Fraction(float(v)) for v in x.flat]
    return quantize(vals, w)


def scalar_from_fraction(q: Fraction, w: int) -> Scalar:
    """Normalized floor quantization of one rational to w bits; exact whenever
    the normalized w-bit mantissa can hold q."""
    q = Fraction(q)
    if q == 0:
        return Scalar(0, 1 - w, w)
    # nu for a general (not necessarily dyadic) rational: the smallest b with
    # -2^(b-1) <= q < 2^(b-1); start below it and walk up (the test is
    # monotone in b)
    b = math.floor(math.log2(abs(q))) - 2
    while not (-Fraction(2) ** (b - 1) <= q < Fraction(2) ** (b - 1)):
        b += 1
    e = b - w
    return Scalar(floor_div_pow2(q, e), e, w)


def scalar_minimal(q: Fraction) -> Scalar:
    """Exact normalized representation of a dyadic rational at its minimal
    width (the smallest w whose normalized mantissa holds q exactly)."""
    z, e = dyadic_parts(Fraction(q))
    if z == 0:
        return Scalar(0, 0, 1)
    while z % 2 == 0:
        z //= 2
        e += 1
    return Scalar(z, e, msb(z))
