"""Pins of the BFP format primitives (Section 2 and Figure 2)."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import bfp
from oracle.bfp import BFP, from_f64, msb, quantize, shr, wrap, clamp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _xw(v, b):
    return -(2 ** (b - 1)) <= v <= 2 ** (b - 1) - 1


def test_msb_brute_force():
    for v in range(-600, 601):
        b = 1
        while not _xw(v, b):
            b += 1
        assert msb(v) == b, v
    assert msb(0) == 1 and msb(-1) == 1 and msb(1) == 2 and msb(-2) == 2


def test_figure2_msb_and_window():
    g = json.load(open(os.path.join(GOLDEN, "fig2_windows.json")))
    v = int(g["bits"], 2)
    assert v == g["value"]
    assert msb(v) == g["mu_star"]
    lam = g["mu_star"] - g["w_out"]
    assert lam == g["lambda_out"]
    out = shr(v, lam)
    assert format(out, f"0{g['w_out']}b") == g["out_bits"]
    # the window's leading bit is the sign bit of the 4-bit result
    assert _xw(out, g["w_out"]) and not _xw(out, g["w_out"] - 1)


def test_bitstring_example():
    g = json.load(open(os.path.join(GOLDEN, "bitstring_example.json")))
    v = int(g["bits"], 2)
    sub = (v >> g["lambda"]) & ((1 << (g["mu"] - g["lambda"])) - 1)
    assert format(sub, f"0{g['width']}b") == g["substring"]
    assert g["mu"] - g["lambda"] == g["width"]


def test_shift_is_floor():
    for v in range(-70, 71):
        for k in range(0, 9):
            assert shr(v, k) == math.floor(Fraction(v, 2 ** k))
            assert shr(v, -k) == v * 2 ** k


def test_wrap_and_clamp_brute():
    for w in range(1, 7):
        lo, hi = -(2 ** (w - 1)), 2 ** (w - 1) - 1
        for v in range(-100, 101):
            r = wrap(v, w)
            assert lo <= r <= hi and (r - v) % (2 ** w) == 0
            c = clamp(v, w)
            assert c == min(max(v, lo), hi)


@settings(max_examples=150, deadline=None)
@given(st.lists(st.tuples(st.integers(-10 ** 12, 10 ** 12), st.integers(-80, 80)),
                min_size=1, max_size=8),
       st.integers(1, 40))
def test_quantize_is_minimal_floor(pairs, w):
    vals = np.empty(len(pairs), dtype=object)
    vals[:] = [Fraction(z) * Fraction(2) ** e for z, e in pairs]
    q = quantize(vals, w)
    assert q.fits()
    if all(v == 0 for v in vals):
        assert q.e == 1 - w and all(m == 0 for m in q.m)
        return
    two = Fraction(2)
    for v, m in zip(vals, q.m):
        assert m * two ** q.e <= v < (m + 1) * two ** q.e
    # minimality: one exponent lower does not fit in w bits
    lower = [math.floor(v / two ** (q.e - 1)) for v in vals]
    assert not all(_xw(m, w) for m in lower)


@settings(max_examples=100, deadline=None)
@given(st.lists(st.floats(allow_nan=False, allow_infinity=False, width=64),
                min_size=1, max_size=6), st.integers(1, 32))
def test_from_f64_exact(xs, w):
    x = np.asarray(xs, dtype=np.float64)
    q = from_f64(x, w)
    assert q.fits()
    two = Fraction(2)
    for v, m in zip(xs, q.m):
        fv = Fraction(v)
        assert m * two ** q.e <= fv < (m + 1) * two ** q.e


def test_from_f64_rejects_nonfinite():
    with pytest.raises(ValueError):
        from_f64(np.array([1.0, np.nan]), 8)


def test_nu_matches_log2():
    for z in range(1, 300):
        for e in (-5, 0, 7):
            q = Fraction(z) * Fraction(2) ** e
            assert bfp.nu(q) == math.floor(math.log2(q)) + 2
            # negative values: smallest b with -2^(b-1) <= q
            b = bfp.nu(-q)
            assert -Fraction(2) ** (b - 1) <= -q and not (-Fraction(2) ** (b - 2) <= -q)


def test_scalar_quantization():
    s = bfp.scalar_from_fraction(Fraction(1, 3), 16)
    assert -(2 ** 15) <= s.m < 2 ** 15
    assert s.value <= Fraction(1, 3) < s.value + Fraction(2) ** s.e
    assert s.m >= 2 ** 14  # normalized
    assert bfp.scalar_minimal(Fraction(-1, 4)) == bfp.Scalar(-1, -2, 1)
    assert bfp.scalar_minimal(Fraction(3, 4)) == bfp.Scalar(3, -2, 3)
