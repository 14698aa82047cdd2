"""Pins of the tiled-BFP oracle (sub-maximal block sizes, Section 2 Remark
"Block size") against facts fixed outside it: a hand-worked example, block
size 1 as floating point (IEEE bit patterns), the maximal block of
oracle.bfp (pinned by the paper's Figure 2), the refinement property the
remark states (a maximal block is the worst case for quantization), and the
exact gemv rows of oracle.blas."""
from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import bfp, blas, fd, tiles
from oracle.bfp import Scalar

GOLD = os.path.join(os.path.dirname(__file__), "golden", "tiles_example.json")


def padded(vals, ndim, n):
    out = np.zeros((n + 2,) * ndim, dtype=object)
    out[(slice(1, -1),) * ndim] = vals
    return out


def rand_values(g, shape, spread=20):
    v = np.empty(shape, dtype=object)
    v.flat[:] = [Fraction(int(g.integers(-2 ** 20, 2 ** 20)), 1) * Fraction(2) ** int(g.integers(-spread, spread))
                 for _ in range(int(np.prod(shape)))]
    return v


def test_hand_worked_example():
    gold = json.load(open(GOLD))
    n = gold["n"]
    vals = np.array([[Fraction(s) for s in row] for row in gold["values"]], dtype=object)
    t = tiles.quantize(padded(vals, 2, n), 2, n, gold["T"], gold["w"])
    assert t.e.tolist() == gold["exponents"]
    assert [[int(v) for v in row] for row in t.m[1:-1, 1:-1]] == gold["mantissas"]
    assert t.m[0, :].tolist() == [0] * (n + 2)


def test_block_size_one_is_floating_point():
    """T = 1 with w >= 54 holds every FP64 value exactly; with w = 25 a
    positive normal value becomes its double with the 29 lowest stored
    significand bits cleared (rounding toward zero to a 24-bit significand,
    which is the floor for positive values)."""
    g = np.random.default_rng(3)
    x = np.zeros((9, 9))
    x[1:-1, 1:-1] = g.standard_normal((7, 7)) * 10.0 ** g.integers(-30, 30, (7, 7))
    t = tiles.from_f64(x, 1, 54)
    assert np.array_equal(t.to_f64(), x)
    xp = np.abs(x)
    t = tiles.from_f64(xp, 1, 25)
    bits = xp.view(np.int64) & ~np.int64((1 << 29) - 1)
    want = bits.view(np.float64)
    want[0, :] = want[-1, :] = want[:, 0] = want[:, -1] = 0
    assert np.array_equal(t.to_f64(), want)


def test_negative_values_round_toward_minus_infinity():
    # w = 3: X_3 = [-4, 3]; -4 is exact (e = 0), -5 -> floor(-5/2) 2 = -6
    vals = np.array([[Fraction(-4), Fraction(-5)]], dtype=object)
    g = np.zeros((4, 4), dtype=object)
    g[1, 1:3] = vals
    t = tiles.quantize(g, 2, 2, 1, 3)
    assert t.values()[1, 1] == -4 and t.values()[1, 2] == -6


@pytest.mark.parametrize("ndim,n", [(2, 13), (3, 5)])
def test_smaller_blocks_never_quantize_worse(ndim, n):
    """Pointwise |Q_T(v) - v| <= |Q_2T(v) - v| <= |Q_maximal(v) - v|."""
    g = np.random.default_rng(ndim * 10 + n)
    vals = padded(rand_values(g, (n,) * ndim), ndim, n)
    big = bfp.quantize(vals, 11).values()
    prev = None
    for T in (64, 16, 8, 4, 2, 1):
        err = np.abs(tiles.quantize(vals, ndim, n, T, 11).values() - vals)
        assert all(a <= b for a, b in zip(err.flat, np.abs(big - vals).flat))
        if prev is not None:
            assert all(a <= b for a, b in zip(err.flat, prev.flat))
        prev = err


def test_row_tiles_with_a_common_scale_equal_the_maximal_block():
    """When every row reaches the block's largest nu, row-long tiles share
    the maximal block's exponent and mantissas."""
    g = np.random.default_rng(5)
    n = 6
    v = rand_values(g, (n, n), spread=3)
    for r in range(n):
        v[r, r] = Fraction(2 ** 40)   # nu = 42 in every row
    vals = padded(v, 2, n)
    big = bfp.quantize(vals, 17)
    t = tiles.quantize(vals, 2, n, 8, 17)
    assert set(t.e.flat) == {big.e}
    assert all(int(a) == int(b) for a, b in zip(t.m.flat, big.m.flat))


def to_single_block(t: tiles.Tiled) -> bfp.BFP:
    """The same values with one exponent (exact: mantissas shifted left)."""
    E = int(t.e.min())
    m = np.zeros(t.m.shape, dtype=object)
    for p in tiles.interior(t.ndim, t.n):
        m[p] = int(t.m[p]) << (t.tile_exp(p) - E)
    w = max(bfp.max_msb(m), 1)
    return bfp.BFP(E, m, w)


@pytest.mark.parametrize("ndim,n,T,with_y", [(2, 11, 4, True), (2, 9, 1, False), (3, 5, 2, True),
                                              (2, 7, 16, True)])
def test_stencil_matches_the_maximal_block_gemv(ndim, n, T, with_y):
    g = np.random.default_rng(ndim * 100 + n + T)
    A = fd.scaled_A(3, ndim)
    x = tiles.quantize(padded(rand_values(g, (n,) * ndim, 12), ndim, n), ndim, n, T, 13)
    y = tiles.quantize(padded(rand_values(g, (n,) * ndim, 12), ndim, n), ndim, n, T, 9)
    alpha, beta = Scalar(-3, 2, 4), Scalar(5, -7, 5)
    z, bad = tiles.stencil_apply(A, x, alpha, beta if with_y else None, y if with_y else None, 10)
    assert bad == 0
    xb, yb = to_single_block(x), to_single_block(y)
    zero = bfp.BFP(0, np.zeros(xb.m.shape, dtype=object), 1)
    ex = blas.gemv(A, xb, yb if with_y else zero, alpha, beta if with_y else Scalar(0, 0, 1))
    rows = ex.rows()
    exact = np.zeros(rows.shape, dtype=object)
    for p in tiles.interior(ndim, n):
        exact[p] = Fraction(int(rows[p])) * Fraction(2) ** ex.e
    ref = tiles.quantize(exact, ndim, n, T, 10)
    assert np.array_equal(ref.e, z.e)
    assert all(int(a) == int(b) for a, b in zip(ref.m.flat, z.m.flat))


def test_axpby_matches_the_maximal_block_axpby():
    g = np.random.default_rng(8)
    n, T = 10, 4
    x = tiles.quantize(padded(rand_values(g, (n, n), 15), 2, n), 2, n, T, 12)
    y = tiles.quantize(padded(rand_values(g, (n, n), 15), 2, n), 2, n, T, 7)
    alpha, beta = Scalar(7, -1, 4), Scalar(-3, 3, 3)
    z, bad = tiles.axpby(alpha, x, beta, y, 9)
    assert bad == 0
    ex = blas.axpby(alpha, to_single_block(x), beta, to_single_block(y))
    rows = ex.rows()
    exact = np.zeros(rows.shape, dtype=object)
    for p in tiles.interior(2, n):
        exact[p] = Fraction(int(rows[p])) * Fraction(2) ** ex.e
    ref = tiles.quantize(exact, 2, n, T, 9)
    assert np.array_equal(ref.e, z.e)
    assert all(int(a) == int(b) for a, b in zip(ref.m.flat, z.m.flat))


def test_exponent_spread_beyond_the_exact_range_is_counted():
    """n = 3, T = 1, every tile at exponent 0 except the centre at 100: the
    centre and its four star neighbours draw on both exponents (spread 100 >
    60), the four corners do not; those five points are zero."""
    n = 3
    m = np.zeros((5, 5), dtype=object)
    m[1:-1, 1:-1] = 1
    e = np.zeros((3, 3), dtype=np.int64)
    e[1, 1] = 100
    x = tiles.Tiled(2, n, 1, 8, e, m)
    A = fd.scaled_A(2, 2)
    z, bad = tiles.stencil_apply(A, x, Scalar(1, 0, 2), None, None, 8)
    assert bad == 5
    vals = z.values()
    assert all(vals[p] == 0 for p in [(1, 2), (2, 1), (2, 2), (2, 3), (3, 2)])
    assert all(vals[p] != 0 for p in [(1, 1), (1, 3), (3, 1), (3, 3)])
