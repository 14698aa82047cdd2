"""Pins of the exact BFP routines, qcomp (Algorithm 1) and nnqcomp
(Algorithm 3) against exact rational arithmetic and the paper's invariants."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import blas, fd
from oracle.bfp import BFP, Scalar, msb, xw_range

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TWO = Fraction(2)


def vec(ms, e, w):
    a = np.empty(len(ms), dtype=object)
    a[:] = [int(v) for v in ms]
    return BFP(e, a, w)


def exact_values(op):
    return [Fraction(int(v)) * TWO ** op.e for v in op.rows().flat]


def q_reference(values, w_out, e_star):
    """qcomp's result recomputed from exact rationals: the smallest exponent
    whose floor quantization fits w_out bits (zero block: e_z* + 1 - w)."""
    nz = [v for v in values if v != 0]
    if not nz:
        return e_star + 1 - w_out, [0] * len(values)
    e = e_star - 200
    lo, hi = xw_range(w_out)
    while not all(lo <= math.floor(v / TWO ** e) <= hi for v in values):
        e += 1
    return e, [math.floor(v / TWO ** e) for v in values]


def nn_reference(values, w_out, gamma):
    k = math.floor(math.log2(gamma))
    while TWO ** k > gamma:
        k -= 1
    while TWO ** (k + 1) <= gamma:
        k += 1
    e = k + 2 - w_out
    lo, hi = xw_range(w_out)
    return e, [min(max(math.floor(v / TWO ** e), lo), hi) for v in values]


mant = st.integers(-(2 ** 31), 2 ** 31 - 1)


def rand_block(draw_list, e, w):
    lo, hi = xw_range(w)
    return vec([min(max(v, lo), hi) for v in draw_list], e, w)


# ------------------------------------------------------ exact operations --

@settings(max_examples=120, deadline=None)
@given(st.lists(mant, min_size=1, max_size=6), st.lists(mant, min_size=6, max_size=6),
       st.integers(1, 32), st.integers(1, 32), st.integers(-60, 60), st.integers(-60, 60),
       st.integers(-300, 300), st.integers(-300, 300), st.integers(-20, 20), st.integers(-20, 20))
def test_axpby_exact(xs, ys, wx, wy, ex, ey, am, bm, ae, be):
    n = len(xs)
    x = rand_block(xs, ex, wx)
    y = rand_block(ys[:n], ey, wy)
    alpha = Scalar(am, ae, max(1, msb(am)))
    beta = Scalar(bm, be, max(1, msb(bm)))
    op = blas.axpby(alpha, x, beta, y)
    got = exact_values(op)
    want = [alpha.value * a + beta.value * b for a, b in zip(x.values(), y.values())]
    assert got == want
    assert op.e == min(ae + ex, be + ey)
    assert all(msb(v) <= op.w for v in op.rows().flat)  # width bound


@settings(max_examples=120, deadline=None)
@given(st.lists(mant, min_size=1, max_size=6), st.lists(mant, min_size=6, max_size=6),
       st.integers(1, 32), st.integers(1, 32), st.integers(-60, 60), st.integers(-60, 60))
def test_sub_exact(xs, ys, wx, wy, ex, ey):
    n = len(xs)
    x = rand_block(xs, ex, wx)
    y = rand_block(ys[:n], ey, wy)
    op = blas.sub(x, y)
    assert exact_values(op) == [a - b for a, b in zip(x.values(), y.values())]
    assert op.e == min(ex, ey)
    assert all(msb(v) <= op.w for v in op.rows().flat)


def _interior(nin, d):
    return [p for p in np.ndindex(*(nin,) * d) if all(0 < c < nin - 1 for c in p)]


def _all_nodes(nin, d):
    return list(np.ndindex(*(nin,) * d))


def dense_operator(kind, j, ndim):
    """Exact dense matrices written from the definitions (not from the
    stencil code): the 5/7-point Laplacian divided by the level scaling,
    nodal interpolation weights prod_k (1 - |o_k|/2), and the restriction
    s_c^-1 2^-d P^T s_f. Returns (rows, cols, dict (row, col) -> value)."""
    s = {jj: (Fraction(4) if ndim == 2 else Fraction(8)) * (1 << (2 * jj)) for jj in (j, j - 1)}
    nf = (1 << j) + 1
    nc = (1 << (j - 1)) + 1
    M = {}
    if kind == "A":
        rows = cols = _interior(nf, ndim)
        h2inv = Fraction(1 << (2 * j))
        for p in rows:
            M[(p, p)] = 2 * ndim * h2inv / s[j]
            for k in range(ndim):
                for sgn in (-1, 1):
                    q = list(p)
                    q[k] += sgn
                    q = tuple(q)
                    if all(0 < c < nf - 1 for c in q):
                        M[(p, q)] = -h2inv / s[j]
        return rows, cols, M
    P = {}
    for p in _interior(nf, ndim):
        for I in _interior(nc, ndim):
            o = [p[k] - 2 * I[k] for k in range(ndim)]
            if all(abs(c) <= 1 for c in o):
                wgt = Fraction(1)
                for c in o:
                    wgt *= Fraction(1, 2) if c else 1
                P[(p, I)] = wgt
    if kind == "P":
        return _interior(nf, ndim), _interior(nc, ndim), P
    scale = s[j] / s[j - 1] / (1 << ndim)
    R = {(I, p): v * scale for (p, I), v in P.items()}
    return _interior(nc, ndim), _interior(nf, ndim), R


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("kind", ["A", "R", "P"])
def test_spmv_exact_against_dense(ndim, kind):
    j = 3 if ndim == 2 else 2
    S = {"A": lambda: fd.scaled_A(j, ndim), "R": lambda: fd.scaled_R(j, ndim),
         "P": lambda: fd.prolongation(ndim)}[kind]()
    rows, cols, M = dense_operator(kind, j, ndim)
    nin = (1 << (j - 1)) + 1 if kind == "P" else (1 << j) + 1
    g = np.random.default_rng(5)
    xm = np.zeros((nin,) * ndim, dtype=object)
    for c in cols:
        xm[c] = int(g.integers(-(2 ** 31), 2 ** 31 - 1))
    x = BFP(-7, xm, 32)
    op = blas.spmv(S, x)
    got = op.rows()
    for r in rows:
        want = sum((v * Fraction(int(xm[c])) for (rr, c), v in M.items() if rr == r), Fraction(0))
        assert Fraction(int(got[r])) * TWO ** S.e == want, r
    # the output ring stays zero
    ring = [p for p in _all_nodes(got.shape[0], ndim) if p not in set(rows)]
    assert all(got[p] == 0 for p in ring)
    assert op.e == S.e + x.e
    assert all(msb(v) <= op.w for v in got.flat)


@settings(max_examples=60, deadline=None)
@given(st.lists(mant, min_size=5, max_size=5), st.integers(-40, 40), st.integers(-40, 40),
       st.integers(-(2 ** 15), 2 ** 15 - 1), st.integers(-(2 ** 15), 2 ** 15 - 1),
       st.integers(-20, 5), st.integers(-20, 5))
def test_gemv_exact(ys, ex, ey, am, bm, ae, be):
    j, ndim = 2, 2
    A = fd.scaled_A(j, ndim)
    g = np.random.default_rng(abs(ex) + 3 * abs(ey))
    xm = np.zeros((5, 5), dtype=object)
    xm[1:-1, 1:-1] = g.integers(-(2 ** 31), 2 ** 31 - 1, size=(3, 3)).astype(object)
    ym = np.zeros((5, 5), dtype=object)
    ym[1:-1, 1:-1] = np.array(ys[:4] + ys[:5], dtype=object).reshape(3, 3)
    x, y = BFP(ex, xm, 32), BFP(ey, ym, 32)
    alpha = Scalar(am, ae, max(1, msb(am)))
    beta = Scalar(bm, be, max(1, msb(bm)))
    op = blas.gemv(A, x, y, alpha, beta)
    Ax = blas.spmv(A, x)
    want = [alpha.value * a + beta.value * b for a, b in zip(exact_values(Ax), y.values().flat)]
    assert exact_values(op) == want
    assert all(msb(v) <= op.w for v in op.rows().flat)


def test_dot_exact():
    g = np.random.default_rng(9)
    for _ in range(20):
        n = int(g.integers(1, 50))
        x = vec(g.integers(-(2 ** 31), 2 ** 31 - 1, n), int(g.integers(-50, 50)), 32)
        y = vec(g.integers(-(2 ** 15), 2 ** 15 - 1, n), int(g.integers(-50, 50)), 16)
        d = blas.dot(x, y)
        assert d.value == sum(a * b for a, b in zip(x.values(), y.values()))
        assert msb(d.m) <= d.w


# -------------------------------------------------------------- qcomp ---

def test_figure2_windows_through_qcomp():
    """A one-element exact result 23 (Figure 2) with the three example
    windows: sufficient (no recompute), overflow and underflow (recompute);
    the output is the same 4-bit block 0101 in every case."""
    g = json.load(open(os.path.join(GOLDEN, "fig2_windows.json")))
    z = vec([g["value"]], 0, 10)
    op = blas.identity(z)
    w_out = g["w_out"]

    def run(mu_tmp, w_tmp):
        gamma = TWO ** (mu_tmp - 2)  # nu(gamma) = mu_tmp with e_z* = 0
        return blas.qcomp(op, w_out, w_tmp, gamma)

    s = g["sufficient"]
    out, info = run(s["mu_tmp"], s["w_tmp"])
    assert s["mu_tmp"] - s["w_tmp"] == s["lambda_tmp"]
    assert not info.recomputed and info.mu_star == g["mu_star"]
    assert list(out.m) == [int(g["out_bits"], 2)] and out.e == g["lambda_out"]

    out, info = run(g["overflow"]["mu_tmp"], w_out)
    assert info.overflow and info.recomputed
    assert list(out.m) == [int(g["out_bits"], 2)] and out.e == g["lambda_out"]

    lam_tmp = g["underflow"]["lambda_tmp"]
    out, info = run(lam_tmp + 6, 6)   # window [4, 10): overestimated gamma
    assert info.underflow and info.recomputed
    assert list(out.m) == [int(g["out_bits"], 2)] and out.e == g["lambda_out"]


@settings(max_examples=120, deadline=None)
@given(st.lists(st.integers(-(2 ** 40), 2 ** 40), min_size=1, max_size=8),
       st.integers(-30, 30), st.integers(1, 33), st.integers(0, 8),
       st.integers(-12, 12), st.integers(1, 2 ** 20))
def test_qcomp_matches_definition_for_any_window(ms, e, w_out, w_add, gshift, gm):
    """P3: the output of Algorithm 1 depends on neither gamma nor w_tmp; it
    is the exact result normalized and floor-truncated to w_out bits."""
    z = vec(ms, e, 41)
    op = blas.identity(z)
    gamma = Fraction(gm) * TWO ** (e + gshift)
    out, info = blas.qcomp(op, w_out, w_out + w_add, gamma)
    ref_e, ref_m = q_reference(exact_values(op), w_out, op.e)
    assert out.e == ref_e and list(out.m) == ref_m
    plain, _ = blas.qcomp_plain(op, w_out)
    assert plain.e == out.e and list(plain.m) == list(out.m)
    assert out.fits()


@settings(max_examples=120, deadline=None)
@given(st.lists(st.integers(-(2 ** 40), 2 ** 40), min_size=1, max_size=8),
       st.integers(-30, 30), st.integers(1, 33), st.integers(-12, 12), st.integers(1, 2 ** 20))
def test_nnqcomp_matches_definition(ms, e, w_out, gshift, gm):
    z = vec(ms, e, 41)
    op = blas.identity(z)
    gamma = Fraction(gm) * TWO ** (e + gshift)
    out, info = blas.nnqcomp(op, w_out, gamma)
    ref_e, ref_m = nn_reference(exact_values(op), w_out, gamma)
    assert out.e == ref_e and list(out.m) == ref_m
    plain = blas.nnqcomp_plain(op, w_out, gamma)
    assert plain.e == out.e and list(plain.m) == list(out.m)
    lo, hi = xw_range(w_out)
    unclamped = [math.floor(v / TWO ** ref_e) for v in exact_values(op)]
    assert info.saturated == sum(1 for v in unclamped if v < lo or v > hi)


@settings(max_examples=150, deadline=None)
@given(st.lists(st.integers(-(2 ** 40), 2 ** 40), min_size=1, max_size=8),
       st.integers(-30, 30), st.integers(2, 33), st.integers(0, 6))
def test_nnqcomp_equals_qcomp_at_exact_gamma(ms, e, w_out, over):
    """P4: with gamma = ||z||_inf nnqcomp returns qcomp's block, except that a
    maximal-magnitude entry equal to minus a power of two costs one bit; an
    overestimate by 2^k costs exactly k more bits (a further floor shift)."""
    if all(v == 0 for v in ms):
        return
    z = vec(ms, e, 41)
    op = blas.identity(z)
    norm = z.norm_inf()
    q, _ = blas.qcomp_plain(op, w_out)
    nn, info = blas.nnqcomp(op, w_out, norm * TWO ** over)
    assert info.saturated == 0
    mx = max(abs(v) for v in ms)
    neg_pow2 = (-mx in ms) and (mx & (mx - 1)) == 0 and (mx not in ms)
    loss = over + (1 if neg_pow2 else 0)
    assert nn.e == q.e + loss
    assert list(nn.m) == [v >> loss for v in q.m]


def test_nnqcomp_saturates_on_underestimate():
    z = vec([1000, -1000, 3], 0, 12)
    out, info = blas.nnqcomp(blas.identity(z), 4, Fraction(10))
    assert list(out.m) == [7, -8, 1] and info.saturated == 2


def test_zero_results():
    z = vec([0, 0, 0], 5, 8)
    q, _ = blas.qcomp_plain(blas.identity(z), 8)
    assert q.e == 5 + 1 - 8 and all(v == 0 for v in q.m)
    nn, _ = blas.nnqcomp(blas.identity(z), 8, Fraction(0))
    assert nn.e == 5 + 1 - 8 and all(v == 0 for v in nn.m)


@settings(max_examples=80, deadline=None)
@given(st.lists(st.integers(-(2 ** 31), 2 ** 31 - 1), min_size=1, max_size=8),
       st.integers(-30, 30), st.integers(1, 32), st.integers(-20, 20), st.integers(1, 2 ** 16))
def test_exponent_shift_equivariance(ms, e, w_out, k, gm):
    """P10: scaling every input by 2^k shifts every output exponent by k and
    leaves all mantissas unchanged (floor is not odd, so no sign symmetry)."""
    a = vec(ms, e, 32)
    b = vec(ms, e + k, 32)
    qa, _ = blas.qcomp_plain(blas.identity(a), w_out)
    qb, _ = blas.qcomp_plain(blas.identity(b), w_out)
    assert qb.e == qa.e + k and list(qa.m) == list(qb.m)
    g = Fraction(gm) * TWO ** e
    na, _ = blas.nnqcomp(blas.identity(a), w_out, g)
    nb, _ = blas.nnqcomp(blas.identity(b), w_out, g * TWO ** k)
    assert nb.e == na.e + k and list(na.m) == list(nb.m)


def test_floor_is_not_odd():
    a = vec([5, -5], 0, 8)
    q, _ = blas.qcomp_plain(blas.identity(a), 2)
    assert list(q.m) == [1, -2]


def test_normalize_and_saturate_truncate():
    z = vec([12, -7, 3], -4, 8)
    n = blas.normalize(z, 3)
    assert (n.e, list(n.m)) == (-4 + 2, [3, -2, 0])
    s, info = blas.saturate_truncate(z, 3, Fraction(1, 4))
    assert s.e == -3 and list(s.m) == [3, -4, 1] and info.saturated == 1
