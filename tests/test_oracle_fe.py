"""The oracle's finite-element multigrid (oracle/fe.py): set-up S and the
per-site quantization against their plain definitions, and the BFP FMG with
wide mantissas converging to the exact discrete solution."""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

from oracle import fe, mg
from workloads import fe as W


def wide(L, w=80):
    d = {j: w for j in range(1, L + 1)}
    return mg.Widths(dict(d), dict(d), dict(d))


def test_setup_s_definitions():
    A, R, P, dg = fe.scaled_operators("poisson", 3, 4)
    K = np.array(W.stiffness(4, 3, 1).dense(), dtype=object)
    Ad = np.array(A[4].dense(), dtype=object)
    for i in range(K.shape[0]):
        assert Ad[i, i] == 1
        for k in range(K.shape[0]):
            assert Ad[i, k] == K[i, k] / K[i, i]
    # R = 2 Dc^-1 P^T Df (m = 1)
    Pd = np.array(P[4].dense(), dtype=object)
    Rd = np.array(R[4].dense(), dtype=object)
    Kc = np.array(W.stiffness(3, 3, 1).dense(), dtype=object)
    for l in range(Rd.shape[0]):
        for k in range(Rd.shape[1]):
            assert Rd[l, k] == 2 * Pd[k, l] * K[k, k] / Kc[l, l]


def test_band_quantization_and_apply():
    A, _, _, _ = fe.scaled_operators("biharmonic", 4, 3)
    B = fe.quantize_band(A[3], 13, "A")
    vals = [Fraction(v) for row in A[3].vals for v in row if v]
    e = max(fe.nu_rational(v) for v in vals) - 13
    assert B.e == e
    assert all(B.taps[i][t] == (Fraction(v) / Fraction(2) ** e).__floor__()
               for i, row in enumerate(A[3].vals) for t, v in enumerate(row))
    g = np.random.default_rng(0)
    x = np.zeros(A[3].ncols + 2, dtype=object)
    x[1:-1] = [int(v) for v in g.integers(-1000, 1000, A[3].ncols)]
    D = np.array(A[3].dense(), dtype=object)
    out = B.apply(x)
    Bd = np.array([[0] * A[3].ncols for _ in range(A[3].nrows)], dtype=object)
    for i in range(A[3].nrows):
        for t, v in enumerate(B.taps[i]):
            Bd[i, A[3].col0[i] + t] = v
    assert list(out[1:-1]) == list(Bd.dot(x[1:-1]))
    assert out[0] == 0 and out[-1] == 0


@pytest.mark.parametrize("kind,p,L,N", [("poisson", 2, 5, 6), ("poisson", 3, 5, 6),
                                        ("biharmonic", 3, 5, 6), ("biharmonic", 4, 4, 8)])
def test_wide_fmg_reaches_the_discrete_solution(kind, p, L, N):
    H = fe.build(kind, p, L, wide(L))
    x = fe.fmg(H, N)
    c = np.array([float(v) for v in x.to_f64()[1:-1]])
    ch = W.discrete_solution(kind, p, L)
    ratio = W.l2_error(kind, p, L, c) / W.l2_error(kind, p, L, ch)
    assert abs(ratio - 1) < 2e-3, ratio


def test_smoother_matches_the_chebyshev_formula():
    S = fe.smoother("poisson", 4, 6)
    A, _, _, _ = fe.scaled_operators("poisson", 4, 5)
    rho = float(max(sum(abs(v) for v in row) for row in A[5].vals))
    eta = 0.23
    a = (1 + eta) * rho / 2
    c = (1 - eta) * rho / 2
    b = a - c * c / (2 * a)
    assert abs(float(S.c1.value) - 2 / b) < 2 ** -13 * 2 / b
    assert abs(float(S.c2.value) + 1 / (a * b)) < 2 ** -13 / (a * b)
