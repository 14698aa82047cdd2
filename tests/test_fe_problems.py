"""The finite-element model problems' data (workloads/fe.py), pinned by
facts outside it: the linear B-spline stiffness matrix is tridiag(-1, 2, -1)
and its prolongation the nodal (1/2, 1, 1/2); nested spaces make the
Galerkin identity P^T K_fine P = 2^(1-2m) K_coarse exact for every degree;
interior rows of P sum to 1 (partition of unity) and carry the binomial
two-scale coefficients; the discrete solutions converge at the L2 rate
h^(p+1) of B-spline finite elements."""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

from workloads import fe


def dense(B):
    return np.array(B.dense(), dtype=object)


def test_linear_elements_closed_form():
    K = dense(fe.stiffness(3, 1, 1))
    n = K.shape[0]
    assert n == 7
    for i in range(n):
        for k in range(n):
            assert K[i, k] == (2 if i == k else -1 if abs(i - k) == 1 else 0)
    P = dense(fe.prolongation(3, 1, 1))
    for i in range(P.shape[0]):
        for l in range(P.shape[1]):
            want = Fraction(1) if i == 2 * l + 1 else Fraction(1, 2) if abs(i - (2 * l + 1)) == 1 else 0
            assert P[i, l] == want


@pytest.mark.parametrize("kind,p", [("poisson", p) for p in range(1, 7)] +
                         [("biharmonic", p) for p in range(3, 7)])
def test_galerkin_identity(kind, p):
    m = 1 if kind == "poisson" else 2
    for j in (2, 3, 4):
        Kf, Kc, P = dense(fe.stiffness(j, p, m)), dense(fe.stiffness(j - 1, p, m)), \
            dense(fe.prolongation(j, p, m))
        G = P.T.dot(Kf).dot(P)
        assert all(G[a, b] == Kc[a, b] * Fraction(2) ** (1 - 2 * m)
                   for a in range(Kc.shape[0]) for b in range(Kc.shape[0]))


@pytest.mark.parametrize("p", range(1, 7))
def test_two_scale_coefficients(p):
    """An interior coarse B-spline is sum_k binom(p+1, k) / 2^p of the fine
    ones; interior fine rows sum to 1."""
    P = dense(fe.prolongation(5, p, 1))
    l = P.shape[1] // 2
    col = [v for v in P[:, l] if v != 0]
    assert col == [Fraction(math.comb(p + 1, k), 2 ** p) for k in range(p + 2)]
    for i in range(2 * p + 2, P.shape[0] - 2 * p - 2):
        assert sum(P[i, :]) == 1


def test_stiffness_is_symmetric_and_positive_definite():
    for kind, p in (("poisson", 3), ("biharmonic", 4)):
        m = 1 if kind == "poisson" else 2
        K = dense(fe.stiffness(4, p, m))
        assert all(K[i, k] == K[k, i] for i in range(K.shape[0]) for k in range(K.shape[0]))
        assert np.linalg.eigvalsh(K.astype(float)).min() > 0


@pytest.mark.parametrize("kind,p", [("poisson", 1), ("poisson", 2), ("poisson", 3),
                                    ("biharmonic", 3), ("biharmonic", 4)])
def test_discretization_error_rate(kind, p):
    e1 = fe.l2_error(kind, p, 4, fe.discrete_solution(kind, p, 4))
    e2 = fe.l2_error(kind, p, 5, fe.discrete_solution(kind, p, 5))
    rate = math.log2(e1 / e2)
    assert abs(rate - (p + 1)) < 0.35, rate
