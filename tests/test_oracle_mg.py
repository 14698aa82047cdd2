"""Pins of the FD operators, the Chebyshev relaxation and the BFP multigrid
solver of the oracle."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import blas, fd, fp64, mg
from oracle.bfp import BFP, from_f64

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TWO = Fraction(2)


# --------------------------------------------------------- FD operators --

def test_scaled_operators_are_the_expected_dyadic_stencils():
    A2 = fd.scaled_A(7, 2).values()
    assert A2[(0, 0)] == 1 and all(A2[o] == Fraction(-1, 4) for o in A2 if o != (0, 0))
    assert fd.scaled_A(7, 2).w == 4 and fd.scaled_A(7, 2).e == -2
    A3 = fd.scaled_A(5, 3).values()
    assert A3[(0, 0, 0)] == Fraction(3, 4)
    assert all(A3[o] == Fraction(-1, 8) for o in A3 if o != (0, 0, 0)) and len(A3) == 7
    R2 = fd.scaled_R(6, 2)
    P2 = fd.prolongation(2)
    assert R2.values() == P2.values()            # R' = P^T in 2D
    R3 = fd.scaled_R(6, 3)
    P3 = fd.prolongation(3)
    assert all(R3.values()[o] == P3.values()[o] / 2 for o in P3.values())  # R' = P^T/2
    assert R2.norm_inf() == 4 and R3.norm_inf() == 4
    assert (R3.w, P3.w, fd.scaled_A(4, 3).w) == (5, 5, 4)


@pytest.mark.parametrize("ndim", [2, 3])
def test_sine_modes_are_eigenvectors(ndim):
    """Closed-form pin of A': for v = prod sin(k pi x), A' v = lambda v with
    lambda = (4/h^2) sum sin^2(k pi h / 2) / s_j."""
    j = 4
    A = fd.scaled_A(j, ndim)
    x = W.coords(j)
    ks = [1, 3, 2][:ndim]
    parts = []
    for k in ks:
        s = np.sin(math.pi * k * x)
        s[0] = s[-1] = 0.0
        parts.append(s)
    v = parts[0]
    for p in parts[1:]:
        v = np.multiply.outer(p, v)
    h = 2.0 ** -j
    lam = (4 / h ** 2) * sum(math.sin(k * math.pi * h / 2) ** 2 for k in ks) / float(fd.level_scale(j, ndim))
    Av = fp64.apply_f64(A, v)
    inner = (slice(1, -1),) * ndim
    assert np.allclose(Av[inner], lam * v[inner], rtol=0, atol=1e-14)


@pytest.mark.parametrize("ndim", [2, 3])
def test_nodal_interpolation_preserves_max_norm(ndim):
    """P7: ||P d||_inf = ||d||_inf for nodal interpolation."""
    g = np.random.default_rng(3)
    j = 3
    n = (1 << (j - 1)) + 1
    for _ in range(5):
        d = np.zeros((n,) * ndim, dtype=object)
        d[(slice(1, -1),) * ndim] = g.integers(-1000, 1000, (n - 2,) * ndim).astype(object)
        x = BFP(-3, d, 12)
        Pd = blas.spmv(fd.prolongation(ndim), x)
        vals = [abs(Fraction(int(v))) * TWO ** Pd.e for v in Pd.rows().flat]
        assert max(vals) == x.norm_inf()


def test_rhs_scaling_is_a_power_of_two():
    assert fd.rhs_log2_scale(5, 2) == -12 and fd.rhs_log2_scale(5, 3) == -13
    f = W.manufactured_f(4, 2)
    b = mg.rhs_block(f, 4, 2, 32)
    b0 = from_f64(f, 32)
    assert b.e == b0.e - 10 and (b.m == b0.m).all()


# ------------------------------------------------------------- Chebyshev --

@pytest.mark.parametrize("eta", [Fraction(13, 100), Fraction(23, 100), Fraction(1, 2)])
def test_chebyshev_two_step_polynomial_equioscillates(eta):
    """The relaxation y = (c1 I + c2 A) r has error polynomial
    p(l) = 1 - c1 l - c2 l^2; two Chebyshev steps make |p| equioscillate on
    [eta rho, rho] (equal magnitude at both ends and at the vertex, with
    alternating sign) and the coefficients have c1 > 0 > c2 (P6)."""
    rho = Fraction(2)
    c1, c2 = mg.cheby_nodes(rho, eta)
    assert c1 > 0 > c2
    p = lambda l: 1 - c1 * l - c2 * l * l
    a, b = eta * rho, rho
    vertex = -c1 / (2 * c2)
    assert a < vertex < b
    assert p(a) == p(b) and p(a) > 0
    # the Chebyshev level: |p| at the vertex, sign opposite to the ends
    assert p(vertex) < 0 and -p(vertex) == p(a)


def test_chebyshev_bounds_in_inf_norm():
    """P6: for the D-scaled 5-point operator (diag 1, E = I - A >= 0):
    ||(c1 I + c2 A) r|| <= c1 ||r|| and ||A y - r|| <= (2 c1 + 1) ||r||."""
    sm = mg.make_smoother(2, Fraction(23, 100))
    c1, c2 = float(sm.c1.value), float(sm.c2.value)
    A = fd.scaled_A(5, 2)
    g = np.random.default_rng(0)
    for _ in range(20):
        r = np.zeros((33, 33))
        r[1:-1, 1:-1] = g.uniform(-1, 1, (31, 31))
        y = c2 * fp64.apply_f64(A, r) + c1 * r
        nr = np.abs(r).max()
        assert np.abs(y).max() <= c1 * nr + 1e-12
        assert np.abs(fp64.apply_f64(A, y) - r).max() <= (2 * c1 + 1) * nr + 1e-12


def test_smoother_quantization():
    sm = mg.make_smoother(3, Fraction(23, 100))
    c1, c2 = mg.cheby_nodes(2, Fraction(23, 100))
    assert sm.c1.value <= c1 * Fraction(4, 3) < sm.c1.value + TWO ** sm.c1.e
    assert sm.c2.value <= c2 * Fraction(16, 9) < sm.c2.value + TWO ** sm.c2.e
    assert sm.c1_gamma.value <= c1 < sm.c1_gamma.value + TWO ** sm.c1_gamma.e
    for s in (sm.c1, sm.c2, sm.c1_gamma):
        assert s.w == 16 and -(2 ** 15) <= s.m < 2 ** 15 and abs(s.m) >= 2 ** 14 - 1


@pytest.mark.slow
def test_eta_is_a_local_minimum_of_the_vcycle_rate():
    """The empirical eta for 2D V(1,0) on level 5: 0.23 beats its neighbours."""
    from oracle import cheby
    rates = {}
    for i in (22, 23, 24):
        c1, c2 = mg.cheby_nodes(2, Fraction(i, 100))
        rates[i] = cheby.vcycle_rate(2, 5, float(c1), float(c2))
    assert rates[23] < rates[22] and rates[23] < rates[24]
    assert 0.3 < rates[23] < 0.35


# --------------------------------------------------------------- solver --

def _hier(L, ndim, widths, policy="nn", nu1=1, nu2=0, eta=Fraction(23, 100), **kw):
    f = {j: W.manufactured_f(j, ndim) for j in range(1, L + 1)}
    return mg.build_hierarchy(f, ndim, L, widths, mg.make_smoother(ndim, eta),
                              policy=policy, nu1=nu1, nu2=nu2, **kw)


def _ratio(x, L, ndim):
    us = W.manufactured_u(L, ndim)
    uh = fp64.discrete_solution_manufactured(us, L)
    return fp64.l2_error(x.to_f64(), us, L) / fp64.l2_error(uh, us, L)


def test_op_count_structure_matches_table2():
    """P8: the quantizing calls an FMG with N IR-V(1,0) iterations makes on
    its finest level (counted from the solve's call trace, on the recursion
    level of each call) are the parenthesized totals of Table 2 for the same
    N."""
    g = json.load(open(os.path.join(GOLDEN, "table2_call_totals.json")))
    pairs = {(e["N"], e["total"]) for e in g["poisson"] + g["biharmonic"]}
    for N, total in sorted(pairs):
        for L in (3, 4):
            H = _hier(L, 2, mg.widths_fixed(L, 24))
            H.trace = []
            mg.fmg(H, N)
            assert sum(1 for t in H.trace if t["level"] == L) == total, (N, L)
            assert len(H.trace) == H.stats.calls


def test_fp64_mg_converges_to_closed_form():
    """P9: iterated to convergence, multigrid reproduces u_h = kappa_h u*;
    its error ratio between levels tends to 4 (O(h^2))."""
    errs = []
    for L in (4, 5, 6):
        f = {j: W.manufactured_f(j, 2) for j in range(1, L + 1)}
        sm = mg.make_smoother(2, Fraction(23, 100))
        m = fp64.FP64MG(f, 2, L, float(sm.c1.value), float(sm.c2.value))
        u = m.solve()
        us = W.manufactured_u(L, 2)
        uh = fp64.discrete_solution_manufactured(us, L)
        assert np.abs(u - uh).max() < 1e-13
        errs.append(fp64.l2_error(uh, us, L))
    assert abs(errs[0] / errs[1] - 4) < 0.02 and abs(errs[1] / errs[2] - 4) < 0.01


def test_large_width_bfp_fmg_matches_fp64_fmg():
    """P11: with 60-bit mantissas everywhere, BFP FMG and FP64 FMG with the
    same schedule and coefficients agree to FP64 rounding."""
    L = 5
    H = _hier(L, 2, mg.widths_fixed(L, 60), policy="q")
    x = mg.fmg(H, 2)
    f = {j: W.manufactured_f(j, 2) for j in range(1, L + 1)}
    m = fp64.FP64MG(f, 2, L, float(H.smoother.c1.value), float(H.smoother.c2.value))
    u = m.fmg(2)
    assert np.abs(x.to_f64() - u).max() <= 1e-13 * np.abs(u).max()


def test_windowed_qcomp_equals_plain_in_the_solver():
    """P3 inside the solver: Table 1 windows (with recomputations) and the
    plain definition give bit-identical FMG iterates."""
    L = 5
    Ha = _hier(L, 2, mg.widths_fixed(L, 20), policy="q", nu1=2, nu2=2, window=True)
    Hb = _hier(L, 2, mg.widths_fixed(L, 20), policy="q", nu1=2, nu2=2, window=False)
    xa, xb = mg.fmg(Ha, 2), mg.fmg(Hb, 2)
    assert xa.e == xb.e and (xa.m == xb.m).all()
    assert Ha.stats.q_calls == Ha.stats.calls


def test_c1_fmg_reaches_discretization_accuracy():
    """33 x 33 grid, all widths 32, qcomp, FMG with N = 2 IR-V(2,2)."""
    L = 5
    H = _hier(L, 2, mg.widths_fixed(L, 32), policy="q", nu1=2, nu2=2, eta=Fraction(13, 100))
    assert _ratio(mg.fmg(H, 2), L, 2) <= 1.1


def test_c1_ir_from_random_guess_converges():
    L = 5
    H = _hier(L, 2, mg.widths_fixed(L, 32), policy="q", nu1=2, nu2=2, eta=Fraction(13, 100))
    x0 = from_f64(W.initial_guess(L, 2, seed=0), 32)
    x, hist = mg.ir_solve(H, x0, 10)
    assert _ratio(x, L, 2) <= 1.1
    norms = [r.norm_inf() for r in hist]
    assert norms[-1] < norms[0] * Fraction(1, 10 ** 6)


@pytest.mark.parametrize("L", [5, 6, 7])
def test_progressive_fmg_with_first_residual_qcomp(L):
    H = _hier(L, 2, mg.widths_progressive(L, 24), policy="nn_ir_first_q")
    assert _ratio(mg.fmg(H, 2), L, 2) <= 1.1
    assert H.stats.saturations == 0


def test_all_nnqcomp_fmg_saturates_the_first_ir_residual():
    """On these FD problems the Table 1 estimate for the first IR residual of
    an FMG level is too small: nnqcomp saturates there, and only there."""
    H = _hier(6, 2, mg.widths_progressive(6, 24), policy="nn")
    mg.fmg(H, 2)
    assert H.stats.saturations > 0


def test_width_schedule_ordering():
    for L in (5, 9, 12):
        for w in (8, 16, 24, 32):
            s = mg.widths_progressive(L, w)
            for j in range(1, L + 1):
                assert s.check[j] >= s.work[j] >= s.inner[j] >= 5
            assert s.inner[L] == min(w, s.work[L])


def test_3d_fmg_reaches_discretization_accuracy():
    L = 4
    H = _hier(L, 3, mg.widths_progressive(L, 24), policy="nn_ir_first_q")
    assert _ratio(mg.fmg(H, 2), L, 3) <= 1.1
