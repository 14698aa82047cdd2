"""The finite-element model problems on the GPU (fe_*): set-up S, the
per-site operators and the whole BFP FMG equal the oracle (oracle/fe.py) bit
for bit — the right-hand side of every level, the Chebyshev coefficients,
and the iterate and last residual of every level — for Poisson with
B-splines of degree 1..6 and the biharmonic equation with degree 3..6."""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import paper_2307_00124_amd as P
from oracle import fe, mg
from workloads import fe as W

pytestmark = pytest.mark.gpu


def widths(kind, p, L):
    """A progressive schedule within the library's 61-bit exact budgets
    (Section 5's growth rates (k+m) j, k j and m j, k = p + 1)."""
    m = 1 if kind == "poisson" else 2
    k = p + 1
    check = {j: min(28, (k + m) * j + 4) for j in range(1, L + 1)}
    work = {j: min(28, k * j + 6) for j in range(1, L + 1)}
    inner = {j: min(20, m * j + 10, work[j]) for j in range(1, L + 1)}
    return check, work, inner


def run_both(kind, p, L, N):
    m = 1 if kind == "poisson" else 2
    ck, wk, inn = widths(kind, p, L)
    K = [W.stiffness(j, p, m) for j in range(1, L + 1)]
    Pm = [None] + [W.prolongation(j, p, m) for j in range(2, L + 1)]
    F = [W.load_vector(kind, j, p) for j in range(1, L + 1)]
    G = P.FEHierarchy(m, L, N, K, Pm, F, ck, wk, inn)
    H = fe.build(kind, p, L, mg.Widths(ck, wk, inn))
    return G, H


def same(gpu, ref, what):
    mant, e = gpu
    refm = np.array([int(v) for v in ref.m], dtype=np.int64)
    bad = np.argwhere(mant.astype(np.int64) != refm)
    assert bad.size == 0, f"{what}: {len(bad)} mantissas differ, first at {bad[0]}"
    assert e == ref.e, f"{what}: exponent gpu {e} oracle {ref.e}"


CASES = [("poisson", p, 6 if p == 1 else 5) for p in range(1, 7)] + \
        [("biharmonic", p, 5) for p in range(3, 7)]


@pytest.mark.parametrize("kind,p,L", CASES)
def test_fe_fmg_matches_oracle(kind, p, L):
    N = W.PAPER_N[(kind, p)]
    G, H = run_both(kind, p, L, N)
    (c1m, c1e), (c2m, c2e) = G.coefficients()
    assert (c1m, c1e) == (H.smoother.c1.m, H.smoother.c1.e)
    assert (c2m, c2e) == (H.smoother.c2.m, H.smoother.c2.e)
    for j in range(1, L + 1):
        same(G.get(j, 1), H.b[j], f"b level {j}")
    G.fmg()
    # the oracle's FMG, keeping every level's iterate and last residual
    xs, rs = {}, {}
    x = H.zero(1, H.widths.work[1])
    for l in range(1, L + 1):
        if l > 1:
            x = mg.fmg_prolongation(H, l, x)
        for i in range(N):
            x, r = mg.ir_iteration(H, l, x, None)
        xs[l], rs[l] = x, r
    for l in range(1, L + 1):
        same(G.get(l, 0), xs[l], f"{kind} p {p}: x level {l}")
        same(G.get(l, 2), rs[l], f"{kind} p {p}: last residual level {l}")


def test_fe_accuracy_where_widths_allow():
    """Poisson with linear elements (dyadic operators) on 8 levels reaches
    the discretization error of the exact discrete solution."""
    L = 8
    G, _ = run_both("poisson", 1, L, 2)
    G.fmg()
    mant, e = G.get(L, 0)
    c = mant[1:-1].astype(np.float64) * 2.0 ** e
    ratio = W.l2_error("poisson", 1, L, c) / W.l2_error("poisson", 1, L, W.discrete_solution("poisson", 1, L))
    assert ratio <= 1.1, ratio


def test_fe_argument_errors():
    K = [W.stiffness(j, 2, 1) for j in (1, 2)]
    Pm = [None, W.prolongation(2, 2, 1)]
    F = [W.load_vector("poisson", j, 2) for j in (1, 2)]
    big = {1: 32, 2: 32}
    with pytest.raises(P.BFPError):      # widths beyond the exact budget
        G = P.FEHierarchy(1, 2, 1, K, Pm, F, big, big, big)
        G.fmg()
    with pytest.raises(P.BFPError):      # m must be 1 or 2
        P.FEHierarchy(3, 2, 1, K, Pm, F, {1: 8, 2: 8}, {1: 8, 2: 8}, {1: 8, 2: 8})
