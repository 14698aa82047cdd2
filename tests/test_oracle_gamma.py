"""Pins of the Table 1 estimates gamma in the oracle's multigrid (Section 6.3).

Only floor(log2 gamma) matters to a quantizing call, so a pin must fix each
estimate to within a factor of two. Each call site is pinned by what the
paper proves about it:

  * the estimate is an upper bound of the exact result's norm (triangle
    inequality for the corrections and the restriction, 0 <= D^-1 A <= 2I
    for the relaxation, ||P d|| = ||d|| for nodal interpolation), and
  * an input on which that bound is attained: a constant interior block for
    the relaxation (A r = 0 away from the boundary) and the restriction (the
    restriction taps sum to ||R||), aligned extremes of opposite sign for the
    corrections, the first residual r = -b of the coarsest FMG level, and
    a sign pattern that makes the V residual reach the row sum of
    c2 A^2 + c1 A - I, below the estimate (1/4)(2 c1 + 1);
  * the IR residual's estimate is the previous residual's norm (the paper's
    assumption that the residual does not grow), checked against the norms
    of the returned residual blocks.

test_every_site_is_pinned plants a mistake in the oracle (one site's gamma
scaled by 2 or by 1/2) and checks that some pin fails."""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import mg
from oracle.bfp import BFP


def _norm(b: BFP) -> Fraction:
    """||b||_inf computed here from the mantissas (not the oracle's helper)."""
    mx = 0
    for v in b.m.flat:
        mx = max(mx, abs(int(v)))
    return Fraction(mx) * Fraction(2) ** b.e


def _hier(ndim: int, L: int, policy: str = "nn", w: int = 32, nu=(1, 0)) -> mg.Hierarchy:
    f = {j: W.manufactured_f(j, ndim) for j in range(1, L + 1)}
    H = mg.build_hierarchy(f, ndim, L, mg.widths_fixed(L, w),
                           mg.make_smoother(ndim, Fraction(23, 100)), policy=policy,
                           nu1=nu[0], nu2=nu[1])
    H.trace = []
    return H


def _block(ndim: int, l: int, entries: dict, w: int = 32, e: int = -30) -> BFP:
    """Level-l block with the given interior entries {index: mantissa}."""
    m = np.zeros(((1 << l) + 1,) * ndim, dtype=object)
    m[...] = 0
    for idx, v in entries.items():
        m[idx] = v
    return BFP(e, m, w)


def _const(ndim: int, l: int, c: int, w: int = 32, e: int = -30) -> BFP:
    m = np.zeros(((1 << l) + 1,) * ndim, dtype=object)
    m[...] = 0
    m[(slice(1, -1),) * ndim] = c
    return BFP(e, m, w)


def _last(H: mg.Hierarchy, site: str) -> dict:
    return [t for t in H.trace if t["site"] == site][-1]


# ------------------------------------------------------------------ pins --

def pin_relaxation_tight():
    for ndim in (2, 3):
        H = _hier(ndim, 3)
        mg.relaxation(H, 3, _const(ndim, 3, 3 << 28))
        t = _last(H, "relax")
        assert t["gamma"] == t["exact_norm"], ("relax", ndim)


def pin_restriction_tight():
    for ndim in (2, 3):
        H = _hier(ndim, 3)
        mg.restriction(H, 3, _const(ndim, 3, -(5 << 27)))
        t = _last(H, "restrict")
        assert t["gamma"] == t["exact_norm"], ("restrict", ndim)


def pin_v_correction_tight():
    for ndim in (2, 3):
        H = _hier(ndim, 3)
        c = (2,) * ndim            # coarse node; fine node 2c
        d = _block(ndim, 2, {c: -(3 << 26)})
        y = _block(ndim, 3, {tuple(2 * k for k in c): 5 << 27, (1,) * ndim: -(1 << 20)})
        mg.v_correction(H, 3, y, d)
        t = _last(H, "v_corr")
        assert t["gamma"] == t["exact_norm"], ("v_corr", ndim)
        z = _block(ndim, 3, {(3,) * ndim: 7 << 26})
        yy = _block(ndim, 3, {(3,) * ndim: -(1 << 29)})
        mg.v_update(H, 3, yy, z)
        t = _last(H, "v_corr")
        assert t["gamma"] == t["exact_norm"], ("v_update", ndim)


def pin_ir_correction_tight():
    for ndim in (2, 3):
        H = _hier(ndim, 3)
        p = (4,) * ndim
        x = _block(ndim, 3, {p: 9 << 26, (1,) * ndim: -(1 << 28)})
        y = _block(ndim, 3, {p: -(3 << 27)}, e=-31)
        mg.ir_correction(H, 3, x, y)
        t = _last(H, "ir_corr")
        assert t["gamma"] == t["exact_norm"], ("ir_corr", ndim)


def _row_of_m(ndim: int, c1: float, c2: float) -> np.ndarray:
    """Row p (the centre of a 5^d patch) of M = c2 B^2 + c1 B - I with
    B = D^-1 A_h (the 5- or 7-point Laplacian scaled to unit diagonal),
    evaluated in FP64 from the finite-difference stencil."""
    n = 5
    def B(u):
        out = u.copy()
        for ax in range(ndim):
            out -= (np.roll(u, 1, ax) + np.roll(u, -1, ax)) / (2 * ndim)
        return out
    row = np.zeros((n,) * ndim)
    for q in np.ndindex(*(n,) * ndim):
        e = np.zeros((n,) * ndim)
        e[q] = 1.0
        Be = B(e)
        row[q] = (c2 * B(Be) + c1 * Be - e)[(2,) * ndim]
    return row


def pin_v_residual_attained_below_estimate():
    """The V residual after the relaxation, on the input that attains the
    row sum of M at one point: its norm lies in [gamma / 2, gamma]."""
    for ndim in (2, 3):
        Hq = _hier(ndim, 3, policy="q")
        s = Hq.smoother
        a_c = 1.0 if ndim == 2 else 0.75
        c1, c2 = float(s.c1.value) * a_c, float(s.c2.value) * a_c * a_c
        row = _row_of_m(ndim, c1, c2)
        ent = {}
        for q in np.ndindex(*row.shape):
            if row[q] != 0:
                ent[tuple(2 + k for k in q)] = (1 << 29) * (1 if row[q] > 0 else -1)
        r = _block(ndim, 3, ent)
        y = mg.relaxation(Hq, 3, r)
        H = _hier(ndim, 3)
        mg.v_residual(H, 3, y, r, mg.v_residual_gamma(H, r))
        t = _last(H, "v_res")
        assert t["exact_norm"] <= t["gamma"] < 2 * t["exact_norm"], ("v_res", ndim, t)


def pin_fmg_prolongation_exact():
    """||P x|| = ||x|| for nodal interpolation: every FMG prolongation's
    estimate equals its exact result's norm."""
    for ndim, L in ((2, 4), (3, 3)):
        H = _hier(ndim, L, policy="nn_ir_first_q")
        mg.fmg(H, 2)
        ts = [t for t in H.trace if t["site"] == "fmg_prol"]
        assert len(ts) == L - 1
        for t in ts:
            assert t["gamma"] == t["exact_norm"], ("fmg_prol", ndim, t["level"])


def pin_first_residual_coarsest_level():
    """On FMG level 1 the iterate is 0, so r = -b and gamma = ||b|| = ||r||."""
    for ndim in (2, 3):
        H = _hier(ndim, 3)
        mg.fmg(H, 1)
        t = [t for t in H.trace if t["site"] == "ir_res_first" and t["level"] == 1][0]
        assert t["gamma"] == t["exact_norm"], ("ir_res_first", ndim)


def pin_ir_residual_is_previous_residual():
    """gamma of IR residual i > 1 = ||r^(i-1)|| of the returned residual
    blocks; gamma of the first residual on FMG level l > 1 = the norm of the
    last residual on level l - 1."""
    for ndim, L in ((2, 4), (3, 3)):
        H = _hier(ndim, L)
        x0 = mg.zero_block(L, ndim, H.widths.work[L])
        _, hist = mg.ir_solve(H, x0, 4)
        gs = [t["gamma"] for t in H.trace if t["site"] == "ir_res"]
        assert gs == [_norm(r) for r in hist[:-1]], ("ir_res", ndim)
        H = _hier(ndim, L)
        mg.fmg(H, 3)
        res = [t for t in H.trace if t["site"] in ("ir_res", "ir_res_first")]
        for l in range(2, L + 1):
            first = [t for t in res if t["level"] == l and t["site"] == "ir_res_first"][0]
            prev = [t for t in res if t["level"] == l - 1][-1]
            assert first["gamma"] == _norm(prev["out"]), ("ir_res_first", ndim, l)
            later = [t for t in res if t["level"] == l]
            for a, b in zip(later, later[1:]):
                assert b["gamma"] == _norm(a["out"]), ("ir_res", ndim, l)


def pin_upper_bounds_in_solves():
    """The bound-based estimates are never below the exact result's norm
    during whole solves (V(1,0) and V(2,2), 2D and 3D)."""
    for ndim, L, nu in ((2, 4, (1, 0)), (2, 3, (2, 2)), (3, 3, (1, 0))):
        H = _hier(ndim, L, policy="nn_ir_first_q", nu=nu)
        mg.fmg(H, 2)
        for t in H.trace:
            if t["site"] in ("ir_corr", "relax", "restrict", "v_corr", "fmg_prol"):
                assert t["gamma"] >= t["exact_norm"], (t["site"], ndim, t["level"])


PINS = [pin_relaxation_tight, pin_restriction_tight, pin_v_correction_tight,
        pin_ir_correction_tight, pin_v_residual_attained_below_estimate,
        pin_fmg_prolongation_exact, pin_first_residual_coarsest_level,
        pin_ir_residual_is_previous_residual, pin_upper_bounds_in_solves]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin()


@pytest.mark.parametrize("site", mg.SITES)
@pytest.mark.parametrize("factor", [Fraction(2), Fraction(1, 2)])
def test_every_site_is_pinned(site, factor, monkeypatch):
    """A gamma off by a factor of two at any one call site fails a pin."""
    orig = mg._quantize_op

    def scaled(H, s, op, w_out, gamma, force_q=False):
        if s == site and gamma is not None:
            gamma = gamma * factor
        return orig(H, s, op, w_out, gamma, force_q)

    monkeypatch.setattr(mg, "_quantize_op", scaled)
    failed = []
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"no pin notices gamma x {factor} at {site}"
