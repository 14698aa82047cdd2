"""Pins of the oracle's solve diagnostics: per (level, call site) counts of
qcomp window gaps and nnqcomp saturations (Section 4's Algorithm 1, the
recomputation table of Section 6.3, Section 6.4)."""
import json
import os
from fractions import Fraction

import pytest

import workloads as W
from oracle import mg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fmg(ndim, L, policy, N, nu=(1, 0), w=32, progressive=True):
    f = {j: W.manufactured_f(j, ndim) for j in range(1, L + 1)}
    widths = mg.widths_progressive(L, w) if progressive else mg.widths_fixed(L, w)
    H = mg.build_hierarchy(f, ndim, L, widths, mg.make_smoother(ndim, Fraction(23, 100)),
                           policy=policy, nu1=nu[0], nu2=nu[1])
    mg.fmg(H, N)
    return H


def test_gap_bins():
    assert [mg.gap_bin(d) for d in (-5, -1, 0, 1, 58, 59, 400)] == [0, 0, 1, 2, 59, 60, 60]
    row = [0] * mg.DIAG_BINS
    row[0], row[1], row[3], row[7] = 2, 5, 1, 4      # d < 0 twice; d = 0, 2, 6
    assert mg.recomputations(row, 0) == 2 + 1 + 4
    assert mg.recomputations(row, 2) == 2 + 4
    assert mg.recomputations(row, 6) == 2


def test_finest_level_call_counts_match_the_recomputation_table():
    """Every call on the finest level of an FMG with qcomp everywhere is a
    windowed qcomp call: their number is the parenthesized total the paper
    prints for the same N (6N + 1 with V(1,0))."""
    g = json.load(open(os.path.join(GOLDEN, "table2_call_totals.json")))
    for N in sorted({e["N"] for e in g["poisson"]} & {1, 2, 3}):
        H = _fmg(2, 4, "q", N)
        a = H.stats.diag_array()
        total = int(a[4, :, :mg.DIAG_GAP_BINS].sum())
        assert total in [e["total"] for e in g["poisson"] if e["N"] == N], (N, total)
        assert int(a[4, :, mg.DIAG_NN_CALLS].sum()) == 0
        # per site: N of each IR/V step (the first IR residual once), one prolongation
        per = a[4, :, :mg.DIAG_GAP_BINS].sum(axis=1)
        expect = {"ir_res_first": 1, "ir_res": N - 1, "ir_corr": N, "relax": N, "v_res": N,
                  "restrict": N, "v_corr": N, "fmg_prol": 1}
        assert {s: int(per[k]) for k, s in enumerate(mg.SITES)} == expect


@pytest.mark.parametrize("ndim,L,nu", [(2, 5, (1, 0)), (2, 4, (2, 2)), (3, 3, (1, 0))])
def test_histogram_gives_algorithm1_recomputations(ndim, L, nu, monkeypatch):
    """Recomputations read off the gap histogram equal those Algorithm 1
    itself (the oracle's step-by-step qcomp) performs, for the windows of
    the estimates table and for each cap w_add <= w_add_max of the
    recomputation table's sweep (the window changes no result, so the
    histogram of one run serves every cap)."""
    H = _fmg(ndim, L, "q", 2, nu)
    a = H.stats.diag_array()
    for cap in (None, 4, 2, 0):
        w_add = {s: (v if cap is None else min(v, cap)) for s, v in mg.W_ADD.items()}
        predicted = sum(mg.recomputations(a[l, k], w_add[mg.SITES[k]])
                        for l in range(1, L + 1) for k in range(len(mg.SITES)))
        monkeypatch.setattr(mg, "W_ADD", w_add)
        H2 = _fmg(ndim, L, "q", 2, nu)
        assert predicted == H2.stats.recomputations, (cap, predicted, H2.stats.recomputations)
        assert (H2.stats.diag_array() == a).all()


def test_saturation_counts_add_up():
    """nnqcomp rows: one count per call, the saturated entries the calls
    report, and the calls that saturated. With nnqcomp everywhere the
    estimate for the first IR residual of an FMG level is too small on these
    FD problems, so those calls (and only those) saturate."""
    H = _fmg(2, 6, "nn", 2, w=24)
    a = H.stats.diag_array()
    sat_sites = {mg.SITES[k] for k in range(len(mg.SITES)) if a[:, k, mg.DIAG_NN_SAT].sum()}
    assert sat_sites == {"ir_res_first"}
    assert int(a[:, :, mg.DIAG_NN_CALLS].sum()) == H.stats.calls - H.stats.q_calls
    assert int(a[:, :, mg.DIAG_NN_SAT].sum()) == H.stats.saturations > 0
    assert 0 < int(a[:, :, mg.DIAG_NN_SAT_CALLS].sum()) <= int(a[:, :, mg.DIAG_NN_CALLS].sum())
    assert int(a[:, :, :mg.DIAG_GAP_BINS].sum()) == 0


# ------------------------------------------ safety fallback (Section 6.4) --

def _ir_hier(L, w, policy, nu=(1, 0)):
    f = {j: W.manufactured_f(j, 2) for j in range(1, L + 1)}
    return mg.build_hierarchy(f, 2, L, mg.widths_progressive(L, w),
                              mg.make_smoother(2, Fraction(23, 100)), policy=policy,
                              nu1=nu[0], nu2=nu[1])


def test_safe_ir_recovers_where_plain_nnqcomp_stalls():
    """IR-V(1,0) from zero with nnqcomp everywhere: the second residual
    outgrows its estimate and saturates, and the plain iteration stalls at a
    saturated power of two (the Remark on skipping normalization in IR-V);
    the fallback reruns the IR residual with qcomp and convergence resumes."""
    L = 6
    H = _ir_hier(L, 24, "nn")
    _, hist = mg.ir_solve(H, mg.zero_block(L, 2, H.widths.work[L]), 8)
    stalled = [r.norm_inf() for r in hist]
    assert stalled[2] == stalled[3] == stalled[4] and H.stats.saturations > 0
    Hs = _ir_hier(L, 24, "nn")
    _, hs, switched = mg.ir_solve_safe(Hs, mg.zero_block(L, 2, Hs.widths.work[L]), 8)
    assert switched > 0
    assert hs[-1].norm_inf() < stalled[3] / 100      # far below the plateau


def test_safe_ir_without_a_trigger_is_plain_ir():
    L = 5
    H = _ir_hier(L, 24, "q")
    x, hist = mg.ir_solve(H, mg.zero_block(L, 2, H.widths.work[L]), 6)
    Hs = _ir_hier(L, 24, "q")
    xs, hs, switched = mg.ir_solve_safe(Hs, mg.zero_block(L, 2, Hs.widths.work[L]), 6,
                                        theta=Fraction(16))
    assert switched == 0 and (xs.m == x.m).all() and xs.e == x.e


def test_safe_ir_always_triggered_is_the_qcomp_residual_policy():
    """With a threshold no residual can meet, every iteration from the third
    on runs the fallback (the first two IR residuals are qcomp by the
    policy; the norm test needs a previous residual): exactly the policy
    that takes qcomp for every IR residual."""
    L = 5
    H = _ir_hier(L, 24, "nn_ir_q")
    x, _ = mg.ir_solve(H, mg.zero_block(L, 2, H.widths.work[L]), 6)
    Hs = _ir_hier(L, 24, "nn_ir_first2_q")
    xs, _, switched = mg.ir_solve_safe(Hs, mg.zero_block(L, 2, Hs.widths.work[L]), 6,
                                       q_iters=1, theta=Fraction(1, 1 << 40))
    assert switched == 4 and (xs.m == x.m).all() and xs.e == x.e
