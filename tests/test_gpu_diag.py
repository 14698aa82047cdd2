"""Solve diagnostics on the GPU against the oracle's, count for count: per
(level, call site) the qcomp window gaps and the nnqcomp saturations, for
launched operations and for the coarse-level executor's programs."""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest
import torch

import paper_2307_00124_amd as P
import workloads as W
from oracle import mg
from oracle.bfp import from_f64
from tests.gpu_util import assert_block_equal

pytestmark = pytest.mark.gpu

POLICY = {"q": P.MG_POLICY_Q, "nn": P.MG_POLICY_NN, "nn_ir_first_q": P.MG_POLICY_NN_IR_FIRST_Q,
          "nn_ir_first2_q": P.MG_POLICY_NN_IR_FIRST2_Q, "nn_ir_q": P.MG_POLICY_NN_IR_Q}


def _pair(ndim, L, w, progressive, policy, nu1, nu2, eta):
    p = P.mg_params_init(ndim, L, w, progressive, nu1, nu2, 2, POLICY[policy], eta)
    f = {j: W.manufactured_f(j, ndim) for j in range(1, L + 1)}
    P.bfp_tuning_set("diagnostics", 1)
    try:
        H = P.Hierarchy(p)
    finally:
        P.bfp_tuning_set("diagnostics", 0)
    for j in range(1, L + 1):
        H.set_rhs(j, torch.from_numpy(np.ascontiguousarray(f[j])).cuda())
    widths = mg.widths_progressive(L, w) if progressive else mg.widths_fixed(L, w)
    O = mg.build_hierarchy(f, ndim, L, widths, mg.make_smoother(ndim, Fraction(eta, 100)),
                           policy=policy, nu1=nu1, nu2=nu2)
    return H, O, f


def _same(dev, ora, L, what):
    d = dev[1:L + 1]
    o = ora.stats.diag_array()[1:L + 1]
    bad = np.argwhere(d != o)
    assert bad.size == 0, (what, [(int(l) + 1, mg.SITES[k], int(b), int(d[l, k, b]), int(o[l, k, b]))
                                 for l, k, b in bad[:8]])


@pytest.mark.parametrize("ndim,L,w,prog,policy,nu", [
    (2, 5, 32, False, "q", (2, 2)),            # the 33 x 33 FMG, all in the executor
    (2, 7, 24, True, "nn_ir_first_q", (1, 0)),  # finest level launched
    (2, 6, 24, True, "nn", (1, 0)),            # saturating first IR residuals
    (2, 7, 16, True, "q", (1, 0)),
    (3, 4, 24, True, "q", (1, 0)),
    (3, 5, 20, True, "nn_ir_first_q", (2, 1))])
def test_fmg_diagnostics_match_oracle(ndim, L, w, prog, policy, nu):
    H, O, _ = _pair(ndim, L, w, prog, policy, nu[0], nu[1], 23 if nu == (1, 0) else 13)
    H.fmg()
    mg.fmg(O, 2)
    _same(H.diagnostics(), O, L, "FMG")


def test_ir_diagnostics_and_reset():
    """10 IR-V(2,2) iterations of the 33 x 33 problem from the seeded guess
    (the first residual has no estimate and is not counted), then a reset."""
    H, O, _ = _pair(2, 5, 32, False, "q", 2, 2, 13)
    x0 = W.initial_guess(5, 2, seed=0)
    H.set_x(5, torch.from_numpy(x0).cuda())
    H.ir(5, 10)
    mg.ir_solve(O, from_f64(x0, 32), 10)
    d = H.diagnostics(reset=True)
    _same(d, O, 5, "IR")
    assert int(d[5, 0].sum()) == 0 and int(d[5, 1, :mg.DIAG_GAP_BINS].sum()) == 9
    assert not H.diagnostics().any()


def test_off_by_default():
    p = P.mg_params_init(2, 4, 24, True, 1, 0, 2, P.MG_POLICY_NN, 23)
    H = P.Hierarchy(p)
    with pytest.raises(P.BFPError):
        H.diagnostics()


def test_fmg_f64_counts_like_separate_calls():
    H, O, f = _pair(2, 8, 24, True, "nn_ir_first_q", 1, 0, 23)
    H.fmg()
    a = H.diagnostics(reset=True)
    H.fmg_f64([torch.from_numpy(np.ascontiguousarray(f[j])).cuda() for j in range(1, 9)])
    b = H.diagnostics()
    assert (a == b).all() and a[8, :, :mg.DIAG_GAP_BINS].sum() + a[8, :, mg.DIAG_NN_CALLS].sum() == 13


@pytest.mark.parametrize("ndim,L,w,policy,nu,iters,q_iters,theta", [
    (2, 6, 24, "nn", (1, 0), 10, 2, (1, 0)),              # saturation triggers
    (2, 7, 24, "nn", (1, 0), 8, 2, (1, 0)),               # finest level launched
    (2, 5, 24, "nn_ir_first2_q", (1, 0), 6, 1, (1, 40)),  # norm test triggers every time
    (3, 4, 24, "nn", (1, 0), 6, 3, (3, 1))])
def test_safe_ir_matches_oracle(ndim, L, w, policy, nu, iters, q_iters, theta):
    """IR-V from zero with the qcomp fallback (Section 6.4): the same
    iterate, last residual and number of fallback iterations as the oracle."""
    H, O, _ = _pair(ndim, L, w, True, policy, nu[0], nu[1], 23)
    n = (1 << L) + 1
    H.set_x(L, torch.zeros((n,) * ndim, dtype=torch.float64, device="cuda"))
    sw = H.ir_safe(L, iters, q_iters, theta)
    x, hist, sw_o = mg.ir_solve_safe(O, mg.zero_block(L, ndim, O.widths.work[L]), iters, q_iters,
                                     Fraction(theta[0], 1 << theta[1]))
    assert sw == sw_o
    assert_block_equal(H.get_vec(L, 0), x, "x")
    assert_block_equal(H.get_vec(L, 2), hist[-1], "last residual")
