"""The library's a priori precision estimation (Section 6.2) and eta scan
(Section 5) against the oracle's, which share no code with them: the error
propagation matrices agree value for value (the BFP V-cycles are bit-exact),
and so do the searches' results."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import estimate as oest
from paper_2307_00124_amd import estimate as est

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ndim,j,qc,qi", [(2, 3, 30, 30), (2, 3, 1, 4), (2, 4, 2, 6), (3, 2, 1, 3)])
def test_error_propagation_matches_oracle(ndim, j, qc, qi):
    p = est.apply_estimate(est.base_params(ndim, j), qc, qi)
    E = est.error_propagation(p)
    Eo = oest.error_propagation(ndim, j, oest.width_rules(j, qc, qi))
    assert np.array_equal(E, Eo)
    assert est.conv_rate(p) == pytest.approx(oest.energy_rate(Eo, oest.dense_A(j, ndim)), rel=1e-10)


def test_estimation_matches_oracle():
    r = est.bfp_prec_est(est.base_params(2, 3), 16, 1.05)
    ro = oest.bfp_prec_est(2, 3, 16, 1.05)
    assert (r["q_check"], r["q_inner"]) == (ro["q_check"], ro["q_inner"])
    assert r["rho"] == pytest.approx(ro["rho"], rel=1e-10)
    assert r["rho_ref"] == pytest.approx(ro["rho_ref"], rel=1e-10)


def test_eta_scan_matches_oracle():
    p = est.apply_estimate(est.base_params(2, 3), 16, 16)
    i, rho, rates = est.eta_scan(p, lo=15, hi=35)
    io, rho_o = oest.estimate_eta(2, 3, oest.width_rules(3, 16, 16), lo=15, hi=35)
    assert i == io and rho == pytest.approx(rho_o, rel=1e-10)
    assert rates[i - 15] == rho and min(rates) == rho
