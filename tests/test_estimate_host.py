"""The library's host-side energy norm (bfp_energy_norm: sine-transform
similarity and Lanczos) against the oracle's dense generalized eigenproblem
(scipy), on random matrices and on a BFP error propagation matrix; and the
width rules of bfp-prec-est (mg_params_apply_estimate). No GPU needed."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import estimate as oest
from oracle import mg
from paper_2307_00124_amd import estimate as est


@pytest.mark.parametrize("ndim,j", [(2, 2), (2, 3), (2, 4), (3, 2), (3, 3)])
def test_energy_norm_random(ndim, j):
    N = ((1 << j) - 1) ** ndim
    g = np.random.default_rng(100 * ndim + j)
    for scale in (1.0, 1e-3):
        E = scale * g.standard_normal((N, N))
        ref = oest.energy_rate(E, oest.dense_A(j, ndim))
        assert est.energy_norm(E, ndim, j) == pytest.approx(ref, rel=1e-10)


def test_energy_norm_low_rank_and_zero():
    j, ndim = 3, 2
    N = 49
    g = np.random.default_rng(7)
    u, v = g.standard_normal(N), g.standard_normal(N)
    E = np.outer(u, v)
    assert est.energy_norm(E, ndim, j) == pytest.approx(
        oest.energy_rate(E, oest.dense_A(j, ndim)), rel=1e-10)
    assert est.energy_norm(np.zeros((N, N)), ndim, j) == 0.0


@pytest.mark.parametrize("ndim,j", [(2, 3), (3, 2)])
def test_energy_norm_of_a_bfp_iteration(ndim, j):
    E = oest.error_propagation(ndim, j, oest.width_rules(j, 2, 5))
    ref = oest.energy_rate(E, oest.dense_A(j, ndim))
    assert est.energy_norm(E, ndim, j) == pytest.approx(ref, rel=1e-10)


def test_width_rules():
    p = est.base_params(2, 6)
    for qc, qi in ((1, 1), (2, 11), (40, 40)):
        q = est.apply_estimate(p, qc, qi)
        o = oest.width_rules(6, qc, qi)
        c, w, i = est.widths(q)
        assert (c, w, i) == (o.check, o.work, o.inner)
