"""The FP64 multigrid comparator on the GPU (fp64_mg_*) against the oracle's
FP64 multigrid with the same schedule and coefficients: equal up to FP64
rounding (the summation orders differ), and at the discretization error."""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest
import torch

import paper_2307_00124_amd as P
import workloads as W
from oracle import fp64, mg

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ndim,L,nu,N", [(2, 5, (1, 0), 2), (2, 8, (1, 0), 2), (2, 6, (2, 2), 2),
                                         (3, 4, (1, 0), 2), (3, 6, (2, 2), 1)])
def test_fp64_fmg_matches_oracle(ndim, L, nu, N):
    p = P.mg_params_init(ndim, L, 32, True, nu[0], nu[1], N, P.MG_POLICY_NN_IR_FIRST_Q, 23)
    F = P.FP64MG(p)
    f = [torch.from_numpy(W.manufactured_f(j, ndim)).cuda() for j in range(1, L + 1)]
    out = torch.zeros(((1 << L) + 1,) * ndim, dtype=torch.float64, device="cuda")
    F.fmg(f, out)
    torch.cuda.synchronize()
    u = out.cpu().numpy()
    sm = mg.make_smoother(ndim, Fraction(23, 100))
    ref = fp64.FP64MG({j: W.manufactured_f(j, ndim) for j in range(1, L + 1)}, ndim, L,
                      float(sm.c1.value), float(sm.c2.value), nu[0], nu[1]).fmg(N)
    assert np.allclose(u, ref, rtol=1e-12, atol=1e-15)
    us = W.manufactured_u(L, ndim)
    uh = fp64.discrete_solution_manufactured(us, L)
    assert fp64.l2_error(u, us, L) <= 1.1 * fp64.l2_error(uh, us, L)
    assert np.all(u[0] == 0) and np.all(u[-1] == 0)
