"""Finite-element ops with at most a set number of outputs (up to 4096,
1..16 per lane of one workgroup) take both qcomp passes in one launch:
every level's iterate, residual and right-hand side after an FMG solve
equal, bit for bit (mantissas and exponents), the same solve with the two
passes launched separately, on hierarchies whose finest levels are above
and below the limit; and the one-launch path is the one that runs (one
launch saved per such op)."""
from __future__ import annotations

import numpy as np
import pytest

import paper_2307_00124_amd as P
from workloads import fe as W

pytestmark = pytest.mark.gpu


def _widths(kind, p, L):
    m = 1 if kind == "poisson" else 2
    k = p + 1
    check = {j: min(28, (k + m) * j + 4) for j in range(1, L + 1)}
    work = {j: min(28, k * j + 6) for j in range(1, L + 1)}
    inner = {j: min(20, m * j + 10, work[j]) for j in range(1, L + 1)}
    return check, work, inner


def _solve(kind, p, L, limit):
    P.bfp_tuning_set("fe_one_launch", limit)
    P.bfp_tuning_set("fe_program", 0)   # op by op
    try:
        m = 1 if kind == "poisson" else 2
        ck, wk, inn = _widths(kind, p, L)
        K = [W.stiffness(j, p, m) for j in range(1, L + 1)]
        Pm = [None] + [W.prolongation(j, p, m) for j in range(2, L + 1)]
        F = [W.load_vector(kind, j, p) for j in range(1, L + 1)]
        G = P.FEHierarchy(m, L, W.PAPER_N[(kind, p)], K, Pm, F, ck, wk, inn)
        _, l0 = G.counters()
        G.fmg()
        _, l1 = G.counters()
        out = {(j, which): G.get(j, which) for j in range(1, L + 1) for which in (0, 1, 2)}
        return out, l1 - l0
    finally:
        P.bfp_tuning_set("fe_one_launch", 4096)
        P.bfp_tuning_set("fe_program", 1)


@pytest.mark.parametrize("limit", [256, 1000, 4096])
@pytest.mark.parametrize("kind,p,L", [("poisson", 1, 12), ("poisson", 2, 5), ("biharmonic", 3, 6),
                                      ("poisson", 1, 4), ("poisson", 1, 10)])
def test_fe_one_launch_matches_two(kind, p, L, limit):
    print(f"fe one launch: {kind} p={p} L={L} limit={limit}", flush=True)
    ref, launches_ref = _solve(kind, p, L, 0)
    got, launches_got = _solve(kind, p, L, limit)
    for key in ref:
        (rm, re), (gm, ge) = ref[key], got[key]
        assert np.array_equal(rm, gm), f"mantissas {key}"
        assert re == ge, f"exponent {key}: {re} vs {ge}"
    assert launches_got < launches_ref, (launches_ref, launches_got)
