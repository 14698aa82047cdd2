"""The finite-element FMG as one recorded single-workgroup program: after
each of two solves in a row, every level's iterate, residual and
right-hand side equal, bit for bit (mantissas and exponents), the same
solve run op by op with the two qcomp passes as separate launches; the
program is the path that runs (one launch per solve); and hierarchies
from one level up to the 4095 unknowns of Poisson p = 1, L = 12 record
one, while larger ones run op by op."""
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


def _solves(kind, p, L, program):
    P.bfp_tuning_set("fe_program", program)
    P.bfp_tuning_set("fe_one_launch", 4096 if program else 0)
    try:
        m = 1 if kind == "poisson" else 2
        ck, wk, inn = _widths(kind, p, L)
        K = [W.stiffness(j, p, m) for j in range(1, L + 1)]
        Pm = [None] + [W.prolongation(j, p, m) for j in range(2, L + 1)]
        F = [W.load_vector(kind, j, p) for j in range(1, L + 1)]
        G = P.FEHierarchy(m, L, W.PAPER_N[(kind, p)], K, Pm, F, ck, wk, inn)
        outs, launches = [], []
        for _ in range(2):
            _, l0 = G.counters()
            G.fmg()
            _, l1 = G.counters()
            launches.append(l1 - l0)
            outs.append({(j, w): G.get(j, w) for j in range(1, L + 1) for w in (0, 1, 2)})
        return outs, launches
    finally:
        P.bfp_tuning_set("fe_program", 1)
        P.bfp_tuning_set("fe_one_launch", 4096)


@pytest.mark.parametrize("kind,p,L", [("poisson", 1, 12), ("poisson", 1, 1), ("poisson", 2, 5),
                                      ("poisson", 6, 4), ("biharmonic", 3, 6), ("biharmonic", 6, 3)])
def test_fe_program_matches_op_by_op(kind, p, L):
    print(f"fe program: {kind} p={p} L={L}", flush=True)
    ref, lref = _solves(kind, p, L, 0)
    got, lgot = _solves(kind, p, L, 1)
    assert lgot == [1, 1], lgot
    assert all(n > 1 for n in lref), lref
    for t in range(2):
        for key in ref[t]:
            (rm, re), (gm, ge) = ref[t][key], got[t][key]
            assert np.array_equal(rm, gm), f"solve {t}: mantissas {key}"
            assert re == ge, f"solve {t}: exponent {key}: {re} vs {ge}"


def test_fe_program_not_recorded_beyond_one_workgroup():
    """Poisson p = 1 on 13 levels (8191 unknowns on the finest level, more
    than one workgroup holds): no program is recorded, the solve runs op by
    op whatever fe_program says, and equals the op-by-op solve with the two
    qcomp passes as separate launches."""
    print("fe program: poisson p=1 L=13 (no program)", flush=True)
    ref, lref = _solves("poisson", 1, 13, 0)
    got, lgot = _solves("poisson", 1, 13, 1)
    assert all(n > 1 for n in lgot) and lgot[0] < lref[0], (lref, lgot)
    for key in ref[1]:
        (rm, re), (gm, ge) = ref[1][key], got[1][key]
        assert np.array_equal(rm, gm), f"mantissas {key}"
        assert re == ge, f"exponent {key}: {re} vs {ge}"
