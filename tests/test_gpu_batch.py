"""Batched solves: one launch runs the right-hand-side conversion and the
whole FMG of every problem; each problem's blocks must equal, bit for bit,
the same problem solved alone through mg_set_rhs + mg_fmg, and (for small
problems) the oracle."""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest
import torch

import paper_2307_00124_amd as P
import workloads as W
from oracle import mg
from tests.gpu_util import assert_block_equal

pytestmark = pytest.mark.gpu


def rhs_arrays(solves, ndim=2):
    """FP64 f_j of every problem on every level, and the pointer table."""
    keep = []
    table = torch.zeros(len(solves) * P.MG_MAX_LEVELS, dtype=torch.int64)
    for i, s in enumerate(solves):
        for j in range(1, s.level + 1):
            f = torch.from_numpy(np.ascontiguousarray(W.sine_f(j, s.modes))).cuda()
            keep.append(f)
            table[i * P.MG_MAX_LEVELS + j - 1] = f.data_ptr()
    return keep, table.cuda()


def same(a: P.Vec, b: P.Vec) -> bool:
    return torch.equal(a.mantissas(), b.mantissas()) and a.host_meta()[:6] == b.host_meta()[:6]


@pytest.mark.parametrize("w_inner", [16, 32])
def test_batch_matches_solo_and_oracle(w_inner):
    g = np.random.default_rng(5)
    solves = [W.BatchSolve(int(s), W.draw_sine_modes(g, 2))
              for s in g.choice([3, 5, 9, 17, 33, 65], 14)]
    prms = [P.batch_params(2, s.level, w_inner) for s in solves]
    B = P.Batch(prms)
    keep, table = rhs_arrays(solves)
    for rep in range(2):                       # a second solve reuses the arena
        B.solve(table)
        torch.cuda.synchronize()
    for i, s in enumerate(solves):
        H = P.Hierarchy(prms[i])
        for j in range(1, s.level + 1):
            H.set_rhs(j, keep[sum(t.level for t in solves[:i]) + j - 1])
        H.fmg()
        torch.cuda.synchronize()
        for j in range(1, s.level + 1):
            for which in (0, 1, 2):
                assert same(B.get_vec(i, j, which), H.get_vec(j, which)), (i, j, which)
    # oracle for the two smallest distinct sizes
    for i in sorted(range(len(solves)), key=lambda k: solves[k].level)[:2]:
        s = solves[i]
        L = s.level
        f = {j: W.sine_f(j, s.modes) for j in range(1, L + 1)}
        p = prms[i]
        widths = mg.Widths({j: p.w_check[j] for j in range(1, L + 1)},
                           {j: p.w_work[j] for j in range(1, L + 1)},
                           {j: p.w_inner[j] for j in range(1, L + 1)})
        O = mg.build_hierarchy(f, 2, L, widths, mg.make_smoother(2, Fraction(23, 100)),
                               policy="nn_ir_first_q", nu1=1, nu2=0)
        x = mg.fmg(O, 2)
        assert_block_equal(B.get_vec(i, L, 0), x, f"problem {i} (side {s.side})")


def test_batch_counters_and_errors():
    prms = [P.batch_params(2, 3), P.batch_params(2, 4)]
    B = P.Batch(prms)
    b, n = B.counters()
    assert b > 0 and n == 0
    bad = P.batch_params(2, 3)
    bad.ndim = 3
    with pytest.raises(P.BFPError):
        P.Batch([prms[0], bad])


@pytest.mark.parametrize("w_inner", [8, 16])
def test_batch_large_sides_match_solo(w_inner):
    """Sides 129 and 257 (levels 7 and 8), which the batch runs entirely in
    its one-workgroup-per-problem executor while a hierarchy of its own runs
    them as launched kernels: every block of every level must agree."""
    g = np.random.default_rng(77 + w_inner)
    solves = [W.BatchSolve(int(s), W.draw_sine_modes(g, 2)) for s in (257, 129, 65, 257, 129)]
    prms = [P.batch_params(2, s.level, w_inner) for s in solves]
    B = P.Batch(prms)
    keep, table = rhs_arrays(solves)
    B.solve(table)
    torch.cuda.synchronize()
    at = 0
    for i, s in enumerate(solves):
        H = P.Hierarchy(prms[i])
        for j in range(1, s.level + 1):
            H.set_rhs(j, keep[at + j - 1])
        at += s.level
        H.fmg()
        torch.cuda.synchronize()
        for j in range(1, s.level + 1):
            for which in (0, 1, 2):
                assert same(B.get_vec(i, j, which), H.get_vec(j, which)), (i, s.side, j, which)
