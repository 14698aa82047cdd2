"""Multigrid parity: IR, V-cycles and FMG of the HIP library against the
oracle, bit for bit, plus the discretization-accuracy gate."""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest
import torch

import paper_2307_00124_amd as P
import workloads as W
from oracle import fp64, mg
from oracle.bfp import from_f64
from tests.gpu_util import assert_block_equal

pytestmark = pytest.mark.gpu

POLICY = {"q": P.MG_POLICY_Q, "nn": P.MG_POLICY_NN, "nn_ir_first_q": P.MG_POLICY_NN_IR_FIRST_Q,
          "nn_ir_first2_q": P.MG_POLICY_NN_IR_FIRST2_Q, "nn_ir_q": P.MG_POLICY_NN_IR_Q}


@pytest.fixture(autouse=True)
def _track_residual(monkeypatch):
    """Record the oracle's last IR residual on its hierarchy (the solver
    functions return only the iterate)."""
    orig = mg.ir_iteration

    def wrapped(H, l, x, g, force_q=False, first=False):
        xn, r = orig(H, l, x, g, force_q=force_q, first=first)
        H.last_r = r
        return xn, r
    monkeypatch.setattr(mg, "ir_iteration", wrapped)
    yield


def setup_pair(ndim, L, w, progressive, policy, nu1, nu2, N, eta, levels=None):
    """Library and oracle hierarchies for the manufactured problem; `levels`
    keeps only the coarsest levels of an L-level schedule."""
    p = P.mg_params_init(ndim, L, w, progressive, nu1, nu2, N, POLICY[policy], eta)
    Lr = levels or L
    p.L = Lr
    f = {j: W.manufactured_f(j, ndim) for j in range(1, Lr + 1)}
    H = P.Hierarchy(p)
    for j in range(1, Lr + 1):
        H.set_rhs(j, torch.from_numpy(np.ascontiguousarray(f[j])).cuda())
    s = mg.widths_progressive(L, w) if progressive else mg.widths_fixed(L, w)
    widths = mg.Widths(*({j: d[j] for j in range(1, Lr + 1)} for d in (s.check, s.work, s.inner)))
    O = mg.build_hierarchy(f, ndim, Lr, widths, mg.make_smoother(ndim, Fraction(eta, 100)),
                           policy=policy, nu1=nu1, nu2=nu2)
    return H, O


def test_rhs_blocks_match():
    H, O = setup_pair(2, 6, 24, True, "nn", 1, 0, 2, 23)
    for j in range(1, 7):
        assert_block_equal(H.get_vec(j, 1), O.b[j], f"b level {j}")


@pytest.mark.parametrize("policy", ["q", "nn"])
def test_c1_fmg_v22(policy):
    """33 x 33, 5 levels, widths 32, FMG with N = 2 IR-V(2,2)."""
    H, O = setup_pair(2, 5, 32, False, policy, 2, 2, 2, 13)
    H.fmg()
    x = mg.fmg(O, 2)
    assert_block_equal(H.get_vec(5, 0), x, "C1 FMG x")
    assert_block_equal(H.get_vec(5, 2), O.last_r, "C1 FMG last residual")


def test_c1_ir_from_random_guess():
    """10 IR-V(2,2) iterations from the seeded uniform[-1, 1] guess, qcomp."""
    H, O = setup_pair(2, 5, 32, False, "q", 2, 2, 2, 13)
    x0 = W.initial_guess(5, 2, seed=0)
    H.set_x(5, torch.from_numpy(x0).cuda())
    H.ir(5, 10)
    xo, hist = mg.ir_solve(O, from_f64(x0, 32), 10)
    assert_block_equal(H.get_vec(5, 0), xo, "C1 IR x")
    assert_block_equal(H.get_vec(5, 2), hist[-1], "C1 IR last residual")
    us = W.manufactured_u(5, 2)
    uh = fp64.discrete_solution_manufactured(us, 5)
    u = P.bfp_vec_to_f64(H.get_vec(5, 0)).cpu().numpy()
    assert fp64.l2_error(u, us, 5) <= 1.1 * fp64.l2_error(uh, us, 5)


@pytest.mark.parametrize("L,w,policy", [(6, 24, "nn_ir_first_q"), (7, 16, "nn_ir_first_q"),
                                        (6, 24, "nn"), (7, 12, "nn_ir_q"),
                                        (8, 24, "nn_ir_first_q")])
def test_progressive_fmg_2d(L, w, policy):
    H, O = setup_pair(2, L, w, True, policy, 1, 0, 2, 23)
    H.fmg()
    x = mg.fmg(O, 2)
    assert_block_equal(H.get_vec(L, 0), x, "FMG x")
    assert_block_equal(H.get_vec(L, 2), O.last_r, "last IR residual")


@pytest.mark.parametrize("L", [3, 4])
def test_progressive_fmg_3d(L):
    H, O = setup_pair(3, L, 24, True, "nn_ir_first_q", 1, 0, 2, 23)
    H.fmg()
    x = mg.fmg(O, 2)
    assert_block_equal(H.get_vec(L, 0), x, "3D FMG x")


def test_3d_v22_plain_ir():
    H, O = setup_pair(3, 4, 24, True, "nn_ir_first2_q", 2, 2, 2, 13)
    H.ir(4, 3)
    x0 = mg.zero_block(4, 3, O.widths.work[4])
    xo, _ = mg.ir_solve(O, x0, 3)
    assert_block_equal(H.get_vec(4, 0), xo, "3D IR x")


def test_vcycle_entry_point():
    H, O = setup_pair(2, 6, 24, True, "nn", 1, 0, 2, 23)
    H.fmg()
    mg.fmg(O, 2)
    y = H.vcycle(6, H.get_vec(6, 2))
    yo = mg.vcycle(O, 6, O.last_r)
    assert_block_equal(y, yo, "V-cycle output")


@pytest.mark.parametrize("w", [24, 32])
def test_full_size_fmg_coarse_levels_and_accuracy(w):
    """The 4097 x 4097 FMG (12 levels): levels 1..8 of the run are checked bit
    for bit against the oracle with the same 12-level schedule. With the
    finest inner width 32 the finest iterate must be within 1.1x of the
    discretization error (24 bits are too few on 12 levels)."""
    L, Lc = 12, 8
    p = P.mg_params_init(2, L, w, True, 1, 0, 2, P.MG_POLICY_NN_IR_FIRST_Q, 23)
    p.min_storage_bits = 32
    H = P.Hierarchy(p)
    for j in range(1, L + 1):
        H.set_rhs(j, torch.from_numpy(W.manufactured_f(j, 2)).cuda())
    H.fmg()
    torch.cuda.synchronize()
    _, O = setup_pair(2, L, w, True, "nn_ir_first_q", 1, 0, 2, 23, levels=Lc)
    x8 = mg.fmg(O, 2)
    assert_block_equal(H.get_vec(Lc, 0), x8, "level-8 iterate of the 12-level FMG")
    u = P.bfp_vec_to_f64(H.get_vec(L, 0))
    us = torch.from_numpy(W.manufactured_u(L, 2)).cuda()
    err = torch.sqrt(((u - us)[1:-1, 1:-1] ** 2).sum() * 2.0 ** (-2 * L)).item()
    disc = (fp64.kappa_h(L) - 1) * math.sqrt(float((us[1:-1, 1:-1] ** 2).sum()) * 2.0 ** (-2 * L))
    if w == 32:
        assert err <= 1.1 * disc, (err, disc)


def _lib_hierarchy(ndim, L, w, progressive, policy, nu1, nu2, N, eta, exec_points):
    P.bfp_tuning_set("exec_max_points", exec_points)
    try:
        p = P.mg_params_init(ndim, L, w, progressive, nu1, nu2, N, POLICY[policy], eta)
        H = P.Hierarchy(p)
    finally:
        P.bfp_tuning_set("exec_max_points", 4096)
    for j in range(1, L + 1):
        H.set_rhs(j, torch.from_numpy(np.ascontiguousarray(W.manufactured_f(j, ndim))).cuda())
    return H


def _same_block(a, b, what):
    assert torch.equal(a.mantissas(), b.mantissas()), what
    assert a.host_meta()[:6] == b.host_meta()[:6], what


@pytest.mark.parametrize("ndim,L,w,prog,policy,nu", [
    (2, 8, 24, True, "nn_ir_first_q", (1, 0)), (2, 7, 32, False, "q", (2, 2)),
    (2, 7, 12, True, "nn", (2, 1)), (3, 5, 20, True, "nn_ir_first_q", (1, 0)),
    (3, 5, 32, False, "q", (2, 2))])
def test_coarse_programs_match_launches(ndim, L, w, prog, policy, nu):
    """FMG and IR with the coarse levels run by the one-workgroup executor
    give the same blocks, bit for bit (mantissas and metadata), as with one
    launch per operation."""
    runs = []
    for pts in (0, 4096):
        H = _lib_hierarchy(ndim, L, w, prog, policy, nu[0], nu[1], 2, 23, pts)
        H.fmg()
        fmg_blocks = [(H.get_vec(j, 0).mantissas().clone(), H.get_vec(j, 0).host_meta()[:6],
                       H.get_vec(j, 2).mantissas().clone(), H.get_vec(j, 2).host_meta()[:6])
                      for j in range(1, L + 1)]
        H.ir(L, 2)
        runs.append((H, fmg_blocks))
        torch.cuda.synchronize()
    (H0, f0), (H1, f1) = runs
    for j in range(1, L + 1):
        for k in range(4):
            a, b = f0[j - 1][k], f1[j - 1][k]
            assert (torch.equal(a, b) if torch.is_tensor(a) else a == b), f"FMG level {j} item {k}"
    _same_block(H0.get_vec(L, 0), H1.get_vec(L, 0), "x after IR")
    _same_block(H0.get_vec(L, 2), H1.get_vec(L, 2), "r after IR")
    b0, l0 = H0.counters()
    b1, l1 = H1.counters()
    assert abs(b0 - b1) <= 1e-9 * b0 and l1 < l0


@pytest.mark.parametrize("ndim,L,w,prog,policy,nu", [
    (2, 5, 32, False, "q", (2, 2)), (2, 6, 24, True, "nn_ir_first2_q", (1, 1)),
    (2, 6, 16, True, "nn_ir_first_q", (1, 0)), (3, 4, 20, True, "nn_ir_q", (2, 1))])
def test_ir_programs_match_launches(ndim, L, w, prog, policy, nu):
    """IR-V on a finest level small enough for the executor (each iteration
    one recorded program: the first, the second and the later ones differ
    in their compression modes) gives the same x and r, bit for bit, as
    with one launch per operation; checked after 1 and after 4 iterations."""
    x0 = torch.from_numpy(np.ascontiguousarray(W.initial_guess(L, ndim, seed=3))).cuda()
    out = []
    for pts in (0, 4096):
        H = _lib_hierarchy(ndim, L, w, prog, policy, nu[0], nu[1], 2, 23, pts)
        H.set_x(L, x0)
        H.ir(L, 1)
        one = (H.get_vec(L, 0).mantissas().clone(), H.get_vec(L, 0).host_meta()[:6])
        H.set_x(L, x0)
        H.ir(L, 4)
        torch.cuda.synchronize()
        out.append((H, one))
    (H0, o0), (H1, o1) = out
    assert torch.equal(o0[0], o1[0]) and o0[1] == o1[1], "x after one IR iteration"
    _same_block(H0.get_vec(L, 0), H1.get_vec(L, 0), "x after 4 IR iterations")
    _same_block(H0.get_vec(L, 2), H1.get_vec(L, 2), "r after 4 IR iterations")
    b0, l0 = H0.counters()
    b1, l1 = H1.counters()
    assert abs(b0 - b1) <= 1e-9 * b0 and l1 == 5 < l0


@pytest.mark.parametrize("ndim,L,w,prog,policy,nu,pts", [
    (2, 8, 24, True, "nn_ir_first_q", (1, 0), 4096), (2, 5, 32, False, "q", (2, 2), 4096),
    (3, 5, 20, True, "nn_ir_first_q", (1, 0), 4096), (2, 7, 16, True, "nn", (1, 0), 0)])
def test_fmg_f64_matches_separate_calls(ndim, L, w, prog, policy, nu, pts):
    """mg_fmg_f64 (coarse right-hand sides quantized inside the coarse-level
    program, finer ones on the side stream) gives the blocks of mg_set_rhs on
    every level followed by mg_fmg, bit for bit; twice in a row, the second
    time with other right-hand sides (so the pointers and the fork/join order
    are exercised)."""
    f1 = [torch.from_numpy(np.ascontiguousarray(W.manufactured_f(j, ndim))).cuda()
          for j in range(1, L + 1)]
    f2 = [(-3.0 * f).contiguous() for f in f1]
    one = _lib_hierarchy(ndim, L, w, prog, policy, nu[0], nu[1], 2, 23, pts)
    sep = _lib_hierarchy(ndim, L, w, prog, policy, nu[0], nu[1], 2, 23, pts)
    for rhs in (f1, f2):
        one.fmg_f64(rhs)
        for j in range(1, L + 1):
            sep.set_rhs(j, rhs[j - 1])
        sep.fmg()
        torch.cuda.synchronize()
        for j in range(1, L + 1):
            for which, name in ((0, "x"), (1, "b"), (2, "r")):
                _same_block(one.get_vec(j, which), sep.get_vec(j, which), f"{name} level {j}")
    b1, _ = one.counters()
    b2, _ = sep.counters()
    assert abs(b1 - b2) <= 1e-9 * b2
