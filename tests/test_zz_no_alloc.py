"""mg_fmg_f64_noalloc (the solve whose hierarchy lives in the library's
static device array) against the existing entry point: the same FMG through
mg_fmg_f64 on a hierarchy in a caller arena, then bfp_vec_to_f64, bit for
bit, on consecutive calls with different (the second smaller) problems and a
repeat of the first."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest
import torch

import paper_2307_00124_amd as P
from paper_2307_00124_amd import abi
import workloads as W

pytestmark = pytest.mark.gpu


def _rhs(ndim, L):
    g = np.random.default_rng(100 * ndim + L)
    modes = W.draw_sine_modes(g, ndim)
    return [torch.from_numpy(np.ascontiguousarray(W.sine_f(j, modes))).cuda()
            for j in range(1, L + 1)]


def _reference(p, rhs):
    H = P.Hierarchy(p)
    H.fmg_f64(rhs)
    out = P.bfp_vec_to_f64(H.get_vec(p.L, 0))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _noalloc(p, rhs):
    L = p.L
    out = torch.full(((1 << L) + 1,) * p.ndim, float("nan"), dtype=torch.float64, device="cuda")
    ptrs = (C.c_void_p * L)(*[f.data_ptr() for f in rhs])
    abi.check(abi.lib.mg_fmg_f64_noalloc(C.byref(p), ptrs, C.c_void_p(out.data_ptr()), None),
            "mg_fmg_f64_noalloc")
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_matches_arena_solve():
    cases = [(2, 9, 24), (2, 6, 16), (3, 5, 24), (2, 9, 24)]   # second one smaller, then a repeat
    for ndim, L, w in cases:
        print(f"no-alloc case ndim {ndim} L {L} w {w}", flush=True)
        p = P.batch_params(ndim, L, w, N=3) if ndim == 3 else \
            P.mg_params_init(ndim, L, w, True, 1, 0, 2, P.MG_POLICY_NN_IR_FIRST_Q, 23)
        rhs = _rhs(ndim, L)
        got = _noalloc(p, rhs)
        ref = _reference(p, rhs)
        assert np.array_equal(got, ref), (ndim, L, w)


def test_noalloc_rejects_problems_beyond_the_array():
    p = P.mg_params_init(2, 11, 32, True, 1, 0, 2, P.MG_POLICY_NN_IR_FIRST_Q, 23)
    assert abi.lib.mg_hierarchy_bytes(C.byref(p)) > abi.MG_NOALLOC_BYTES
    rhs = [torch.zeros(((1 << j) + 1,) * 2, dtype=torch.float64, device="cuda") for j in range(1, 12)]
    ptrs = (C.c_void_p * 11)(*[f.data_ptr() for f in rhs])
    out = torch.zeros((2049, 2049), dtype=torch.float64, device="cuda")
    rc = abi.lib.mg_fmg_f64_noalloc(C.byref(p), ptrs, C.c_void_p(out.data_ptr()), None)
    assert rc == abi.BFP_ENOMEM
    assert b"static" in abi.lib.bfp_last_error()
