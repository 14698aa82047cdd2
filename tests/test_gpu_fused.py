"""The V-cycle's relaxation and residual in one launch (2D, nnqcomp): every
block of an FMG solve and of a lone V-cycle equals, bit for bit (mantissas
and metadata), the same solve with the two ops launched separately, over
grid sizes with one and several column segments and march lengths that
leave ragged last bands; and the fused path is the one that runs (fewer
launches). The fusion is a tuning option (off by default); with it off
the separate launches are the ones the oracle comparisons of the solver
check."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_2307_00124_amd as P
import workloads as W

pytestmark = pytest.mark.gpu


def _snapshot(H, L):
    out = {}
    for j in range(1, L + 1):
        for which in (0, 2):
            v = H.get_vec(j, which)
            out[(j, which)] = (v.mantissas().clone(), v.host_meta()[:6])
    return out


def _run(L, w, fuse, rows, min_bits):
    P.bfp_tuning_set("fuse_relax_res", fuse)
    P.bfp_tuning_set("relax_res_rows", rows)
    P.bfp_tuning_set("relax_res_max_n", 1 << 20)   # every launched level
    try:
        p = P.mg_params_init(2, L, w, True, 1, 0, 2, P.MG_POLICY_NN_IR_FIRST_Q, 23)
        if min_bits:
            p.min_storage_bits = min_bits
        H = P.Hierarchy(p)
        for j in range(1, L + 1):
            H.set_rhs(j, torch.from_numpy(np.ascontiguousarray(W.manufactured_f(j, 2))).cuda())
        _, l0 = H.counters()
        H.fmg()
        torch.cuda.synchronize()
        _, l1 = H.counters()
        snap = _snapshot(H, L)
        y = H.vcycle(L, H.get_vec(L, 2))
        torch.cuda.synchronize()
        snap["vcycle_y"] = (y.mantissas().clone(), y.host_meta()[:6])
        return snap, l1 - l0
    finally:
        P.bfp_tuning_set("fuse_relax_res", 0)
        P.bfp_tuning_set("relax_res_rows", 0)
        P.bfp_tuning_set("relax_res_max_n", 255)


@pytest.mark.parametrize("L,w,rows,min_bits", [
    (7, 32, 0, 32), (7, 32, 1, 32), (8, 32, 3, 32), (9, 32, 0, 32), (9, 28, 5, 32),
    (10, 32, 2, 32), (11, 32, 0, 32), (8, 16, 0, 0)])
def test_fused_relax_residual_matches_two_launches(L, w, rows, min_bits):
    print(f"fused relax+residual: L={L} w={w} rows={rows} min_bits={min_bits}", flush=True)
    ref, launches_ref = _run(L, w, 0, rows, min_bits)
    got, launches_got = _run(L, w, 1, rows, min_bits)
    for key in ref:
        assert torch.equal(ref[key][0], got[key][0]), f"mantissas {key}"
        assert ref[key][1] == got[key][1], f"metadata {key}: {ref[key][1]} vs {got[key][1]}"
    if min_bits == 32:
        # one launch saved per V-cycle visit of a launched level (levels
        # 7..L; N = 2 IR-V iterations per FMG level)
        visits = sum(2 * (L - l + 1) for l in range(7, L + 1))
        assert launches_ref - launches_got == visits, (launches_ref, launches_got, visits)
    else:
        assert launches_ref == launches_got   # 16-bit storage: not fused
