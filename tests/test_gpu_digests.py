"""Bit parity at the benchmark sizes: the library's solves against per-level
digests of the oracle's (tests/golden/fmg_digests.json, written by
tests/golden/make_fmg_digests.py, which calls only the oracle). Covers every
level of the 4097^2 FMG the benchmark times (the 2D star kernel's four-row
pipeline, both qcomp passes of the first IR residual per level, the
transfers, the coarse-level executor) and 3D FMG and IR-V(2,2) solves on
129^3 (the multi-plane 3D march)."""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import pytest
import torch

import paper_2307_00124_amd as P
import workloads as W

pytestmark = pytest.mark.gpu

GOLD_PATH = os.path.join(os.path.dirname(__file__), "golden", "fmg_digests.json")
GOLD = json.load(open(GOLD_PATH)) if os.path.exists(GOLD_PATH) else {}
POLICY = {"q": P.MG_POLICY_Q, "nn": P.MG_POLICY_NN, "nn_ir_first_q": P.MG_POLICY_NN_IR_FIRST_Q,
          "nn_ir_first2_q": P.MG_POLICY_NN_IR_FIRST2_Q, "nn_ir_q": P.MG_POLICY_NN_IR_Q}


def digest(v: P.Vec) -> dict:
    torch.cuda.synchronize()
    m = v.mantissas().cpu().numpy().astype("<i8")
    meta = v.host_meta()
    return {"exp": meta[P.BFP_META_EXP], "sha256": hashlib.sha256(m.tobytes()).hexdigest(),
            "max": meta[P.BFP_META_MAX], "min": meta[P.BFP_META_MIN]}


@pytest.mark.parametrize("name", sorted(GOLD))
def test_solve_matches_oracle_digests(name):
    g = GOLD[name]
    c = g["params"]
    ndim, L = c["ndim"], c["L"]
    print(f"digest case {name}", flush=True)
    p = P.mg_params_init(ndim, L, c["w"], True, c["nu"][0], c["nu"][1], c.get("N", 2),
                         POLICY[c["policy"]], c["eta"])
    H = P.Hierarchy(p)
    if c.get("iters"):
        f = torch.from_numpy(W.manufactured_f(L, ndim)).cuda()
        H.set_rhs(L, f)
        H.set_x(L, torch.zeros_like(f))
        H.ir(L, c["iters"])
    else:
        H.fmg_f64([torch.from_numpy(W.manufactured_f(j, ndim)).cuda() for j in range(1, L + 1)])
    for lev, ref in sorted(g["levels"].items(), key=lambda kv: int(kv[0])):
        for which, key in ((0, "x"), (2, "r")):
            got = digest(H.get_vec(int(lev), which))
            assert got == ref[key], f"{name} level {lev} {key}: gpu {got} oracle {ref[key]}"


def test_digest_cases_present():
    """The golden file holds the headline case (the GPU test above needs it)."""
    assert "c2_4097sq" in GOLD and len(GOLD["c2_4097sq"]["levels"]) == 12


@pytest.mark.parametrize("tuner", ["ops", "solve"])
def test_autotuned_shapes_keep_the_headline_digests(tuner):
    """After mg_autotune (launches timed one op at a time) or
    mg_autotune_solve (whole solves timed) picks per-level launch shapes on
    the 4097^2 hierarchy, the solve still matches the oracle's digests on
    every level."""
    g = GOLD["c2_4097sq"]
    c = g["params"]
    p = P.mg_params_init(2, c["L"], c["w"], True, 1, 0, c["N"], POLICY[c["policy"]], c["eta"])
    H = P.Hierarchy(p)
    f = [torch.from_numpy(W.manufactured_f(j, 2)).cuda() for j in range(1, c["L"] + 1)]
    try:
        if tuner == "ops":
            report = H.autotune(reps=3)
        else:
            for j in range(1, c["L"] + 1):
                H.set_rhs(j, f[j - 1])
            report = H.autotune_solve(reps=1)
            for j, r in report.items():
                assert r["star_us"] > 0 and r["star_default_us"] > 0, (j, r)
        print(f"autotuned shapes: {report}", flush=True)
        H.fmg_f64(f)
        for lev, ref in g["levels"].items():
            for which, key in ((0, "x"), (2, "r")):
                got = digest(H.get_vec(int(lev), which))
                assert got == ref[key], f"autotuned level {lev} {key}: gpu {got} oracle {ref[key]}"
    finally:
        P.bfp_tuning_set("level_rows_clear", 0)
