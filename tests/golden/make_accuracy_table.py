"""Write tests/golden/accuracy_table.json: the discretization-error ratio
||u - u*|| / ||u_h - u*|| (discrete L2) of the oracle's BFP FMG on the 2D
manufactured problem for several inner-width schedules, policies and
iteration counts, and of an FP64 model of the same FMG whose every
quantized result is rounded to the same widths either by floor (the
method's truncation) or to nearest. Calls only oracle/ and workloads/; run
from the repository root (about 10 minutes):

    python tests/golden/make_accuracy_table.py

What it shows: inner widths that grow by one bit per level (j + c, the
Section 5 rule with m = 1, which bounds the energy-norm convergence rate)
leave an algebraic error that grows against the O(h^2) discretization error
in the L2 norm; with floor truncation every residual carries a bias of about
half a unit in its last place, a smooth perturbation that the V-cycle maps
to a smooth error of about 2^-w relative size, while the discretization
error falls as 4^-j. Rounding to nearest at the same widths removes the
effect; two bits per level (2j + c) keep it below the gate."""
from __future__ import annotations

import json
import math
import os
import sys
import time
from fractions import Fraction

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import fp64, mg  # noqa: E402
from oracle.fp64 import FP64MG, apply_f64  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "accuracy_table.json")


def inner_rule(rule: str):
    kind, c = rule.split("+")
    c = int(c)
    return (lambda j: j + c) if kind == "j" else (lambda j: 2 * j + c)


def oracle_ratio(L: int, rule: str, N: int, policy: str) -> dict:
    work = {j: min(32, 2 * j + 8) for j in range(1, L + 1)}
    fn = inner_rule(rule)
    inner = {j: min(work[j], max(5, fn(j))) for j in range(1, L + 1)}
    wd = mg.Widths({j: 32 for j in range(1, L + 1)}, work, inner)
    f = {j: W.manufactured_f(j, 2) for j in range(1, L + 1)}
    H = mg.build_hierarchy(f, 2, L, wd, mg.make_smoother(2, Fraction(23, 100)), policy=policy)
    u = mg.fmg(H, N).to_f64()
    us = W.manufactured_u(L, 2)
    uh = fp64.discrete_solution_manufactured(us, L)
    d = fp64.l2_error(uh, us, L)
    return {"ratio": round(fp64.l2_error(u, us, L) / d, 4),
            "algebraic_over_disc": round(fp64.l2_error(u, uh, L) / d, 4)}


class RoundedMG(FP64MG):
    """The FP64 FMG with every result of the BFP schedule rounded to its
    width relative to its own maximum (qcomp's exponent), by floor or to
    nearest."""

    def __init__(self, *a, inner, work, nearest, **k):
        super().__init__(*a, **k)
        self.inner, self.work, self.nearest = inner, work, nearest

    def q(self, v, w):
        m = np.abs(v).max()
        if m == 0:
            return v
        e = math.floor(math.log2(m)) + 2 - w
        s = v / 2.0 ** e
        return (np.round(s) if self.nearest else np.floor(s)) * 2.0 ** e

    def relax0(self, l, r):
        return self.q(super().relax0(l, r), self.inner[l])

    def vcycle(self, l, r):
        w = self.inner[l]
        y = self.relax0(l, r)
        if l > 1:
            rv = self.q(apply_f64(self.A[l], y) - r, w)
            d = self.vcycle(l - 1, self.q(apply_f64(self.R[l], rv), w))
            y = self.q(y - apply_f64(self.P, d), w)
        return y

    def ir(self, l, x):
        r = self.q(apply_f64(self.A[l], x) - self.b[l], self.inner[l])
        return self.q(x - self.vcycle(l, r), self.work[l])

    def fmg(self, N, L=None):
        x = np.zeros((3, 3))
        for l in range(1, self.L + 1):
            if l > 1:
                x = self.q(apply_f64(self.P, x), self.work[l])
            for _ in range(N):
                x = self.ir(l, x)
        return x


def model_ratio(L: int, rule: str, N: int, nearest: bool) -> float:
    sm = mg.make_smoother(2, Fraction(23, 100))
    work = {j: min(32, 2 * j + 8) for j in range(1, L + 1)}
    fn = inner_rule(rule)
    inner = {j: min(work[j], max(5, fn(j))) for j in range(1, L + 1)}
    f = {j: W.manufactured_f(j, 2) for j in range(1, L + 1)}
    m = RoundedMG(f, 2, L, float(sm.c1.value), float(sm.c2.value), inner=inner, work=work,
                  nearest=nearest)
    u = m.fmg(N)
    us = W.manufactured_u(L, 2)
    uh = fp64.discrete_solution_manufactured(us, L)
    return round(fp64.l2_error(u, us, L) / fp64.l2_error(uh, us, L), 4)


def main() -> None:
    t = time.time()
    table = {"oracle": [], "fp64_model": []}
    for L in (8, 9, 10):
        for rule, N, policy in (("j+12", 2, "nn_ir_first_q"), ("j+12", 2, "q"),
                                ("j+12", 3, "nn_ir_first_q"), ("j+12", 4, "nn_ir_first_q"),
                                ("2j+6", 2, "nn_ir_first_q"), ("2j+8", 2, "nn_ir_first_q")):
            r = oracle_ratio(L, rule, N, policy)
            table["oracle"].append({"L": L, "inner": rule, "N": N, "policy": policy, **r})
            print(table["oracle"][-1], flush=True)
    for L in (8, 10, 12):
        for rule in ("j+12", "j+16", "2j+4", "2j+8"):
            for nearest in (False, True):
                table["fp64_model"].append({"L": L, "inner": rule, "N": 2,
                                            "rounding": "nearest" if nearest else "floor",
                                            "ratio": model_ratio(L, rule, 2, nearest)})
                print(table["fp64_model"][-1], flush=True)
    table["seconds"] = round(time.time() - t, 1)
    with open(OUT, "w") as fh:
        json.dump(table, fh, indent=1)


if __name__ == "__main__":
    main()
