"""Write tests/golden/fmg_digests.json: per-level digests of the oracle's
solves at the sizes the benchmark workloads run, for the GPU parity test
(tests/test_gpu_digests.py). Calls only oracle/ and workloads/ (no GPU, no
library); run from the repository root:

    python tests/golden/make_fmg_digests.py            # every case
    python tests/golden/make_fmg_digests.py c2_4097sq  # one case

A digest is the block exponent and the sha256 of its mantissas as
little-endian int64 over the whole padded (2^j + 1)^d array (ring
included), C order. The 4097^2 case takes the oracle about 10 minutes and a
few GB of memory."""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time
from fractions import Fraction

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import mg  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fmg_digests.json")

# name -> solve: FMG with N IR-V(nu1, nu2) per level, or IR from x0 = 0 on
# the finest level only (iters > 0)
CASES = {
    # the headline workload: 2D 4097^2, 12 levels, finest inner width 32,
    # progressive widths, nnqcomp except the first IR residual per level
    "c2_4097sq": dict(ndim=2, L=12, w=32, policy="nn_ir_first_q", eta=23, nu=(1, 0), N=2),
    # 3D FMG on 129^3 (7 levels), finest inner width 24
    "fmg3d_129": dict(ndim=3, L=7, w=24, policy="nn_ir_first_q", eta=23, nu=(1, 0), N=2),
    # the 3D solve schedule (IR-V(2,2) from zero, qcomp IR residuals) on 129^3
    "ir3d_129": dict(ndim=3, L=7, w=24, policy="nn_ir_q", eta=13, nu=(2, 2), iters=6),
}


def digest(b) -> dict:
    m = np.asarray(b.m.astype(np.int64), dtype="<i8")
    return {"exp": int(b.e), "sha256": hashlib.sha256(m.tobytes()).hexdigest(),
            "max": int(m.max()), "min": int(m.min())}


def run(name: str, c: dict) -> dict:
    ndim, L = c["ndim"], c["L"]
    f = {j: W.manufactured_f(j, ndim) for j in range(1, L + 1)}
    H = mg.build_hierarchy(f, ndim, L, mg.widths_progressive(L, c["w"]),
                           mg.make_smoother(ndim, Fraction(c["eta"], 100)), policy=c["policy"],
                           nu1=c["nu"][0], nu2=c["nu"][1])
    t = time.time()
    out = {"params": {k: (list(v) if isinstance(v, tuple) else v) for k, v in c.items()}}
    if c.get("iters"):
        x0 = mg.zero_block(L, ndim, H.widths.work[L])
        x, hist = mg.ir_solve(H, x0, c["iters"])
        out["levels"] = {str(L): {"x": digest(x), "r": digest(hist[-1])}}
    else:
        last = {}
        orig = mg.ir_iteration

        def tracked(H_, l, x, g, force_q=False, first=False):
            xn, r = orig(H_, l, x, g, force_q=force_q, first=first)
            last[l] = (xn, r)
            return xn, r
        mg.ir_iteration = tracked
        try:
            mg.fmg(H, c["N"])
        finally:
            mg.ir_iteration = orig
        out["levels"] = {str(l): {"x": digest(last[l][0]), "r": digest(last[l][1])}
                         for l in range(1, L + 1)}
    out["oracle_seconds"] = round(time.time() - t, 1)
    return out


def main(names) -> None:
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        print(f"{name} ...", flush=True)
        data[name] = run(name, CASES[name])
        print(f"{name}: {data[name]['oracle_seconds']} s", flush=True)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
