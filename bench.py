"""Benchmark: BFP full multigrid for 2D Poisson on a 4097 x 4097 grid on one
MI355X.

One step = one complete solve through the library: FP64 right-hand sides
(already resident in HBM) quantized to BFP on every level, FMG with N = 2
IR-V(1,0) iterations per level on 12 levels with progressive widths
(nnqcomp everywhere except the first IR residual of each level, which uses
qcomp), then the normalized BFP solution and the exact dot product of the
final residual. Prints one JSON line.

Also measured: the dominant kernel (the finest-level 5-point residual) timed
with HIP events on the stream it runs on, the finest inner width sweep, the
discretization-accuracy gate, and the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--level", type=int, default=12)
    ap.add_argument("--w", type=int, default=32, help="finest inner mantissa width")
    ap.add_argument("--sweep", default="8,12,16,24,32")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-level", type=int, default=10)
    ap.add_argument("--kernel-reps", type=int, default=50)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solves of "
              "this workload are single-GPU and no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2307_00124_amd as P
    import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    L = args.level
    n = (1 << L) - 1
    dof = n * n

    def make(w):
        p = P.mg_params_init(2, L, w, True, 1, 0, 2, P.MG_POLICY_NN_IR_FIRST_Q, 23)
        p.min_storage_bits = 32
        H = P.Hierarchy(p)
        return H

    f = [None] + [torch.from_numpy(W.manufactured_f(j, 2)).to(dev) for j in range(1, L + 1)]
    us = torch.from_numpy(W.manufactured_u(L, 2)).to(dev)
    h2 = 2.0 ** (-2 * L)
    kappa = (math.pi * 2.0 ** -L) ** 2 / (4.0 * math.sin(math.pi * 2.0 ** -L / 2.0) ** 2)
    disc = (kappa - 1.0) * math.sqrt(float((us[1:-1, 1:-1] ** 2).sum()) * h2)
    dot_out = torch.zeros(P.BFP_META_SLOTS, dtype=torch.int64, device=dev)

    def step(H, xout):
        for j in range(1, L + 1):
            H.set_rhs(j, f[j], stream)                  # a1: FP64 -> BFP (b_j)
        H.fmg(stream)                                   # a2-a13
        x = H.get_vec(L, 0)
        P.bfp_normalize(x, x.w, xout, stream)           # a7: normalized solution
        r = H.get_vec(L, 2)
        P.bfp_dot(r, r, dot_out, stream)                # a5: exact r.r

    def timed(H, xout, steps, warmup):
        for _ in range(warmup):
            step(H, xout)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            step(H, xout)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def accuracy(xout):
        u = P.bfp_vec_to_f64(xout)
        err = math.sqrt(float(((u - us)[1:-1, 1:-1] ** 2).sum()) * h2)
        return err / disc

    # ---------------------------------------------------------- main run --
    H = make(args.w)
    xout = P.Vec(2, n, H.get_vec(L, 0).w, 32)
    ms = timed(H, xout, args.steps, args.warmup)
    ratio = accuracy(xout)
    bytes_before, launches_before = H.counters()
    step(H, xout)
    torch.cuda.synchronize()
    bytes_after, launches_after = H.counters()
    step_bytes = bytes_after - bytes_before
    step_launches = launches_after - launches_before

    # -------------------------------------- dominant kernel, HIP events ---
    # the finest-level IR residual r = A x - b in saturate mode: the 5-point
    # star kernel with a y stream, the same launch the FMG issues
    x, b, r = H.get_vec(L, 0), H.get_vec(L, 1), H.get_vec(L, 2)
    A = P.Stencil(2, P.BFP_STENCIL_A, -2, [0, -1, 0, -1, 4, -1, 0, -1, 0], 4)
    g = P.gamma_norm(r)
    for _ in range(3):
        P.bfp_residual(A, x, b, r.w, P.BFP_SATURATE, g, r, stream)
    torch.cuda.synchronize()
    k0 = torch.cuda.Event(enable_timing=True)
    k1 = torch.cuda.Event(enable_timing=True)
    k0.record(stream)
    for _ in range(args.kernel_reps):
        P.bfp_residual(A, x, b, r.w, P.BFP_SATURATE, g, r, stream)
    k1.record(stream)
    torch.cuda.synchronize()
    kern_us = k0.elapsed_time(k1) * 1000.0 / args.kernel_reps
    kern_bytes = dof * (x.storage_bits + b.storage_bits + r.storage_bits) / 8.0
    kern_gbs = kern_bytes / (kern_us * 1e-6) / 1e9
    # restore the solver state touched above
    step(H, xout)
    torch.cuda.synchronize()

    # ------------------------------------------------------ width sweep ---
    sweep = []
    for w in [int(s) for s in args.sweep.split(",") if s]:
        Hs = make(w)
        xs = P.Vec(2, n, Hs.get_vec(L, 0).w, 32)
        msw = timed(Hs, xs, 3, 1)
        sweep.append({"w": w, "ms": round(msw, 3), "dof_per_s": dof / (msw * 1e-3),
                      "err_over_disc": round(accuracy(xs), 4),
                      "at_disc_error": accuracy(xs) <= 1.1})
        del Hs, xs
        torch.cuda.empty_cache()

    # ---------------------------------------------------- CPU baseline ----
    cpu = None
    if not args.no_cpu:
        from fractions import Fraction

        from oracle import mg as omg
        Lc = args.cpu_level
        fo = {j: W.manufactured_f(j, 2) for j in range(1, Lc + 1)}
        O = omg.build_hierarchy(fo, 2, Lc, omg.widths_progressive(Lc, args.w),
                                omg.make_smoother(2, Fraction(23, 100)), policy="nn_ir_first_q")
        t0 = time.perf_counter()
        omg.fmg(O, 2)
        t = time.perf_counter() - t0
        ndof = ((1 << Lc) - 1) ** 2
        cpu = {"value": ndof / t, "unit": "DoF/s", "cores": 1, "kind": "oracle",
               "sample": f"one FMG solve of the same method on the {(1 << Lc) + 1}^2 grid "
                         f"({Lc} levels, finest inner width {args.w}), exact Python integers, "
                         f"{t:.1f} s"}

    out = {
        "metric": "BFP-FMG DoF/s at discretization error vs FP64 MG; stencil GB/s; p99 latency",
        "value": dof / (ms * 1e-3),
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32 mantissas, int64 accumulate",
        "data": "synthetic: manufactured solution sin(pi x) sin(pi y), f = 2 pi^2 u*",
        "config": {"workload": f"2D Poisson, 5-point, {(1 << L) + 1}x{(1 << L) + 1} grid, "
                               f"BFP FMG {L} levels, N=2 IR-V(1,0), progressive widths, "
                               f"finest inner w={args.w}, nnqcomp with qcomp for the first IR "
                               f"residual per level", "dof": dof,
                   "err_over_disc": round(ratio, 4), "at_disc_error": ratio <= 1.1,
                   "launches_per_step": step_launches,
                   "algorithmic_bytes_per_step": step_bytes},
        "roofline": {"bound": "hbm", "achieved": round(kern_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(kern_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_star2d (5-point residual A x - b, int32, finest level)",
                     "avg_us": round(kern_us, 2), "bytes_per_launch": kern_bytes},
        "solve_algorithmic_gbs": step_bytes / (ms * 1e-3) / 1e9,
        "sweep": sweep,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
