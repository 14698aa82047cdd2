"""Benchmark: BFP full multigrid for 2D Poisson on a 4097 x 4097 grid on one
MI355X.

One step = one complete solve through the library: FP64 right-hand sides
(already resident in HBM) quantized to BFP on every level, FMG with N = 2
IR-V(1,0) iterations per level on 12 levels with progressive widths
(nnqcomp everywhere except the first IR residual of each level, which uses
qcomp), then the normalized BFP solution and the exact dot product of the
final residual. Prints one JSON line.

Also measured (extra keys of the same line): the dominant kernel (the
finest-level 5-point residual) timed with HIP events on the stream it runs
on, the plain 5-point and 7-point stencil applies (4095^2 and 511^3, int32),
the finest inner width sweep, the discretization-accuracy gate, the batched
workload (4096 independent 2D solves of sides 33..257 in one launch) against
a one-solve-at-a-time loop, and the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM traffic of the dominant kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs, valid while the kernel sources hash to the recorded value
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "residual_4095sq_traffic.json")
KERNEL_SOURCES = ["common.hpp", "device.hpp", "epilogue.hpp", "kernels.hpp", "star_impl.hpp",
                  "k_star_x32.hip", "k_star.hip"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2307_00124_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


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
    ap.add_argument("--batch", type=int, default=4096, help="problems of the batched leg (0: skip)")
    ap.add_argument("--loop-sample", type=int, default=32,
                    help="problems solved one at a time for the batched comparison")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes (no autotuning before timing)")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="oracle processes of the CPU baseline (at most the cores available)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the diagnostics, fallback and precision-estimation legs")
    ap.add_argument("--level3d", type=int, default=9, help="3D solve level (0: skip)")
    ap.add_argument("--serve", type=int, default=2000,
                    help="requests of the serving trace (0: skip)")
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="GPU_MAX_HW_QUEUES for this process (0: leave the environment's)")
    ap.add_argument("--fe-program", type=int, choices=[0, 1], default=1,
                    help="finite-element solves as one recorded program (1) or op by op (0)")
    ap.add_argument("--only", choices=["all", "kernel", "copy", "streamcopy", "solve", "fp64",
                                       "coarse", "tiles", "fe"],
                    default="all",
                    help="kernel: only the dominant-kernel loop (for profiler runs); copy: only "
                         "a plain 1 GiB device copy (counter calibration); streamcopy: only the "
                         "library's streaming copy of 1 GiB; solve: only --warmup + "
                         "--steps headline solves (autotuned shapes), nothing else; fp64: only "
                         "the FP64 comparator's solves; coarse: only FMG solves of the 65^2 grid "
                         "(6 levels, all of them inside the coarse-level executor); tiles: only "
                         "the tiled residual loop (T = 64, 4095^2); fe: only the finite-element "
                         "model problems")
    return ap.parse_args()


T0 = time.perf_counter()


def progress(what: str) -> None:
    """One progress line per finished leg on stderr (the JSON result is the
    only line on stdout)."""
    print(f"[bench {time.perf_counter() - T0:7.1f} s] {what}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solves of "
              "this workload are single-GPU and no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)
    # the request server overlaps its slots only as far as HIP has hardware
    # queues (HIP's default is 4); must be set before HIP initializes
    if args.hw_queues > 0:
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
    import numpy as np
    import torch

    import paper_2307_00124_amd as P
    import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    def ev():
        return torch.cuda.Event(enable_timing=True)

    if args.only == "copy":
        a = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 4, "launches": 5}))
        return
    P.bfp_tuning_set("fe_program", args.fe_program)
    if args.only == "fe":
        print(json.dumps({"only": "fe", "finite_elements": bench_fe(P, np, torch, stream, ev)}))
        return
    if args.only == "streamcopy":
        # the library's streaming copy of 1 GiB, plain then non-temporal, for the profiler
        a = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        out = {}
        for nt in (False, True):
            for _ in range(2):
                P.bfp_stream_copy(a, b, nt, stream)
            torch.cuda.synchronize()
            e0, e1 = ev(), ev()
            e0.record(stream)
            for _ in range(10):
                P.bfp_stream_copy(a, b, nt, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 100.0
            out["nt" if nt else "plain"] = {"avg_us": round(us, 1),
                                            "gbs": round(2 * a.numel() * 4 / (us * 1e-6) / 1e9, 1)}
        print(json.dumps({"stream_copy_bytes_each_way": a.numel() * 4, **out}))
        return

    L = args.level
    n = (1 << L) - 1
    dof = n * n
    A2 = P.Stencil(2, P.BFP_STENCIL_A, -2, [0, -1, 0, -1, 4, -1, 0, -1, 0], 4)

    def make(w, N=2, policy=P.MG_POLICY_NN_IR_FIRST_Q):
        p = P.mg_params_init(2, L, w, True, 1, 0, N, policy, 23)
        p.min_storage_bits = 32
        return P.Hierarchy(p)

    f = [None] + [torch.from_numpy(W.manufactured_f(j, 2)).to(dev) for j in range(1, L + 1)]

    def time_kernel(fn, reps):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        k0, k1 = ev(), ev()
        k0.record(stream)
        for _ in range(reps):
            fn()
        k1.record(stream)
        torch.cuda.synchronize()
        return k0.elapsed_time(k1) * 1000.0 / reps

    if args.only == "tiles":
        A, x, b, r, st = tiles_residual_setup(P, W, torch, dev, stream, L, 64)
        one, mone = P.scalar(1, 0, 2), P.scalar(-1, 0, 1)
        t = time_kernel(lambda: P.bfp_tiles_stencil_apply(A, x, one, mone, b, r, st, stream),
                        args.kernel_reps)
        print(json.dumps({"kernel": "tiled residual 4095^2 int32 T=64", "avg_us": t}))
        return

    if args.only in ("solve", "fp64", "coarse"):
        # profiler runs: the headline solve (or the FP64 comparator, or a
        # solve that runs entirely in the coarse-level executor) alone
        rhs = [f[j] for j in range(1, L + 1)]
        if args.only == "coarse":
            pc = P.mg_params_init(2, 6, args.w, True, 1, 0, 2, P.MG_POLICY_NN_IR_FIRST_Q, 23)
            pc.min_storage_bits = 32
            Hc = P.Hierarchy(pc)
            for j in range(1, 7):
                Hc.set_rhs(j, f[j])
            run = lambda: Hc.fmg(stream)
        elif args.only == "solve":
            H = make(args.w)
            for j in range(1, L + 1):
                H.set_rhs(j, f[j], stream)
            if not args.no_autotune:
                H.autotune_solve(reps=3, stream=stream)
            run = lambda: H.fmg_f64(rhs, stream)
        else:
            F = P.FP64MG(P.mg_params_init(2, L, 32, True, 1, 0, 2, P.MG_POLICY_NN_IR_FIRST_Q, 23))
            xo = torch.zeros(((1 << L) + 1,) * 2, dtype=torch.float64, device=dev)
            run = lambda: F.fmg(rhs, xo, stream)
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record(stream)
        for _ in range(args.steps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        print(json.dumps({"only": args.only, "steps": args.steps,
                          "ms_per_step": e0.elapsed_time(e1) / args.steps}))
        return

    # ----------------------------------- dominant kernel, HIP events ---
    # the finest-level IR residual r = A x - b in saturate mode: the 5-point
    # star kernel with a y stream, on the iterate of a finished solve (the
    # same launch the FMG issues)
    H = make(args.w)
    for j in range(1, L + 1):
        H.set_rhs(j, f[j], stream)
    H.fmg(stream)
    x, b, r = H.get_vec(L, 0), H.get_vec(L, 1), H.get_vec(L, 2)
    g = P.gamma_norm(r)
    kern_us = time_kernel(lambda: P.bfp_residual(A2, x, b, r.w, P.BFP_SATURATE, g, r, stream),
                          args.kernel_reps)
    kern_bytes = dof * (x.storage_bits + b.storage_bits + r.storage_bits) / 8.0
    kern_gbs = kern_bytes / (kern_us * 1e-6) / 1e9
    if args.only == "kernel":
        print(json.dumps({"kernel": "residual 4095^2 int32", "avg_us": kern_us, "gbs": kern_gbs}))
        return

    us = torch.from_numpy(W.manufactured_u(L, 2)).to(dev)
    h2 = 2.0 ** (-2 * L)
    kappa = (math.pi * 2.0 ** -L) ** 2 / (4.0 * math.sin(math.pi * 2.0 ** -L / 2.0) ** 2)
    disc = (kappa - 1.0) * math.sqrt(float((us[1:-1, 1:-1] ** 2).sum()) * h2)
    dot_out = torch.zeros(P.BFP_META_SLOTS, dtype=torch.int64, device=dev)

    def step(H, xout):
        # FP64 -> BFP (b_j on every level) and FMG, in one call: the coarse
        # levels' quantization runs inside the coarse-level program, the
        # finer levels' on a second stream meanwhile
        H.fmg_f64(f[1:], stream)
        xl = H.get_vec(L, 0)
        P.bfp_normalize(xl, xl.w, xout, stream)         # normalized solution
        rl = H.get_vec(L, 2)
        P.bfp_dot(rl, rl, dot_out, stream)              # exact r.r

    def timed(H, xout, steps, warmup):
        for _ in range(warmup):
            step(H, xout)
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
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

    progress("dominant kernel timed")
    # ---------------------------------------------------------- main run --
    # per-level launch shapes of the star and transfer kernels, chosen by
    # the library's autotuner from the time of whole solves on this
    # hierarchy (results do not depend on them)
    tune = H.autotune_solve(reps=3, stream=stream) if not args.no_autotune else None
    xout = P.Vec(2, n, H.get_vec(L, 0).w, 32)
    ms = timed(H, xout, args.steps, args.warmup)
    ratio = accuracy(xout)
    bytes_before, launches_before = H.counters()
    step(H, xout)
    torch.cuda.synchronize()
    bytes_after, launches_after = H.counters()
    step_bytes = bytes_after - bytes_before
    step_launches = launches_after - launches_before
    # the same step without the FP64 -> BFP quantization of the right-hand
    # sides (b_j already set): FMG, normalized solution, exact r.r
    for _ in range(2):
        H.fmg(stream)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record(stream)
    for _ in range(args.steps):
        H.fmg(stream)
        P.bfp_normalize(H.get_vec(L, 0), H.get_vec(L, 0).w, xout, stream)
        P.bfp_dot(H.get_vec(L, 2), H.get_vec(L, 2), dot_out, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_no_conv = e0.elapsed_time(e1) / args.steps
    # the solve's hierarchy (and the second stream mg_fmg_f64 created for it,
    # which holds one of HIP's hardware queues) is not needed by the later legs
    del H, x, b, r, xout
    torch.cuda.empty_cache()

    progress("headline solve timed")
    # ------------------------------------- FP64 multigrid comparator ---
    fp64 = bench_fp64(P, torch, f, L, us, h2, disc, stream, ev)

    progress("FP64 comparator timed")
    # --------------------------------------- plain stencil applies ------
    # z = A x (two int32 streams), 2D 4095^2 and 3D 511^3
    stencils = {}
    xs = P.Vec(2, n, 30, 32)
    P.bfp_vec_from_f64(f[L], 0, xs, stream)
    zs = P.Vec(2, n, 32, 32)
    gz = P.gamma_norm(xs, P.scalar(1, 1))
    t2 = time_kernel(lambda: P.bfp_stencil_apply(A2, xs, None, None, None, 32, P.BFP_SATURATE,
                                                 gz, zs, stream), args.kernel_reps)
    stencils["5pt_4095sq_int32"] = {"avg_us": round(t2, 2), "bytes": dof * 8.0,
                                    "gbs": round(dof * 8.0 / (t2 * 1e-6) / 1e9, 1)}
    # a plain device copy of the same bytes (torch), the practical ceiling
    ca = torch.ones(dof * 4, dtype=torch.int32, device=dev)
    cb = torch.empty_like(ca)
    tcp = time_kernel(lambda: cb.copy_(ca), args.kernel_reps)
    stencils["copy_8x4095sq_int32"] = {"avg_us": round(tcp, 2), "bytes": dof * 32.0,
                                       "gbs": round(dof * 32.0 / (tcp * 1e-6) / 1e9, 1)}
    # the library's own streaming copy (16-byte words, four in flight per
    # thread; plain and non-temporal): the hand-written bandwidth reference
    for nt in (False, True):
        tsc = time_kernel(lambda: P.bfp_stream_copy(ca, cb, nt, stream), args.kernel_reps)
        stencils["stream_copy" + ("_nt" if nt else "") + "_8x4095sq_int32"] = {
            "avg_us": round(tsc, 2), "bytes": dof * 32.0,
            "gbs": round(dof * 32.0 / (tsc * 1e-6) / 1e9, 1)}
    del ca, cb
    del xs, zs
    if not args.no_3d:
        n3 = 511
        A3 = P.Stencil(3, P.BFP_STENCIL_A, -3,
                       [6 if k == 13 else (-1 if k in (4, 10, 12, 14, 16, 22) else 0)
                        for k in range(27)], 4)
        x3 = P.Vec(3, n3, 24, 32)
        z3 = P.Vec(3, n3, 32, 32)
        f3 = torch.from_numpy(W.manufactured_f(9, 3)).to(dev)
        P.bfp_vec_from_f64(f3, 0, x3, stream)
        del f3
        g3 = P.gamma_norm(x3, P.scalar(1, 1))
        t3 = time_kernel(lambda: P.bfp_stencil_apply(A3, x3, None, None, None, 32,
                                                     P.BFP_SATURATE, g3, z3, stream), 20)
        d3 = n3 ** 3
        stencils["7pt_511cube_int32"] = {"avg_us": round(t3, 2), "bytes": d3 * 8.0,
                                         "gbs": round(d3 * 8.0 / (t3 * 1e-6) / 1e9, 1)}
        del x3, z3
        torch.cuda.empty_cache()

    progress("stencil applies timed")
    tiles = bench_tiles(P, W, torch, dev, stream, time_kernel, L, args.kernel_reps)
    progress("sub-maximal block sizes timed")
    fe_rows = bench_fe(P, np, torch, stream, ev)
    # -------------------------------------------------- 33x33 latency ---
    c1 = bench_c1(P, W, torch, dev, stream, ev)

    progress("33x33 latencies timed")
    # ------------------------------------------------------- 3D solve ---
    solve3d = None
    if args.level3d > 0:
        solve3d = bench_3d(args, P, W, torch, dev, stream, ev)

    progress("3D solve done")
    # ------------------------------------------------------ width sweep ---
    # per finest inner width w (progressive: one bit less per coarser level):
    # the error with N = 2, then the smallest N <= 8 IR-V iterations per
    # level that reaches 1.1x the discretization error, and its time
    gate_fp64 = 1.1 * fp64["err_over_disc"]
    sweep = []
    for w in [int(s) for s in args.sweep.split(",") if s]:
        row = {"w": w}
        for N in range(2, 9):
            Hs = make(w, N)
            xw = P.Vec(2, n, Hs.get_vec(L, 0).w, 32)
            msw = timed(Hs, xw, 3, 1)
            acc = accuracy(xw)
            del Hs, xw
            if N == 2:
                row.update({"ms_N2": round(msw, 3), "err_over_disc_N2": round(acc, 4)})
            if acc <= 1.1:
                row.update({"N": N, "ms": round(msw, 3), "dof_per_s": dof / (msw * 1e-3),
                            "err_over_disc": round(acc, 4), "at_disc_error": True,
                            "within_1.1x_fp64_mg": acc <= gate_fp64})
                break
        else:
            row.update({"N": "unreached up to 8", "err_over_disc_N8": round(acc, 4),
                        "at_disc_error": False})
        sweep.append(row)
        torch.cuda.empty_cache()
    # the literal "no intermediate normalisation" schedule: nnqcomp for every
    # call, finest inner width args.w, N = 2
    Hn = make(args.w, 2, P.MG_POLICY_NN)
    xn = P.Vec(2, n, Hn.get_vec(L, 0).w, 32)
    ms_nn = timed(Hn, xn, 3, 1)
    acc_nn = accuracy(xn)
    all_nn = {"ms": round(ms_nn, 3), "dof_per_s": dof / (ms_nn * 1e-3),
              "err_over_disc": round(acc_nn, 4), "at_disc_error": acc_nn <= 1.1}
    del Hn, xn
    torch.cuda.empty_cache()

    progress("width sweep done")
    # ----------------------------------------- solve diagnostics -------
    diagnostics = estimation = None
    if not args.no_extras:
        diagnostics = bench_diag(P, torch, f, L, timed, stream)
        diagnostics["ir_fallback"] = bench_fallback(P, W, torch, dev, stream, ev)
        estimation = bench_estimate(torch)
        # the headline solve on the schedule the estimation gives: check and
        # inner widths from q_check / q_inner, eta from the V(1,0) scan; the
        # smallest N per level that reaches the discretization error
        from paper_2307_00124_amd import estimate as est
        pe = est.apply_estimate(P.mg_params_init(2, L, args.w, True, 1, 0, 2,
                                                 P.MG_POLICY_NN_IR_FIRST_Q,
                                                 estimation["eta_v10"]["percent"]),
                                estimation["q_check"], estimation["q_inner"])
        pe.min_storage_bits = 32
        est_solve = {"inner_widths": [pe.w_inner[j] for j in range(1, L + 1)],
                     "check_widths": [pe.w_check[j] for j in range(1, L + 1)],
                     "eta_percent": estimation["eta_v10"]["percent"]}
        for N in range(2, 9):
            pe.N = N
            He = P.Hierarchy(pe)
            xe = P.Vec(2, n, He.get_vec(L, 0).w, 32)
            mse = timed(He, xe, 3, 1)
            acce = accuracy(xe)
            del He, xe
            if N == 2:
                est_solve.update({"ms_N2": round(mse, 3), "err_over_disc_N2": round(acce, 4)})
            if acce <= 1.1:
                est_solve.update({"N": N, "ms": round(mse, 3), "dof_per_s": dof / (mse * 1e-3),
                                  "err_over_disc": round(acce, 4), "at_disc_error": True})
                break
        else:
            est_solve.update({"N": "unreached up to 8", "err_over_disc_N8": round(acce, 4),
                              "at_disc_error": False})
        estimation["solve_4097sq"] = est_solve
        torch.cuda.empty_cache()

    progress("diagnostics and estimation done")
    # --------------------------------------------------- batched solves ---
    batch = None
    if args.batch > 0:
        batch = bench_batch(args, P, W, np, torch, dev, stream, ev)

    progress("batched leg done")
    # ---------------------------------------------------------- serving ---
    serving = None
    if args.serve > 0:
        serving = bench_serve(args, P, W, np, torch, dev)

    progress("serving leg done")
    # ---------------------------------------------------- CPU baseline ----
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.cpu_level, args.w, args.cpu_workers)

    traffic = None
    try:
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("source_sha256") == kernel_source_hash():
            traffic = tr["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        traffic = None

    out = {
        "metric": "BFP-FMG DoF/s at discretization error vs FP64 MG; stencil GB/s; p99 latency",
        "value": dof / (ms * 1e-3),
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_step_without_rhs_quantization": round(ms_no_conv, 3),
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
                   "err_over_fp64_mg_err": round(ratio / fp64["err_over_disc"], 4),
                   "within_1.1x_fp64_mg": ratio <= 1.1 * fp64["err_over_disc"],
                   "launches_per_step": step_launches,
                   "algorithmic_bytes_per_step": step_bytes},
        "roofline": {"bound": "hbm", "achieved": round(kern_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(kern_gbs / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "k_star2d (5-point residual A x - b, int32, finest level)",
                     "avg_us": round(kern_us, 2), "bytes_per_launch": kern_bytes},
        "solve_roofline": {"bound": "hbm", "achieved": round(step_bytes / (ms * 1e-3) / 1e9, 1),
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                           "bytes_per_step": step_bytes,
                           "what": "every input of every quantized operation of the step read "
                                   "once and every output written once (qcomp's second read "
                                   "and halo re-reads not counted), over the step time"},
        "autotune": tune,
        "fp64_mg_comparator": fp64,
        "bfp_over_fp64_dof_per_s": round((dof / (ms * 1e-3)) / fp64["dof_per_s"], 2),
        "stencil_apply": stencils,
        "sub_maximal_blocks": tiles,
        "finite_elements": fe_rows,
        "solve_3d": solve3d,
        "c1_33x33": c1,
        "sweep": sweep,
        "all_nnqcomp_N2": all_nn,
        "diagnostics": diagnostics,
        "precision_estimation": estimation,
        "batched": batch,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def _oracle_fmg(level, w):
    """One oracle FMG solve (test infrastructure: the CPU baseline only)."""
    from fractions import Fraction

    import workloads as W
    from oracle import mg as omg
    fo = {j: W.manufactured_f(j, 2) for j in range(1, level + 1)}
    O = omg.build_hierarchy(fo, 2, level, omg.widths_progressive(level, w),
                            omg.make_smoother(2, Fraction(23, 100)), policy="nn_ir_first_q")
    t0 = time.perf_counter()
    omg.fmg(O, 2)
    return time.perf_counter() - t0


def cpu_baseline(level, w, workers):
    """The oracle (exact Python integers, not tuned) on the host cores: one
    FMG solve of the same method on the (2^level + 1)^2 grid per worker
    process, all workers at once; DoF/s = the workers' fine-grid unknowns
    over the wall time."""
    import multiprocessing as mp
    cores = len(os.sched_getaffinity(0))
    k = max(1, min(workers, cores))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(k) as pool:
        secs = pool.starmap(_oracle_fmg, [(level, w)] * k)
    wall = time.perf_counter() - t0
    ndof = ((1 << level) - 1) ** 2
    return {"value": k * ndof / wall, "unit": "DoF/s", "cores": k, "kind": "oracle",
            "sample": f"{k} concurrent oracle FMG solves (one per process and core) of the same "
                      f"method on the {(1 << level) + 1}^2 grid ({level} levels, finest inner "
                      f"width {w}), exact Python integers; {wall:.1f} s wall, "
                      f"{min(secs):.1f}-{max(secs):.1f} s per solve; {cores} cores available"}


def tiles_residual_setup(P, W, torch, dev, stream, L, T):
    """x (manufactured solution plus noise) and b (f scaled as the solver's
    b), both int32 tiles of T points, and the scaled 5-point operator."""
    n = (1 << L) - 1
    u = torch.from_numpy(W.manufactured_u(L, 2)).to(dev)
    u[1:-1, 1:-1] += 1e-9 * torch.sin(torch.arange(n, device=dev, dtype=torch.float64) * 0.37)
    fb = torch.from_numpy(W.manufactured_f(L, 2)).to(dev) * 2.0 ** (-2 * L - 2)
    x, b, r = (P.Tiles(2, n, T, 32, 32) for _ in range(3))
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    P.bfp_tiles_from_f64(u, x, st, stream)
    P.bfp_tiles_from_f64(fb, b, st, stream)
    A = P.Stencil(2, P.BFP_STENCIL_A, -2, [0, -1, 0, -1, 4, -1, 0, -1, 0], 4)
    return A, x, b, r, st


def bench_tiles(P, W, torch, dev, stream, time_kernel, L, reps):
    """Sub-maximal block sizes: the residual r = A x - b with one exponent
    per tile of T row points (int32, 4095^2) for several T, against the
    maximal block's residual; and the FP64 -> BFP quantization error by
    block size (the paper's remark that the maximal block is the worst
    case)."""
    n = (1 << L) - 1
    dof = n * n
    out = {"residual_4095sq_int32": {}, "quantization_rel_l2_error": {}}
    one, mone = P.scalar(1, 0, 2), P.scalar(-1, 0, 1)
    for T in (1, 8, 64, 256):
        A, x, b, r, st = tiles_residual_setup(P, W, torch, dev, stream, L, T)
        t = time_kernel(lambda: P.bfp_tiles_stencil_apply(A, x, one, mone, b, r, st, stream), reps)
        ntiles = n * -(-n // T)
        nbytes = dof * 12.0 + 3 * 4.0 * ntiles
        out["residual_4095sq_int32"][f"T{T}"] = {
            "avg_us": round(t, 2), "bytes": nbytes, "gbs": round(nbytes / (t * 1e-6) / 1e9, 1),
            "beyond_exact_range": int(st.item())}
        del A, x, b, r, st
    # the fields: the manufactured solution and a residual-like field of
    # many scales (its FP64 residual after a perturbation)
    u = torch.from_numpy(W.manufactured_u(L, 2)).to(dev)
    g = torch.Generator(device=dev).manual_seed(5)
    noise = torch.zeros_like(u)
    noise[1:-1, 1:-1] = torch.randn((n, n), generator=g, device=dev, dtype=torch.float64)
    res = torch.zeros_like(u)
    res[1:-1, 1:-1] = (4 * noise[1:-1, 1:-1] - noise[:-2, 1:-1] - noise[2:, 1:-1] -
                       noise[1:-1, :-2] - noise[1:-1, 2:]) * torch.exp(
        -20.0 * torch.linspace(0, 1, n, device=dev, dtype=torch.float64))[None, :]
    for name, fld in (("solution", u), ("residual", res)):
        ref = float(fld.norm())
        row = {}
        for w in (8, 12, 16):
            v = P.Vec(2, n, w, P.storage_for(w))
            P.bfp_vec_from_f64(fld, 0, v, stream)
            errs = {"maximal": float((P.bfp_vec_to_f64(v) - fld).norm()) / ref}
            for T in (256, 64, 8, 1):
                t = P.Tiles(2, n, T, w, P.storage_for(w))
                P.bfp_tiles_from_f64(fld, t, None, stream)
                back = torch.zeros_like(fld)
                P.bfp_tiles_to_f64(t, back, stream)
                errs[f"T{T}"] = float((back - fld).norm()) / ref
            row[f"w{w}"] = {k: float(f"{e:.3e}") for k, e in errs.items()}
        out["quantization_rel_l2_error"][name] = row
    return out


def fe_widths(kind, p, L):
    """The widest schedule the library's 61-bit exact budgets allow for the
    finite-element problems: A and b at 28 bits, x at 28, the V-cycle at 20
    (the paper's widths for these problems grow past 32 bits on fine
    levels, so the levels below are chosen where these suffice)."""
    return ({j: 28 for j in range(1, L + 1)}, {j: 28 for j in range(1, L + 1)},
            {j: 20 for j in range(1, L + 1)})


def bench_fe(P, np, torch, stream, ev):
    """The paper's finite-element model problems (Section 6): BFP FMG on 1D
    B-spline discretizations, the error against the exact discrete solution
    (FP64 with exactly computed residuals), the smallest N up to 8 that
    reaches 1.1x the discretization error (the paper's N first), time per
    solve (HIP events), launches and DoF/s."""
    from workloads import fe as FW
    out = []
    for kind, p, L in (("poisson", 1, 12), ("poisson", 2, 5), ("poisson", 3, 4),
                       ("biharmonic", 3, 6), ("biharmonic", 5, 3), ("biharmonic", 6, 3)):
        m = 1 if kind == "poisson" else 2
        ck, wk, inn = fe_widths(kind, p, L)
        K = [FW.stiffness(j, p, m) for j in range(1, L + 1)]
        Pm = [None] + [FW.prolongation(j, p, m) for j in range(2, L + 1)]
        F = [FW.load_vector(kind, j, p) for j in range(1, L + 1)]
        disc = FW.l2_error(kind, p, L, FW.discrete_solution(kind, p, L))
        paper_N = FW.PAPER_N[(kind, p)]
        row = {"problem": kind, "p": p, "L": L, "dof": FW.n_unknowns(L, p, m), "paper_N": paper_N,
               "widths": [ck[L], wk[L], inn[L]]}
        tried = [paper_N] + [n for n in range(1, 9) if n != paper_N]
        for N in tried:
            G = P.FEHierarchy(m, L, N, K, Pm, F, ck, wk, inn)
            for _ in range(2):
                G.fmg(stream)
            torch.cuda.synchronize()
            b0, l0 = G.counters()
            e0, e1 = ev(), ev()
            e0.record()
            reps = 10
            for _ in range(reps):
                G.fmg(stream)
            e1.record()
            torch.cuda.synchronize()
            b1, l1 = G.counters()
            ms = e0.elapsed_time(e1) / reps
            mant, e = G.get(L, 0)
            ratio = FW.l2_error(kind, p, L, mant[1:-1].astype(np.float64) * 2.0 ** e) / disc
            if N == paper_N:
                row.update({"err_over_disc_paper_N": round(ratio, 4), "ms_paper_N": round(ms, 3)})
            if ratio <= 1.1:
                row.update({"N": N, "ms": round(ms, 3), "err_over_disc": round(ratio, 4),
                            "launches": int((l1 - l0) / reps), "at_disc_error": True,
                            "dof_per_s": row["dof"] / (ms * 1e-3)})
                break
            del G
        else:
            row.update({"N": "unreached up to 8", "err_over_disc_N8": round(ratio, 4),
                        "at_disc_error": False})
        row["discretization_error_l2"] = disc
        progress(f"finite elements {kind} p {p} L {L}: N = {row['N']}")
        out.append(row)
    return out


def bench_batch(args, P, W, np, torch, dev, stream, ev):
    """The batched workload: independent 2D solves (sides 33..257, 8 sine
    modes, inner width 16 in int16, x and b in int32), all in one launch,
    against the same kind of solves issued one at a time. N per side is the
    calibrated number of IR-V iterations per level that reaches the
    discretization error (calibrate_n); every solve's error is checked."""
    solves = W.batch_trace(args.batch, seed=1)
    sched = {}
    for L in sorted({s.level for s in solves}):
        sched[L] = calibrate_n(P, W, torch, dev, 2, L, 16)
        progress(f"batched schedule level {L}: N = {sched[L][0]} (error {sched[L][1]:.3f}x)")
    prms = [P.batch_params(2, s.level, 16, N=sched[s.level][0] or 16) for s in solves]
    keep = {}
    table = torch.zeros(len(solves) * P.MG_MAX_LEVELS, dtype=torch.int64)
    for i, s in enumerate(solves):
        for j in range(1, s.level + 1):
            t = torch.from_numpy(np.ascontiguousarray(W.sine_f(j, s.modes))).to(dev)
            keep[(i, j)] = t
            table[i * P.MG_MAX_LEVELS + j - 1] = t.data_ptr()
    table = table.to(dev)
    B = P.Batch(prms)
    dof = sum(((1 << s.level) - 1) ** 2 for s in solves)
    for _ in range(2):
        B.solve(table, stream)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    reps = 5
    e0.record(stream)
    for _ in range(reps):
        B.solve(table, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    bytes_per, _ = B.counters()

    # accuracy of every solve: error to the continuum solution over the
    # discrete solution's (closed form: sine modes are eigenvectors of A_h)
    ratios = [err_ratio(torch, P.bfp_vec_to_f64(B.get_vec(i, s.level, 0)), s.level, s.modes, 2, dev)
              for i, s in enumerate(solves)]
    worst = max(ratios)

    # one solve at a time through the per-solve calls, on a sample holding
    # every side equally
    by_side = {}
    for i, s in enumerate(solves):
        by_side.setdefault(s.side, []).append(i)
    per = max(1, args.loop_sample // len(by_side))
    sample = [i for side in sorted(by_side) for i in by_side[side][:per]]
    Hs = [P.Hierarchy(prms[i]) for i in sample]

    def loop():
        for Hh, i in zip(Hs, sample):
            for j in range(1, solves[i].level + 1):
                Hh.set_rhs(j, keep[(i, j)], stream)
            Hh.fmg(stream)

    loop()
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record(stream)
    loop()
    e1.record(stream)
    torch.cuda.synchronize()
    loop_ms = e0.elapsed_time(e1)
    loop_dof = sum(((1 << solves[i].level) - 1) ** 2 for i in sample)
    loop_rate = loop_dof / (loop_ms * 1e-3)
    rate = dof / (ms * 1e-3)
    return {"workload": f"{len(solves)} independent 2D Poisson FMG solves, sides "
                        "{33,65,129,257} (seed 1), 8 sine modes, N IR-V(1,0) per level "
                        "calibrated per side to reach the discretization error, inner w=16 "
                        "int16, x and b int32, one launch", "dof": dof, "ms": round(ms, 3),
            "schedule_N": {str((1 << L) + 1): (v[0] or "unreached") for L, v in sched.items()},
            "dof_per_s": rate, "algorithmic_gbs": bytes_per / (ms * 1e-3) / 1e9,
            "worst_err_over_disc": round(worst, 4),
            "solves_missing_disc_error": sum(q > 1.1 for q in ratios),
            "loop_dof_per_s": loop_rate, "loop_sample": len(sample),
            "speedup_vs_loop": round(rate / loop_rate, 2)}


def bench_fp64(P, torch, f, L, us, h2, disc, stream, ev):
    """FP64 multigrid on the same GPU with the same schedule (FMG, N = 2
    IR-V(1,0), the same Chebyshev coefficients and scaled operators), the
    library's hand-written HIP solver (fp64_mg_*): the floating-point
    comparator of the metric."""
    prm = P.mg_params_init(2, L, 32, True, 1, 0, 2, P.MG_POLICY_NN_IR_FIRST_Q, 23)
    F = P.FP64MG(prm)
    out = torch.zeros(((1 << L) + 1,) * 2, dtype=torch.float64, device=us.device)
    rhs = [f[j] for j in range(1, L + 1)]
    for _ in range(3):
        F.fmg(rhs, out, stream)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    reps = 10
    e0.record(stream)
    for _ in range(reps):
        F.fmg(rhs, out, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    err = math.sqrt(float(((out - us)[1:-1, 1:-1] ** 2).sum()) * h2)
    dof = ((1 << L) - 1) ** 2
    del F, out
    return {"what": "FP64 FMG, same schedule, coefficients and scaled operators, hand-written "
                    "HIP kernels on the same GPU (fp64_mg_fmg; levels of <= 4096 points in one "
                    "single-workgroup launch)",
            "ms": round(ms, 3), "dof_per_s": dof / (ms * 1e-3),
            "err_over_disc": round(err / disc, 4)}


# The estimates table's extra window bits w*_add per call site (Section 6.3,
# Table 1), in the order of the diagnostics sites: IR residual (first /
# later iteration), IR correction, relaxation, V residual, restriction,
# V correction, FMG prolongation.
W_ADD_STAR = (5, 4, 0, 2, 4, 6, 1, 0)
DIAG_SITES = ("ir_res_first", "ir_res", "ir_corr", "relax", "v_res", "restrict", "v_corr",
              "fmg_prol")


def bench_diag(P, torch, f, L, timed, stream):
    """The recomputation table of Section 6.3 for this problem: one FMG with
    qcomp for every call, its finest-level window gaps read from the device
    diagnostics, and the calls Algorithm 1 would recompute with
    w_tmp = w_out + min(w*_add, w_add_max); plus the nnqcomp saturations of
    one step of the timed solve."""
    def make_diag(policy):
        p = P.mg_params_init(2, L, 32, True, 1, 0, 2, policy, 23)
        p.min_storage_bits = 32
        P.bfp_tuning_set("diagnostics", 1)
        try:
            return P.Hierarchy(p)
        finally:
            P.bfp_tuning_set("diagnostics", 0)

    Hq = make_diag(P.MG_POLICY_Q)
    Hq.fmg_f64(f[1:], stream)
    d = Hq.diagnostics(reset=True, stream=stream)[L]
    gaps = P.abi.MG_DIAG_GAP_BINS

    def recomputed(site, w_add):
        row = d[site]
        return int(row[0]) + int(row[2 + w_add:gaps].sum())

    table = {}
    for cap in (None, 4, 2, 0):
        per = {DIAG_SITES[k]: recomputed(k, W_ADD_STAR[k] if cap is None else min(W_ADD_STAR[k], cap))
               for k in range(len(DIAG_SITES))}
        table["inf" if cap is None else str(cap)] = {"total": sum(per.values()),
                                                     "per_site": {k: v for k, v in per.items() if v}}
    xq = P.Vec(2, (1 << L) - 1, Hq.get_vec(L, 0).w, 32)
    ms_q = timed(Hq, xq, 3, 1)
    del Hq, xq
    torch.cuda.empty_cache()
    Hd = make_diag(P.MG_POLICY_NN_IR_FIRST_Q)      # the timed solve's configuration
    xd = P.Vec(2, (1 << L) - 1, Hd.get_vec(L, 0).w, 32)
    ms_d = timed(Hd, xd, 3, 1)
    Hd.diagnostics(reset=True, stream=stream)
    timed(Hd, xd, 1, 0)
    dh = Hd.diagnostics(reset=True, stream=stream)
    del Hd, xd
    torch.cuda.empty_cache()
    return {"what": "finest-level (j = %d) qcomp calls of one FMG with qcomp everywhere "
                    "(progressive widths, N = 2 IR-V(1,0)) that Algorithm 1 recomputes with "
                    "w_tmp = w_out + min(w*_add, w_add_max), w*_add from the estimates table; "
                    "and the nnqcomp saturations of one step of the timed solve" % L,
            "qcomp_calls_finest": int(d[:, :gaps].sum()),
            "recomputations_by_w_add_max": table,
            "all_qcomp_fmg_ms": round(ms_q, 3),
            "timed_solve_ms_with_diagnostics": round(ms_d, 3),
            "timed_solve_nnqcomp_calls": int(dh[:, :, P.abi.MG_DIAG_BINS - 3].sum()),
            "timed_solve_saturated_entries": int(dh[:, :, P.abi.MG_DIAG_BINS - 2].sum())}


def bench_fallback(P, W, torch, dev, stream, ev, L=10, iters=12):
    """IR-V(1,0) from zero on the 1025^2 grid with nnqcomp everywhere (the
    Remark on skipping normalization in IR-V): plain, and with the qcomp
    fallback of mg_ir_safe (q_iters = 2, theta = 1); error over the
    discretization error after `iters` iterations, and the time."""
    n = (1 << L) + 1
    us = torch.from_numpy(W.manufactured_u(L, 2)).to(dev)
    h2 = 2.0 ** (-2 * L)
    kappa = (math.pi * 2.0 ** -L) ** 2 / (4.0 * math.sin(math.pi * 2.0 ** -L / 2.0) ** 2)
    disc = (kappa - 1.0) * math.sqrt(float((us[1:-1, 1:-1] ** 2).sum()) * h2)
    out = {"workload": "2D 1025x1025, IR-V(1,0) from zero, %d iterations, nnqcomp, progressive "
                       "widths (inner 24)" % iters}
    for name in ("plain", "fallback"):
        p = P.mg_params_init(2, L, 24, True, 1, 0, 2, P.MG_POLICY_NN, 23)
        p.min_storage_bits = 32
        H = P.Hierarchy(p)
        for j in range(1, L + 1):
            H.set_rhs(j, torch.from_numpy(W.manufactured_f(j, 2)).to(dev), stream)
        H.set_x(L, torch.zeros((n, n), dtype=torch.float64, device=dev), stream)
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record(stream)
        sw = H.ir_safe(L, iters, 2, (1, 0), stream) if name == "fallback" else H.ir(L, iters, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        u = P.bfp_vec_to_f64(H.get_vec(L, 0))
        err = math.sqrt(float(((u - us)[1:-1, 1:-1] ** 2).sum()) * h2)
        out[name] = {"err_over_disc": round(err / disc, 3), "ms": round(e0.elapsed_time(e1), 3)}
        if name == "fallback":
            out[name]["fallback_iterations"] = sw
        del H
    torch.cuda.empty_cache()
    return out


def bench_estimate(torch, j_c=5, q_max=64, rho_thresh=1.05):
    """Algorithm bfp-prec-est (Section 6.2) on the 33 x 33 level with the
    paper's j_c = 5, q_max = 64 and rho_thresh = 1.05, and the scan of the
    Chebyshev parameter eta = i / 100 minimizing rho_v (Section 5) for the
    two cycle shapes the solves use; searches, device solves and energy
    norms all run in the library."""
    from paper_2307_00124_amd import estimate as est
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = est.bfp_prec_est(est.base_params(2, j_c), q_max, rho_thresh)
    t1 = time.perf_counter()
    for name, nu in (("eta_v10", (1, 0)), ("eta_v22", (2, 2))):
        wide = est.apply_estimate(est.base_params(2, j_c, nu=nu), q_max, q_max)
        i, rho, rates = est.eta_scan(wide, 1, 99)
        r[name] = {"percent": i, "rho_v": round(rho, 6),
                   "rho_v_at_23": round(rates[22], 6), "rho_v_at_13": round(rates[12], 6)}
    torch.cuda.synchronize()
    r = {k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()}
    r.update({"what": "bfp-prec-est on level %d (%d basis vectors), q_max = %d, rho_thresh = %.2f; "
                      "check width rule 3j + q_check, inner width rule j + q_inner (m = 1, k = 2); "
                      "eta = i / 100, i = 1..99, minimizing rho_v for V(1,0) and V(2,2)" %
                      (j_c, ((1 << j_c) - 1) ** 2, q_max, rho_thresh),
              "seconds_prec_est": round(t1 - t0, 2),
              "seconds": round(time.perf_counter() - t0, 2)})
    return r


def bench_c1(P, W, torch, dev, stream, ev):
    """The 33 x 33 problem (5 levels, widths 32): latency of one FMG with
    N = 2 IR-V(2,2) (qcomp) and of 10 IR-V(2,2) iterations from the seeded
    random initial guess, on one stream."""
    p = P.mg_params_init(2, 5, 32, False, 2, 2, 2, P.MG_POLICY_Q, 13)
    H = P.Hierarchy(p)
    for j in range(1, 6):
        H.set_rhs(j, torch.from_numpy(W.manufactured_f(j, 2)).to(dev), stream)
    x0 = torch.from_numpy(W.initial_guess(5, 2, seed=0)).to(dev)

    def lat(fn, reps=20):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1000.0 / reps

    def ir10():
        H.set_x(5, x0, stream)
        H.ir(5, 10, stream)

    return {"workload": "2D 33x33, 5 levels, widths 32, qcomp", "fmg_n2_v22_us": round(lat(lambda: H.fmg(stream)), 1),
            "ir10_v22_from_random_us": round(lat(ir10), 1)}


def bench_3d(args, P, W, torch, dev, stream, ev):
    """3D Poisson, 7-point, (2^L + 1)^3 grid: IR-V(2,2) from zero with
    progressive widths (finest inner 24, working 2L + 8), qcomp for IR
    residuals, nnqcomp elsewhere, until the error reaches 1.1x the
    discretization error; then the same number of iterations timed."""
    L = args.level3d
    n = (1 << L) - 1
    p = P.mg_params_init(3, L, 24, True, 2, 2, 2, P.MG_POLICY_NN_IR_Q, 13)
    p.min_storage_bits = 32
    H = P.Hierarchy(p)
    f = torch.from_numpy(W.manufactured_f(L, 3)).to(dev)
    us = torch.from_numpy(W.manufactured_u(L, 3)).to(dev)
    h = 2.0 ** -L
    kappa = (math.pi * h) ** 2 / (4.0 * math.sin(math.pi * h / 2.0) ** 2)
    inner = (slice(1, -1),) * 3
    norm_us = math.sqrt(float((us[inner] ** 2).sum()) * h ** 3)
    disc = (kappa - 1.0) * norm_us
    x0 = torch.zeros_like(f)
    H.set_rhs(L, f, stream)
    H.set_x(L, x0, stream)
    ratios = []
    for it in range(1, 25):
        H.ir(L, 1, stream)
        u = P.bfp_vec_to_f64(H.get_vec(L, 0), stream=stream)
        err = math.sqrt(float(((u - us)[inner] ** 2).sum()) * h ** 3)
        ratios.append(round(err / disc, 4))
        del u
        if err <= 1.1 * disc:
            break
    K = len(ratios)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record(stream)
    H.set_rhs(L, f, stream)
    H.set_x(L, x0, stream)
    H.ir(L, K, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    b0, _ = H.counters()
    H.ir(L, 1, stream)
    torch.cuda.synchronize()
    b1, _ = H.counters()
    del H, f, us, x0
    torch.cuda.empty_cache()
    return {"workload": f"3D Poisson 7-point {(1 << L) + 1}^3, {L} levels, IR-V(2,2) from zero, "
                        "progressive widths (inner 24, working 2L+8), int32",
            "dof": n ** 3, "iterations": K, "err_over_disc_per_iteration": ratios,
            "at_disc_error": ratios[-1] <= 1.1, "ms": round(ms, 3),
            "dof_per_s": n ** 3 / (ms * 1e-3),
            "algorithmic_gbs_per_iteration": (b1 - b0) / (ms * 1e-3 / K) / 1e9}


def sine_f_dev(torch, j, modes, ndim, dev):
    """The workload's sine-mode right-hand side on the padded level-j grid,
    evaluated on the device (input generation only)."""
    side = (1 << j) + 1
    x = torch.arange(side, dtype=torch.float64, device=dev) * (2.0 ** -j)
    f = torch.zeros((side,) * ndim, dtype=torch.float64, device=dev)
    for i in range(modes.k.shape[0]):
        parts = []
        for d in range(ndim):
            s = torch.sin(math.pi * float(modes.k[i, d]) * x)
            s[0] = 0.0
            s[-1] = 0.0
            parts.append(s)
        t = parts[0]
        for v in parts[1:]:
            t = torch.multiply(v.reshape((-1,) + (1,) * t.dim()), t)
        f += float(modes.a[i]) * t
    return f


def sine_u_dev(torch, j, modes, ndim, dev, discrete):
    """Solution of -Laplace u = sine_f: per mode a_i / lambda_i times the
    mode, lambda_i = pi^2 |k_i|^2 (continuum) or (4 / h^2) sum_d
    sin^2(k_d pi h / 2) (the 5- / 7-point discrete solution; sine modes are
    eigenvectors of the FD operator). Problem data, not BFP arithmetic."""
    h = 2.0 ** -j
    side = (1 << j) + 1
    x = torch.arange(side, dtype=torch.float64, device=dev) * h
    u = torch.zeros((side,) * ndim, dtype=torch.float64, device=dev)
    for i in range(modes.k.shape[0]):
        ks = [float(k) for k in modes.k[i]]
        if discrete:
            lam = (4.0 / h ** 2) * sum(math.sin(k * math.pi * h / 2.0) ** 2 for k in ks)
        else:
            lam = math.pi ** 2 * sum(k * k for k in ks)
        t = None
        for k in ks:
            sv = torch.sin(math.pi * k * x)
            sv[0] = 0.0
            sv[-1] = 0.0
            t = sv if t is None else torch.multiply(sv.reshape((-1,) + (1,) * t.dim()), t)
        u += (float(modes.a[i]) / lam) * t
    return u


def err_ratio(torch, u, j, modes, ndim, dev):
    """||u - u*|| / ||u_h - u*|| (discrete L2 norms over the interior): the
    error of a BFP solution over the discretization error."""
    inner = (slice(1, -1),) * ndim
    us = sine_u_dev(torch, j, modes, ndim, dev, False)
    uh = sine_u_dev(torch, j, modes, ndim, dev, True)
    e = float(((u - us)[inner] ** 2).sum())
    d = float(((uh - us)[inner] ** 2).sum())
    return math.sqrt(e / d) if d > 0 else float("inf")


def calibrate_n(P, W, torch, dev, ndim, L, w, target=1.05, nmax=16, samples=2, seed=99):
    """Schedule autotuning for an accuracy target: the smallest number N of
    IR-V(1,0) iterations per FMG level with which the batched-workload
    schedule (inner width w on every level) brings sine-mode problems of this
    shape (calibration draws, not the trace's) within `target` times the
    discretization error. Returns (N, worst ratio at N) or (None, ratio at
    nmax) when no N up to nmax does."""
    import numpy as np
    g = np.random.default_rng(seed + 1000 * ndim + 10 * L + w)
    draws = [W.draw_sine_modes(g, ndim) for _ in range(samples)]
    rhs = [[sine_f_dev(torch, j, m, ndim, dev) for j in range(1, L + 1)] for m in draws]
    worst = float("inf")
    for N in range(2, nmax + 1):
        H = P.Hierarchy(P.batch_params(ndim, L, w, N=N))
        worst = 0.0
        for m, r in zip(draws, rhs):
            H.fmg_f64(r)
            u = P.bfp_vec_to_f64(H.get_vec(L, 0))
            worst = max(worst, err_ratio(torch, u, L, m, ndim, dev))
        del H
        if worst <= target:
            return N, worst
    return None, worst


def bench_serve(args, P, W, np, torch, dev):
    """The serving workload: open-loop Poisson arrivals (2000 req/s) of mixed
    2D/3D solves of mixed sizes and widths, run by the request server with
    several slots, against the same trace through a one-slot server (solves
    one after the other). Each request's schedule keeps its width w as the
    inner width on every level and takes the number of IR-V iterations per
    FMG level that calibration solves of its shape need to reach the
    discretization error (calibrate_n); every served result is then checked
    against the closed-form discrete solution, and requests that miss 1.1x
    are reported apart."""
    trace = W.serving_trace(args.serve, rate=2000.0, seed=2)
    classes = sorted({(r.ndim, r.level, r.w) for r in trace})
    t0 = time.perf_counter()
    sched = {}
    for c in classes:
        sched[c] = calibrate_n(P, W, torch, dev, *c)
        progress(f"serving schedule {c[0]}D level {c[1]} w {c[2]}: N = {sched[c][0]} "
                 f"(error {sched[c][1]:.3f}x)")
    calib_s = time.perf_counter() - t0
    prms, rhs, outs, dofs = [], [], [], []
    for r in trace:
        L = r.level
        N = sched[(r.ndim, L, r.w)][0] or 16
        prms.append(P.batch_params(r.ndim, L, r.w, N=N))
        rhs.append([sine_f_dev(torch, j, r.modes, r.ndim, dev) for j in range(1, L + 1)])
        outs.append(torch.zeros(((1 << L) + 1,) * r.ndim, dtype=torch.float64, device=dev))
        dofs.append(((1 << L) - 1) ** r.ndim)
    torch.cuda.synchronize()

    def run(slots, count):
        S = P.Server(48 << 30, max_slots=slots)
        # warm-up: one resident hierarchy per parameter set and slot
        seen = {}
        for i in range(count):
            key = (trace[i].ndim, trace[i].level, trace[i].w)
            seen.setdefault(key, i)
        warm = {S.submit(prms[i], rhs[i], outs[i]) for i in seen.values() for _ in range(slots)}
        while warm:
            for t, st, _ in S.collect():
                warm.discard(t)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nxt, pending, lat, done_at = 0, {}, [0.0] * count, []
        while nxt < count or pending:
            now = time.perf_counter() - t0
            while nxt < count and trace[nxt].t_arrival <= now:
                pending[S.submit(prms[nxt], rhs[nxt], outs[nxt])] = nxt
                nxt += 1
            for t, st, _ in S.collect():
                i = pending.pop(t)
                fin = time.perf_counter() - t0
                lat[i] = fin - trace[i].t_arrival
                done_at.append(fin)
        span = max(done_at) - trace[0].t_arrival
        return lat, span

    def summary(lat, span, idx):
        if not idx:
            return {"requests": 0}
        ms = np.asarray([lat[i] for i in idx]) * 1e3
        return {"requests": len(idx), "p50_ms": round(float(np.percentile(ms, 50)), 3),
                "p99_ms": round(float(np.percentile(ms, 99)), 3),
                "dof_per_s": sum(dofs[i] for i in idx) / span}

    lat, span = run(args.serve_slots, len(trace))
    torch.cuda.synchronize()
    ratios = [err_ratio(torch, outs[i], r.level, r.modes, r.ndim, dev) for i, r in enumerate(trace)]
    ok = [i for i, q in enumerate(ratios) if q <= 1.1]
    miss = [i for i, q in enumerate(ratios) if q > 1.1]
    served = summary(lat, span, list(range(len(trace))))
    served.update({"slots": args.serve_slots, "span_s": round(span, 3)})
    at_disc = summary(lat, span, ok)
    seq_n = min(len(trace), 500)
    lat1, span1 = run(1, seq_n)
    seq = summary(lat1, span1, list(range(seq_n)))
    seq.update({"slots": 1, "span_s": round(span1, 3)})
    offered = sum(dofs) / trace[-1].t_arrival
    by_w = {}
    for w in sorted({r.w for r in trace}):
        idx = [i for i, r in enumerate(trace) if r.w == w]
        by_w[str(w)] = {"requests": len(idx), "at_disc_error": sum(ratios[i] <= 1.1 for i in idx),
                        "worst_err_over_disc": round(max(ratios[i] for i in idx), 4)}
    # alone vs in the mix: re-solve a few requests one at a time
    same = True
    mix = [outs[i].clone() for i in range(8)]
    S1 = P.Server(8 << 30, max_slots=1)
    for i in range(8):
        outs[i].zero_()
        t = S1.submit(prms[i], rhs[i], outs[i])
        while S1.poll(t) is None:
            pass
    torch.cuda.synchronize()
    for i in range(8):
        same = same and bool(torch.equal(outs[i], mix[i]))
    return {"workload": f"{len(trace)} requests, Poisson arrivals at 2000/s (seed 2), 50% 2D "
                        "sides 65..1025, 50% 3D sides 33..129, w in {8,16,24,32} (the inner "
                        "width on every level), FMG with N IR-V(1,0) per level, N calibrated "
                        "per (dim, level, w) to reach the discretization error",
            "schedule_N": {f"{c[0]}D L{c[1]} w{c[2]}": (v[0] if v[0] else "unreached")
                           for c, v in sched.items()},
            "calibration_s": round(calib_s, 2),
            "offered_dof_per_s": offered,
            "server": served, "server_at_disc_error": at_disc,
            "requests_missing_disc_error": len(miss), "by_w": by_w,
            "sequential_one_slot": seq,
            "speedup_dof_per_s": round(served["dof_per_s"] / seq["dof_per_s"], 2),
            "alone_equals_mix": same}


if __name__ == "__main__":
    main()
