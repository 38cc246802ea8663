"""Benchmark of the SMPM deflated Schur complement solver on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|mixed]

A step is one full solve (Algorithm 3: right-hand side, null-space projections,
B A^{-1}, deflated block-Jacobi GMRES to the 1e-10 relative tolerance,
back-substitution, constant removal) of the 16 x 16 element, n = 16 workload
on [0,2]^2 (r = 65,536 nodes, k = 15,360 interface slots) with a seeded
random-Fourier source.  Inputs are resident in HBM before the timed region.

Prints one JSON line.  Besides the headline solves/s it reports the roofline of
the metric kernel, the Schur apply on the 128 x 128, n = 16 stretched grid with
8 right-hand sides over rotated cold buffers (timed with HIP events around graph
replays on the stream it is launched on), the batched and mixed-precision forms,
the concurrent solve of the three side grids, and the CPU oracle timed on a
bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import faulthandler

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import smpm_workloads as wl  # noqa: E402

HBM_PEAK_GBS = 8000.0


# HBM traffic of the metric kernel per launch, from two rocprofv3 --pmc runs of
# `python bench.py --roofline-only` (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch,
# averaged over the timed launches), each scaled by the counter's reading for a
# plain kernel of known size (FETCH_SIZE reads half of a 64 MiB elementwise read,
# so x2.0; WRITE_SIZE matches a 64 MiB fill, x1.0).  Valid only for the kernel
# source it was measured on (sha256 of the Schur section below); otherwise null.
SCHUR_TRAFFIC = {"fetch_kib": 36565.6, "write_kib": 65024.0,
                 "kernels_sha256": "53deb40964168ebb0fcbe34120be1a09179a4ce398415059bf339da90bab6ff4"}


def kernels_sha256():
    """sha256 of the metric kernel's source: the matrix-core helpers of the Schur
    apply section of csrc/smpm_kernels.hip and the column-pipelined kernel."""
    import hashlib
    path = os.path.join(ROOT, "paper_1601_03432_amd", "csrc", "smpm_kernels.hip")
    txt = open(path).read()
    a = txt.index("// ------------------------------------------------------------------ Schur apply on matrix cores")
    b = txt.index("// KT = 4-deep steps (4*KT >= 4n")
    c = txt.index("// Column-pipelined variant (no side sums)")
    d = txt.index("// Warp-specialized persistent variant (no side sums)")
    return hashlib.sha256((txt[a:b] + txt[c:d]).encode()).hexdigest()


def graph_time_us(launch, launches, replays=20):
    """Average duration of one launch: `launches` calls of `launch` captured in a HIP
    graph, replayed `replays` times between HIP events on the replaying stream, after
    replays // 2 untimed replays (the GPU clock settles; the first replays after setup
    run a few percent slower)."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(3):
            launch()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(launches):
            launch()
    for _ in range(max(1, replays // 2)):
        g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(replays):
        g.replay()
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) * 1e3 / (replays * launches)


def rotated_schur_us(ctx, ncol, pool_bytes=600e6, precision=None):
    """Average Schur-apply launch time over (v, Sv) buffer pairs rotated so that
    the pool exceeds the 256 MB Infinity Cache: every launch streams from HBM.
    precision: None for smpm_schur_apply (FP64), else the operator precision of
    smpm_schur_apply_prec."""
    import torch
    nbuf = max(2, int(np.ceil(pool_bytes / (2 * ncol * ctx.k * 8))))
    ins = [torch.randn(ncol, ctx.k, dtype=torch.float64, device="cuda") for _ in range(nbuf)]
    outs = [torch.empty(ncol, ctx.k, dtype=torch.float64, device="cuda") for _ in range(nbuf)]
    it = {"i": 0}

    def one():
        i = it["i"] % nbuf
        if precision is None:
            ctx.schur_apply_into(ins[i], outs[i])
        else:
            ctx.schur_apply_prec(ins[i], outs[i], precision)
        it["i"] += 1

    us = graph_time_us(one, nbuf, replays=max(4, 200 // nbuf))
    return us, nbuf


def c5_context(smpm, w5):
    """The large stretched grid's context with the metric kernel's launch shape fixed
    (the column-pipelined matrix-core kernel, one tile and 8 columns per workgroup:
    the fastest shape for 8 columns in the autotuner's timings), so every run times
    the same kernel."""
    keys = ("SMPM_SCHUR_NC", "SMPM_SCHUR_PERSIST", "SMPM_SCHUR_CPW")
    saved = {k: os.environ.get(k) for k in keys}
    os.environ.pop("SMPM_SCHUR_NC", None)
    os.environ["SMPM_SCHUR_PERSIST"], os.environ["SMPM_SCHUR_CPW"] = "3", "8"
    try:
        return smpm.Context.from_workload(w5)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def schur_roofline(ctx5, ncol=8, precision=None):
    """The metric kernel: the FP64 Schur apply t = S y on the large stretched grid
    (128 x 128 elements, n = 16) for its 8 right-hand sides, launched as
    k_schur_cols<false,16,8,double,true> (the standalone apply, output written with
    non-temporal stores).  Algorithmic bytes per launch: each column's y read and t
    written once (2 k 8 B per column) plus every distinct element operator once.
    precision = MIXED_FP32 times the same kernel with the FP32 operator copies (FP32
    matrix cores and accumulation, FP64 vectors), the mixed-precision solves' apply."""
    from paper_1601_03432_amd import smpm
    if precision is None or precision == smpm.FP64:
        us, nbuf = rotated_schur_us(ctx5, ncol)
        op_bytes = ctx5.stats()["schur_operator_bytes"]
        kname = "k_schur_cols<false,16,8,double,true>"
    else:
        us, nbuf = rotated_schur_us(ctx5, ncol, precision=precision)
        op_bytes = ctx5.stats()["schur_operator_bytes"] // 2
        kname = "k_schur_cols<false,16,8,float,false>"
    alg_bytes = 2 * ncol * ctx5.k * 8 + op_bytes
    achieved = alg_bytes / (us * 1e-6) / 1e9
    traffic = None
    if (precision is None or precision == smpm.FP64) and SCHUR_TRAFFIC \
            and SCHUR_TRAFFIC.get("kernels_sha256") == kernels_sha256():
        traffic = 1024 * (2.0 * SCHUR_TRAFFIC["fetch_kib"] + 1.0 * SCHUR_TRAFFIC["write_kib"])
    return {"kernel": "%s (Schur apply, 128x128 n=16 stretched grid, %d columns, %d rotated buffer pairs)"
                      % (kname, ncol, nbuf),
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "alg_bytes_per_launch": alg_bytes, "avg_launch_us": us}


def _l2_mean_free(w, a):
    """GLL-quadrature L2 norm of a after removing its weighted mean."""
    a = a - (w @ a) / w.sum()
    return float(np.sqrt(w @ (a * a)))


def paper_study(smpm, torch):
    """The paper's experiments on the GPU path (Sec. 3.1-3.3): lambda = 7 cosine source,
    zero Neumann data, tolerance 1e-10; iterations of Algorithms 1/2/3 with the
    library's stopping rule (relative to |b_hat|) and of Algorithm 3 with the paper's
    (relative to the initial GMRES residual |P b_hat|), the discretization error of the
    solution against the analytic one (GLL-quadrature L2 after removing the means),
    for the default Robin reading and for the literal R = I + n.grad."""
    def run(m, n, robin, alpha):
        c = smpm.Context(m, m, n, wl.uniform_breaks(m), wl.uniform_breaks(m), alpha, robin=robin)
        xs, ys = c.node_coords()
        ua, fa = wl.manufactured_cos(xs, ys, lam=7)
        fs = torch.tensor(fa, device="cuda").reshape(1, -1)
        its, u3 = [], None
        for v in (1, 2, 3):
            u, info = c.solve(fs, tol=1e-10, maxit=1000, variant=v, raise_on_noconv=False)
            its.append(info.iterations if info.status == smpm.OK else None)
            if v == 3:
                u3 = u.cpu().numpy()[0]
        _, info_p = c.solve(fs, tol=1e-10, maxit=1000, variant=3, stop_rule=1, raise_on_noconv=False)
        paper_rule = info_p.cycle_iterations[0] if info_p.status == smpm.OK else None
        w = c.quadrature_weights()
        err = _l2_mean_free(w, u3 - ua) / _l2_mean_free(w, ua)
        return {"alg1": its[0], "alg2": its[1], "alg3": its[2],
                "alg3_paper_rule": paper_rule,
                "rel_l2_error": err}

    res = {"columns": "iterations of Algorithms 1/2/3 (stop at 1e-10 |b_hat|), Algorithm 3 under the paper's "
                      "rule (1e-10 |P b_hat|), relative GLL-L2 error vs the analytic solution",
           "paper_context": "m=32, n=5: unpreconditioned slightly below 110, deflated slightly above 30 "
                            "(Sec. 3.2); m=4: all under 40, preconditioned under 15 (Sec. 3.3); the error "
                            "falls with h and spectrally with p (Sec. 3.1)"}
    # the literal reading runs at penalty 32: at 8 its S is nearly singular beyond the
    # null vector on the finer grids (sigma_2 ~ 3e-6 at m = 32) and no iteration converges
    for robin, alpha in (("min", smpm.DEFAULT_PENALTY), ("literal", 32.0)):
        res[robin] = {
            "penalty": alpha,
            "h_refinement_n5": {str(m): run(m, 5, robin, alpha) for m in (4, 8, 12, 16, 20, 24, 28, 32)},
            "p_refinement_m4": {str(q): run(4, q + 1, robin, alpha) for q in (4, 6, 8, 10, 12, 14)},
        }
    return res


def main():
    faulthandler.enable()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="form timed as the headline step (the other form is reported beside it)")
    ap.add_argument("--batch", type=int, default=32, help="right-hand sides of the batched measurement")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the 64x64, n=12 batched measurement")
    ap.add_argument("--no-c4", action="store_true", help="skip the 32x32, n=10 differentiation measurement")
    ap.add_argument("--cpu-solves", type=int, default=2)
    ap.add_argument("--no-paper-study", action="store_true", help="skip the paper's iteration-count study")
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the headline form (e.g. for kernel traces of the solve)")
    ap.add_argument("--large-single-only", action="store_true",
                    help="time only the large stretched grid's one-column FP64 solve (e.g. for kernel traces)")
    ap.add_argument("--large-batched-only", action="store_true",
                    help="time only the large stretched grid's 8-column solve in --precision (e.g. for kernel "
                         "traces)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only a plain 64 MiB device copy, 20 times: the reference kernel that scales the "
                         "hardware byte counters")
    ap.add_argument("--block", action="store_true",
                    help="with --large-batched-only: block GMRES over the 8 columns")
    ap.add_argument("--roofline-only", action="store_true",
                    help="time only the metric kernel (no solves), e.g. for hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; sharding over several GPUs is "
                                   "not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1601_03432_amd import smpm

    torch.cuda.set_device(0)
    if args.copy_calibration:
        a = torch.randn(8 << 20, dtype=torch.float64, device="cuda")  # 64 MiB
        b = torch.empty_like(a)
        for _ in range(20):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": a.numel() * 8}), flush=True)
        return
    stream = torch.cuda.current_stream()
    w = wl.workload("c2")
    ctx = smpm.Context.from_workload(w)
    x, y = ctx.node_coords()
    params = wl.random_fourier_params(wl.SEED_BASE + 2, 20, 8)
    f_host = wl.eval_fourier(params, x, y, w.Lx, w.Ly)
    f = torch.tensor(f_host, device="cuda").reshape(1, -1)
    w5 = wl.workload("c5")
    ctx5 = None if (args.no_large or args.headline_only) and not (args.roofline_only or args.large_single_only or
                                                                  args.large_batched_only) \
        else c5_context(smpm, w5)
    if args.roofline_only:
        print(json.dumps({"roofline": schur_roofline(ctx5),
                          "roofline_fp32_operators": schur_roofline(ctx5, precision=smpm.MIXED_FP32)}), flush=True)
        return

    def solve_fp64(rhs):
        return ctx.solve(rhs, tol=1e-10, maxit=600)

    def solve_mixed(rhs):
        return ctx.solve(rhs, tol=1e-10, maxit=600, precision=smpm.MIXED_FP32, inner_tol=1e-5, max_refine=30)

    def timed(fn, rhs, steps, warmup):
        info = None
        for _ in range(max(1, warmup)):
            u, info = fn(rhs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            u, info = fn(rhs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return (t1 - t0) / steps, info, u

    if args.large_single_only:
        x5, y5 = ctx5.node_coords()
        F5, G5 = wl.c5_sources("c5", x5, y5, ctx5.boundary_arc(), w5.Lx, w5.Ly)
        f5, g5 = torch.tensor(F5[:1], device="cuda"), torch.tensor(G5[:1], device="cuda")
        ctx5.autotune(1)
        sec, info, _ = timed(lambda r: ctx5.solve(r, g5, tol=1e-10, maxit=600), f5, args.steps, args.warmup)
        print(json.dumps({"form": "fp64, large stretched grid, one column", "solves_per_s": 1.0 / sec,
                          "ms_per_step": sec * 1e3, "iterations": info.iterations,
                          "true_rel_residual": info.rel_residual}), flush=True)
        return
    if args.large_batched_only:
        x5, y5 = ctx5.node_coords()
        F5, G5 = wl.c5_sources("c5", x5, y5, ctx5.boundary_arc(), w5.Lx, w5.Ly)
        F5, G5 = torch.tensor(F5, device="cuda"), torch.tensor(G5, device="cuda")
        ctx5.autotune(8)
        prec = smpm.FP64 if args.precision == "fp64" else smpm.MIXED_FP32
        sec, info, _ = timed(lambda r: ctx5.solve(r, G5, tol=1e-10, maxit=200 if args.block else 600,
                                                  precision=prec, inner_tol=1e-5, max_refine=30, block=args.block),
                             F5, args.steps, args.warmup)
        form = args.precision + (" block GMRES" if args.block else " batched") + ", large stretched grid, 8 columns"
        print(json.dumps({"form": form, "solves_per_s": 8 / sec,
                          "ms_per_step": sec * 1e3, "iterations": info.iterations,
                          "refinements": info.refinements, "true_rel_residual": info.rel_residual}), flush=True)
        return
    if args.headline_only:
        fn = solve_fp64 if args.precision == "fp64" else solve_mixed
        sec, info, _ = timed(fn, f, args.steps, args.warmup)
        print(json.dumps({"form": args.precision, "solves_per_s": 1.0 / sec, "ms_per_step": sec * 1e3,
                          "iterations": info.iterations, "true_rel_residual": info.rel_residual}), flush=True)
        return
    # launch shapes chosen by the library's autotuner for one column and for the batch
    tuned = {"1": ctx.autotune(1), str(args.batch): ctx.autotune(args.batch)}
    # the headline form is timed as the benchmark step; the other form beside it
    forms = {"fp64": solve_fp64, "mixed": solve_mixed}
    other = "mixed" if args.precision == "fp64" else "fp64"
    sec, info, u_main = timed(forms[args.precision], f, args.steps, args.warmup)
    ms_per_step = sec * 1e3
    solves_per_s = 1.0 / sec
    sec_o, info_o, u_o = timed(forms[other], f, max(3, args.steps // 2), 1)
    u64 = u_main if args.precision == "fp64" else u_o
    umx = u_o if args.precision == "fp64" else u_main
    mixed_err = float(torch.linalg.norm(umx - u64) / torch.linalg.norm(u64))
    # batched: `batch` right-hand sides (seeded random-Fourier sources) in one call, both forms
    fb = []
    for i in range(args.batch):
        pb = wl.random_fourier_params(wl.SEED_BASE + 200 + i, 20, 8)
        fb.append(wl.eval_fourier(pb, x, y, w.Lx, w.Ly))
    fb = torch.tensor(np.stack(fb), device="cuda")
    secb64, infob64, _ = timed(solve_fp64, fb, 3, 1)
    secbmx, infobmx, _ = timed(solve_mixed, fb, 3, 1)


    out = {
        "metric": "solves/s to 1e-10 rel. residual (FP64 vs mixed-prec); Schur-matvec HBM GB/s",
        "value": solves_per_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": "c2: 16x16 elements, n=16, [0,2]^2, r=65536, k=15360, random-Fourier source "
                               "(20 modes, k<=8, seed 160103434), g=0, FP64, tol 1e-10",
                   "form": args.precision, "gmres_iterations": info.iterations,
                   "refinements": info.refinements, "true_rel_residual": info.rel_residual,
                   "penalty": smpm.DEFAULT_PENALTY, "parallelism": "single GPU"},
        "forms": {
            args.precision: {"solves_per_s": solves_per_s, "iterations": info.iterations,
                             "refinements": info.refinements, "true_rel_residual": info.rel_residual},
            other: {"solves_per_s": 1.0 / sec_o, "iterations": info_o.iterations,
                    "refinements": info_o.refinements, "true_rel_residual": info_o.rel_residual},
            "mixed_vs_fp64_rel_l2": mixed_err,
            f"batched{args.batch}_fp64": {"solves_per_s": args.batch / secb64, "ms_per_call": secb64 * 1e3,
                                          "iterations_max": infob64.iterations,
                                          "true_rel_residual_max": infob64.rel_residual},
            f"batched{args.batch}_mixed": {"solves_per_s": args.batch / secbmx, "ms_per_call": secbmx * 1e3,
                                           "iterations_max": infobmx.iterations,
                                           "refinements": infobmx.refinements,
                                           "true_rel_residual_max": infobmx.rel_residual},
            "autotuned": tuned,
        },
    }
    # the Schur apply on the c2 grid itself (one column, warm): latency-bound
    v = torch.randn(1, ctx.k, dtype=torch.float64, device="cuda")
    sv = torch.empty_like(v)
    c2_us = graph_time_us(lambda: ctx.schur_apply_into(v, sv), 100)
    c2_bytes = 2 * ctx.k * 8 + ctx.stats()["schur_operator_bytes"]
    out["schur_c2"] = {"columns": 1, "avg_launch_us": c2_us, "alg_bytes_per_launch": c2_bytes,
                       "GB_s": c2_bytes / (c2_us * 1e-6) / 1e9,
                       "note": "385 KB per launch: bound by launch and wave latency, not HBM"}

    if not args.no_c3:
        # batched workload: 64x64 elements, n = 12, 32 advected sources; plain FP64 one
        # right-hand side at a time vs FP64 and mixed FP32 batched, all to 1e-10
        w3 = wl.workload("c3")
        c3 = smpm.Context.from_workload(w3)
        x3, y3 = c3.node_coords()
        F3 = torch.tensor(wl.advected_sources(wl.SEED_BASE + 3, x3, y3, count=w3.nrhs), device="cuda")

        def s3_fp64(rhs):
            return c3.solve(rhs, tol=1e-10, maxit=600)

        def s3_mixed(rhs, prec=smpm.MIXED_FP32):
            return c3.solve(rhs, tol=1e-10, maxit=600, precision=prec, inner_tol=1e-5, max_refine=30)

        tuned3 = {"1": c3.autotune(1), str(w3.nrhs): c3.autotune(w3.nrhs)}
        t1, i1, _ = timed(s3_fp64, F3[:1].contiguous(), 5, 1)
        tb, ib, u3b = timed(s3_fp64, F3, 3, 1)
        tm, im, _ = timed(s3_mixed, F3, 3, 1)
        tbf, ibf, _ = timed(lambda r: s3_mixed(r, smpm.MIXED_BF16), F3, 3, 1)
        # block GMRES: all 32 columns in one block Krylov space (FP64)
        tbk, ibk, u3k = timed(lambda r: c3.solve(r, tol=1e-10, maxit=200, block=True), F3, 2, 1)
        tbm, ibm, _ = timed(lambda r: c3.solve(r, tol=1e-10, maxit=200, block=True, precision=smpm.MIXED_FP32,
                                               inner_tol=1e-5, max_refine=30), F3, 2, 1)
        blk_diff = float(max(torch.linalg.norm(u3k[c] - u3b[c]) / torch.linalg.norm(u3b[c]) for c in range(w3.nrhs)))
        out["batched_c3"] = {
            "workload": "c3: 64x64 elements, n=12, [0,1]^2, r=589824, k=193536, d=8064 (substructured coarse "
                        "solve), 32 advected random-Fourier sources + noise (std 1e-3), tol 1e-10",
            "fp64_single_solves_per_s": 1.0 / t1, "fp64_single_iterations": i1.iterations,
            "fp64_batched32_solves_per_s": w3.nrhs / tb, "fp64_batched32_iterations_max": ib.iterations,
            "fp64_batched32_true_rel_residual_max": ib.rel_residual,
            "mixed_fp32_batched32_solves_per_s": w3.nrhs / tm, "mixed_batched32_iterations": im.iterations,
            "mixed_batched32_refinements": im.refinements, "mixed_batched32_true_rel_residual_max": im.rel_residual,
            "mixed_batched_vs_fp64_single": (w3.nrhs / tm) * t1,
            "mixed_bf16_batched32_solves_per_s": w3.nrhs / tbf, "mixed_bf16_batched32_iterations": ibf.iterations,
            "mixed_bf16_batched32_refinements": ibf.refinements,
            "mixed_bf16_batched32_final_schur_precision": ["fp64", "fp32", "bf16"][ibf.schur_precision],
            "mixed_bf16_batched32_true_rel_residual_max": ibf.rel_residual,
            "fp64_block32_solves_per_s": w3.nrhs / tbk, "fp64_block32_block_steps": ibk.iterations,
            "fp64_block32_refinements": ibk.refinements, "fp64_block32_true_rel_residual_max": ibk.rel_residual,
            "fp64_block32_vs_batched32_rel_l2_max": blk_diff,
            "mixed_fp32_block32_solves_per_s": w3.nrhs / tbm, "mixed_block32_block_steps": ibm.iterations,
            "mixed_block32_refinements": ibm.refinements, "mixed_block32_true_rel_residual_max": ibm.rel_residual,
            "autotuned": tuned3,
        }
        del c3, F3, u3b, u3k

    if not args.no_c4:
        # differentiation workload: 32x32 elements, n = 10, FP64; loss |u(f, g) - u_t|^2,
        # gradient by the differentiable solve (forward solve + adjoint solve), checked by
        # central differences along 50 unit directions (one 100-column batched solve)
        w4 = wl.workload("c4")
        c4 = smpm.Context.from_workload(w4)
        x4, y4 = c4.node_coords()
        f4 = torch.tensor(wl.eval_fourier(wl.random_fourier_params(wl.SEED_BASE + 40, 20, 8), x4, y4, 1.0, 1.0),
                          device="cuda")
        g4 = torch.tensor(wl.eval_edge(wl.random_edge_params(wl.SEED_BASE + 41), *c4.boundary_arc(), 1.0, 1.0),
                          device="cuda")
        ut4 = torch.tensor(wl.eval_fourier(wl.random_fourier_params(wl.SEED_BASE + 42, 20, 8), x4, y4, 1.0, 1.0),
                           device="cuda")

        def grad4(tol):
            ft, gt = f4.clone().requires_grad_(True), g4.clone().requires_grad_(True)
            u = smpm.solve_differentiable(c4, ft, gt, tol=tol, maxit=800)
            ((u - ut4) ** 2).sum().backward()
            return ft.grad, gt.grad

        for _ in range(2):
            grad4(1e-10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 10
        for _ in range(reps):
            dfg = grad4(1e-10)
        torch.cuda.synchronize()
        tg = (time.perf_counter() - t0) / reps
        tf4, i4, _ = timed(lambda r: c4.solve(r, g4.reshape(1, -1), tol=1e-10, maxit=800), f4.reshape(1, -1), 10, 2)
        ta4, ia4, _ = timed(lambda r: c4.solve(r, tol=1e-10, maxit=800, transpose=True), ut4.reshape(1, -1), 10, 2)
        gf, gg = grad4(1e-12)
        nd, h = 50, 1e-6
        Df = torch.tensor(wl.random_directions(wl.SEED_BASE + 43, nd, c4.r), device="cuda")
        Dg = torch.tensor(wl.random_directions(wl.SEED_BASE + 44, nd, c4.nbdry), device="cuda")
        ad = (Df * gf).sum(dim=1) + (Dg * gg).sum(dim=1)
        Fp = torch.cat([f4 + h * Df, f4 - h * Df]).contiguous()
        Gp = torch.cat([g4 + h * Dg, g4 - h * Dg]).contiguous()
        tfd, ifd, U = timed(lambda r: c4.solve(r, Gp, tol=1e-12, maxit=800), Fp, 1, 1)
        Lp = ((U - ut4) ** 2).sum(dim=1)
        fd = (Lp[:nd] - Lp[nd:]) / (2 * h)
        out["differentiation_c4"] = {
            "workload": "c4: 32x32 elements, n=10, [0,1]^2, r=%d, FP64; loss |u(f,g) - u_t|^2 with random-Fourier "
                        "f (seed 160103472), edge data g (160103473), target u_t (160103474)" % c4.r,
            "gradients_per_s": 1.0 / tg, "ms_per_gradient": tg * 1e3,
            "forward_solves_per_s": 1.0 / tf4, "forward_iterations": i4.iterations,
            "adjoint_solves_per_s": 1.0 / ta4, "adjoint_iterations": ia4.iterations,
            "fd_check": {"directions": nd, "h": h, "tol": 1e-12,
                         "max_abs_fd_minus_ad_over_max_abs_ad": float((fd - ad).abs().max() / ad.abs().max()),
                         "batched100_solves_per_s": 2 * nd / tfd, "batched100_iterations_max": ifd.iterations},
        }
        del c4, U, Fp, Gp

    if not args.no_large:
        out["roofline"] = schur_roofline(ctx5)
        out["roofline_fp32_operators"] = schur_roofline(ctx5, precision=smpm.MIXED_FP32)
        us1, _ = rotated_schur_us(ctx5, 1)
        b1 = 2 * ctx5.k * 8 + ctx5.stats()["schur_operator_bytes"]
        out["schur_c5_1col"] = {"avg_launch_us": us1, "GB_s": b1 / (us1 * 1e-6) / 1e9,
                                "frac_of_8TBs": b1 / (us1 * 1e-6) / 1e9 / HBM_PEAK_GBS}
        # the large uneven workload: 8 right-hand sides with nonzero Neumann data
        x5, y5 = ctx5.node_coords()
        F5, G5 = wl.c5_sources("c5", x5, y5, ctx5.boundary_arc(), w5.Lx, w5.Ly)
        F5, G5 = torch.tensor(F5, device="cuda"), torch.tensor(G5, device="cuda")
        tuned5 = {"1": ctx5.autotune(1), "8": ctx5.autotune(8)}

        def s5(rhs, g, prec):
            return ctx5.solve(rhs, g, tol=1e-10, maxit=600, precision=prec, inner_tol=1e-5, max_refine=30)

        t51, i51, _ = timed(lambda r: s5(r, G5[:1].contiguous(), smpm.FP64), F5[:1].contiguous(), 2, 1)
        t5b, i5b, u5b = timed(lambda r: s5(r, G5, smpm.FP64), F5, 2, 1)
        t5m, i5m, u5m = timed(lambda r: s5(r, G5, smpm.MIXED_FP32), F5, 2, 1)
        t5h, i5h, _ = timed(lambda r: s5(r, G5, smpm.MIXED_BF16), F5, 1, 1)
        t5k, i5k, u5k = timed(lambda r: ctx5.solve(r, G5, tol=1e-10, maxit=200, block=True), F5, 1, 1)
        t5km, i5km, u5km = timed(lambda r: ctx5.solve(r, G5, tol=1e-10, maxit=200, block=True,
                                                      precision=smpm.MIXED_FP32, inner_tol=1e-5, max_refine=30),
                                 F5, 2, 1)
        out["c5"] = {
            "workload": "c5: 128x128 elements, n=16, x-stretched (ratio 1.05, aspect <= 8) on [0,1]x[0,%.4f], "
                        "r=%d, k=%d, d=%d (substructured coarse solve), 8 random-Fourier sources + nonzero "
                        "Neumann data, tol 1e-10" % (w5.Ly, ctx5.r, ctx5.k, ctx5.d),
            "fp64_single_solves_per_s": 1.0 / t51, "fp64_single_iterations": i51.iterations,
            "fp64_batched8_solves_per_s": 8 / t5b, "fp64_batched8_iterations_max": i5b.iterations,
            "fp64_batched8_true_rel_residual_max": i5b.rel_residual,
            "mixed_fp32_batched8_solves_per_s": 8 / t5m, "mixed_batched8_iterations": i5m.iterations,
            "mixed_batched8_refinements": i5m.refinements,
            "mixed_batched8_final_schur_precision": ["fp64", "fp32", "bf16"][i5m.schur_precision],
            "mixed_batched8_true_rel_residual_max": i5m.rel_residual,
            "mixed_vs_fp64_rel_l2_max": float(max(torch.linalg.norm(u5m[c] - u5b[c]) / torch.linalg.norm(u5b[c])
                                                  for c in range(8))),
            "mixed_batched_vs_fp64_single": (8 / t5m) * t51,
            "mixed_bf16_batched8_solves_per_s": 8 / t5h, "mixed_bf16_batched8_iterations": i5h.iterations,
            "mixed_bf16_batched8_refinements": i5h.refinements,
            "mixed_bf16_batched8_true_rel_residual_max": i5h.rel_residual,
            "fp64_block8_solves_per_s": 8 / t5k, "fp64_block8_block_steps": i5k.iterations,
            "fp64_block8_refinements": i5k.refinements, "fp64_block8_true_rel_residual_max": i5k.rel_residual,
            "fp64_block8_vs_batched8_rel_l2_max": float(max(torch.linalg.norm(u5k[c] - u5b[c]) /
                                                            torch.linalg.norm(u5b[c]) for c in range(8))),
            "mixed_fp32_block8_solves_per_s": 8 / t5km, "mixed_block8_block_steps": i5km.iterations,
            "mixed_block8_refinements": i5km.refinements,
            "mixed_block8_true_rel_residual_max": i5km.rel_residual,
            "mixed_block8_vs_fp64_batched8_rel_l2_max": float(max(torch.linalg.norm(u5km[c] - u5b[c]) /
                                                                  torch.linalg.norm(u5b[c]) for c in range(8))),
            "mixed_block_vs_fp64_single": (8 / t5km) * t51,
            "autotuned": tuned5,
        }
        del ctx5, F5, G5, u5b, u5m, u5k, u5km
        # the three side grids, 8 right-hand sides each, as one concurrent group
        side = []
        for name in wl.C5_SIDE_GRIDS:
            ws = wl.workload(name)
            cs = smpm.Context.from_workload(ws)
            xs, ys = cs.node_coords()
            Fs, Gs = wl.c5_sources(name, xs, ys, cs.boundary_arc(), ws.Lx, ws.Ly)
            cs.autotune(8)
            side.append((cs, torch.tensor(Fs, device="cuda"), torch.tensor(Gs, device="cuda")))
        gkw = dict(tol=1e-10, maxit=600, precision=smpm.MIXED_FP32, inner_tol=1e-5, max_refine=30)

        def group(_):
            res = smpm.solve_group([c for c, _, _ in side], [f for _, f, _ in side], [g for _, _, g in side], **gkw)
            return res[0][0], res[0][1]

        def sequential(_):
            for c, f, g in side:
                u, info = c.solve(f, g, **gkw)
            return u, info

        tg, _, _ = timed(group, None, 3, 1)
        ts, _, _ = timed(sequential, None, 3, 1)
        res = smpm.solve_group([c for c, _, _ in side], [f for _, f, _ in side], [g for _, _, g in side], **gkw)
        out["c5_side_grids_group"] = {
            "grids": "16x16 n=8, 32x32 n=12, 48x48 n=10 on [0,1]^2, 8 right-hand sides each, mixed FP32, tol 1e-10",
            "group_solves_per_s": 24 / tg, "sequential_solves_per_s": 24 / ts,
            "iterations": [i.iterations for _, i in res], "refinements": [i.refinements for _, i in res],
            "true_rel_residual_max": max(i.rel_residual for _, i in res),
        }
        del side, res

    if not args.no_paper_study:
        out["paper_study"] = paper_study(smpm, torch)

    if not args.no_cpu_baseline:
        from oracle import smpm_oracle as O
        g = O.Grid(w.n, w.x_breaks, w.y_breaks)
        m = O.Method(g)
        xo, yo = g.node_coords()
        fo = wl.eval_fourier(params, xo, yo, w.Lx, w.Ly)
        import threadpoolctl
        t0 = time.perf_counter()
        for _ in range(args.cpu_solves):
            m.solve(fo, variant=3, tol=1e-10, maxit=600)
        t1 = time.perf_counter()
        # the threads the oracle's numeric libraries actually had (their pools' sizes)
        pools = threadpoolctl.threadpool_info()
        cores = max([p.get("num_threads", 1) for p in pools] + [1])
        with threadpoolctl.threadpool_limits(limits=1):
            s0 = time.perf_counter()
            m.solve(fo, variant=3, tol=1e-10, maxit=600)
            s1 = time.perf_counter()
        model = ""
        try:
            with open("/proc/cpuinfo") as fh:
                model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
        except OSError:
            pass
        out["cpu_baseline"] = {"value": args.cpu_solves / (t1 - t0), "unit": "solves/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{args.cpu_solves} oracle Algorithm-3 solves of the same c2 problem "
                                         f"(numpy/scipy FP64, setup excluded)",
                               "one_core": {"value": 1.0 / (s1 - s0), "cores": 1,
                                            "sample": "1 solve of the same problem, numeric libraries on one thread"},
                               "cpu_model": model}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
