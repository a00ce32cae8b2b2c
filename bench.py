#!/usr/bin/env python3
"""Benchmark of the TC2 + response solve on one MI355X.

One step = one complete solve (``tc2_run``): Gershgorin bounds, initial
matrices, every TC2 / TC2-CPSCF update (symbolic pattern, MFMA block
products, drop, reductions, branch) until the stopping rule, with the inputs
already resident in HBM (uploaded by ``tc2_setup`` before timing).

Prints one JSON line.  ``value`` is useful GFLOP/s of the chosen precision
variant (2 b^3 per block triple landing on a kept output block, times the
1 + 2D block products of an update); ``ms_per_step`` is seconds per solve in
ms.  The plain FP64 path is run too and the chosen variant is gated against
it (max |dX1| < 1e-6, relative |d alpha| < 1e-6).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
HBM_PEAK_GBS = 8000.0


SHAPES = ((8, 8), (4, 8), (8, 4), (4, 4))   # sub-tile shape id -> (rows, columns)


def kernel_name(kernel: str, kind: int, D: int, shape: int) -> str:
    """Template instance of the numeric kernel of one kind (FP64, FP32, BF16
    operands, FP32 with FP64 sums), as rocprofv3 names it."""
    T = "double" if kind == 0 else "float"
    if kernel == "block":
        return f"k_numeric<{T}, {D}>"
    sp, tq = SHAPES[max(shape, 0)]
    return (f"k_tile_numeric<{T}, {D}, {sp}, {tq}, {'true' if kind == 2 else 'false'}, "
            f"{'true' if kind == 3 else 'false'}>")

KERNEL_SOURCES = ("paper_2009_03551_amd/csrc/tc2_tile.hip", "paper_2009_03551_amd/csrc/tc2_device.h",
                  "paper_2009_03551_amd/csrc/tc2_internal.h", "paper_2009_03551_amd/csrc/tc2_kernels.hip")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, tag: str):
    """HBM bytes per launch of ``kernel`` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by the copy-kernel calibration), or None
    when there is none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{tag}_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(mib: int, reps: int) -> int:
    """Plain device copy of a known size, the reference for the HBM byte
    counters: each launch reads and writes ``mib`` MiB."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_calibration_bytes_read": n * 4, "bytes_written": n * 4,
                      "launches": reps, "GBps_read_plus_write": round(2 * n * 4 / dt / 1e9, 1)}),
          flush=True)
    return 0


def cpu_baseline(sysm, gpu_iters: int, useful_flops: float, iters_sample: int = 1) -> dict:
    """The FP64 oracle on the host cores: ``iters_sample`` full-size TC2 updates
    (dense products, block drop, band energies) timed, scaled to a whole solve
    by the GPU's update count."""
    import numpy as np
    from oracle import tc2_oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()
                       if p.get("user_api") == "blas"] or [os.cpu_count() or 1])
    except Exception:
        threads = os.cpu_count() or 1
    H = O.bsr_to_dense(sysm.H.nb, sysm.H.b, sysm.H.row_ptr, sysm.H.col, sysm.H.val)
    H1s = [O.bsr_to_dense(h.nb, h.b, h.row_ptr, h.col, h.val) for h in sysm.H1]
    emin, emax = O.gershgorin(H)
    X0, X1s = O.tc2_init(H, H1s, emin, emax)
    b = sysm.H.b
    t0 = time.perf_counter()
    for _ in range(iters_sample):
        sq = np.trace(X0) >= sysm.n_occ
        X0, X1s = O.tc2_step(X0, X1s, sq)
        X0 = O.block_drop(X0, b, sysm.eps)
        X1s = [O.block_drop(X, b, sysm.eps) for X in X1s]
        O.band_energies(X0, X1s, H, H1s)
    dt = (time.perf_counter() - t0) / iters_sample
    solve_s = dt * gpu_iters
    return {"value": round(useful_flops / solve_s / 1e9, 3), "unit": "GFLOP/s",
            "cores": int(threads), "kind": "oracle",
            "s_per_solve": round(solve_s, 2),
            "sample": f"{iters_sample} dense FP64 oracle update(s) at full size "
                      f"(N={sysm.H.n}), {dt:.1f} s each, scaled by {gpu_iters} updates"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube10")
    # default: the fastest variant that passes the gate on this workload (FP32
    # block products summed in FP64 over the column blocks, 4 leading FP64
    # updates, exact screen, closing FP64 pair)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--kernel", default="tile", choices=["tile", "block"])
    ap.add_argument("--skip", default="bound", choices=["none", "bound"])
    ap.add_argument("--fp64-first", type=int, default=4)
    ap.add_argument("--wide", type=int, default=1, choices=[0, 1],
                    help="FP32 stages: FP64 sums of the per-block FP32 products")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the sub-tile shapes (timed in the warm-up solve)")
    ap.add_argument("--tune-cache", default=None, help="tuned-shape cache file (read and appended)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=1)
    ap.add_argument("--no-reference", action="store_true",
                    help="skip the plain FP64 runs and the gate (profiling the chosen variant alone)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): this build has "
              "no multi-GPU path", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2009_03551_amd import tc2 as T
    from paper_2009_03551_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration, 10)
    stream = torch.cuda.current_stream().cuda_stream

    sysm = W.config_system(args.workload)
    log(f"workload {args.workload}: atoms={sysm.H.nb} b={sysm.H.b} N={sysm.H.n} "
        f"nnzb(H)={sysm.H.nnzb} dirs={len(sysm.H1)} eps={sysm.eps} tol={sysm.tol}")

    def timed(solver):
        for _ in range(args.warmup):
            solver.run(stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [solver.run(stream=stream)[0] for _ in range(args.steps)]
        torch.cuda.synchronize()
        return res, (time.perf_counter() - t0) / args.steps * 1e3

    # plain FP64 path (every candidate block computed): reference for the gate
    # and the speed-up, timed the same way as the chosen variant
    ref = None
    if not args.no_reference:
        tune = dict(tune=args.tune, tune_cache=args.tune_cache) if args.kernel == "tile" else {}
        ref_solver = T.Solver(sysm, precision="fp64", export=True, kernel=args.kernel, **tune)
        ref = ref_solver.run(stream=stream)[0]
        ref_solver.close()
        plain_solver = T.Solver(sysm, precision="fp64", export=False, kernel=args.kernel, **tune)
        _, ref_ms = timed(plain_solver)
        plain_solver.close()
        log(f"plain fp64: {ref.status_name} iters={ref.iters} {ref.branches} "
            f"alpha={ref.alpha} kept={ref.kept_blocks} {ref_ms:.1f} ms/solve")

    chosen = args.precision
    closing = 0 if chosen == "fp64" else 2
    variant = dict(precision=chosen, closing_fp64=closing, kernel=args.kernel, skip=args.skip,
                   fp64_first=args.fp64_first if chosen != "fp64" else 0,
                   wide=bool(args.wide and chosen != "fp64"))
    if args.tune and args.kernel == "tile":
        variant.update(tune=True, tune_cache=args.tune_cache)
    solver = T.Solver(sysm, export=False, profile=True, **variant)
    results, ms_per_step = timed(solver)
    r = results[-1]
    value = r.useful_flops / (ms_per_step * 1e-3) / 1e9
    ms_num = sum(x.ms_numeric for x in results) / len(results)
    launches = results[-1].numeric_launches
    # roofline of the dominant kernel: the numeric kernel kind (FP64, FP32,
    # BF16 operands, FP32 with FP64 sums) that takes most of the numeric time
    nk = len(results)
    ms_kind = [sum(x.ms_numeric_kind[k] for x in results) / nk for k in range(4)]
    dom = max(range(4), key=lambda k: ms_kind[k])
    dom_launches = results[-1].numeric_launches_kind[dom]
    dom_flops = r.useful_flops_kind[dom]
    achieved = dom_flops / (ms_kind[dom] * 1e-3) / 1e12
    peak = PEAK_TFLOPS[("fp64", "fp32", "bf16", "fp32")[dom]]
    kname = kernel_name(args.kernel, dom, len(sysm.H1), r.tile_shape[dom])
    log(f"{chosen}: {ms_per_step:.1f} ms/solve, numeric {ms_num:.1f} ms in {launches} launches, "
        f"symbolic {r.ms_symbolic:.1f} ms, compact {r.ms_compact:.1f} ms, "
        f"useful {r.useful_flops / 1e12:.3f} TF, executed {r.executed_flops / 1e12:.3f} TF")

    # gate of the chosen variant against the plain FP64 path
    gate = None
    if ref is not None:
        g = T.Solver(sysm, export=True, **variant).run(stream=stream)[0]
        dx1 = max(float(np.abs(T.bsr_dense(a) - T.bsr_dense(b)).max())
                  for a, b in zip(g.X1, ref.X1))
        dal = max(abs(x - y) / abs(y) for x, y in zip(g.alpha, ref.alpha))
        gate = {"max_abs_dX1": dx1, "rel_dalpha": dal, "pass": bool(dx1 < 1e-6 and dal < 1e-6),
                "against": "plain FP64 GPU path"}
    traffic = measured_traffic(kname.split("<")[0], args.workload,
                               ("fp64", "fp32", "bf16", "fp32w")[dom])
    out = {
        "metric": "TC2+response s/solve & useful GFLOP/s, chosen vs plain FP64 at max|dX1|<1e-6",
        "value": round(value, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "s_per_solve": round(ms_per_step * 1e-3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[chosen],
        "data": "synthetic",
        "config": {"workload": args.workload, "atoms": sysm.H.nb, "b": sysm.H.b,
                   "N": sysm.H.n, "directions": len(sysm.H1), "eps": sysm.eps,
                   "tol": sysm.tol, "precision": chosen, "closing_fp64": closing,
                   "iters": r.iters, "status": r.status_name, "kernel": args.kernel,
                   "skip": args.skip, "fp64_first": variant["fp64_first"],
                   "wide_accumulate": variant["wide"], "tuned": bool(args.tune),
                   "tile_shape": r.tile_shape,
                   "screened_blocks": r.screened_blocks},
        "plain_fp64": None if ref is None else {
            "s_per_solve": round(ref_ms * 1e-3, 4),
            "useful_gflops": round(ref.useful_flops / (ref_ms * 1e-3) / 1e9, 3)},
        "speedup_vs_plain_fp64": None if ref is None else round(ref_ms / ms_per_step, 3),
        "gate": gate,
        "useful_tflop_per_solve": round(r.useful_flops / 1e12, 4),
        "executed_tflop_per_solve": round(r.executed_flops / 1e12, 4),
        "roofline": {"bound": "mfma",
                     "kernel": kname, "achieved": round(achieved, 3),
                     "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                     "traffic": traffic,
                     "launches_per_solve": dom_launches,
                     "avg_launch_ms": round(ms_kind[dom] / max(dom_launches, 1), 4),
                     "useful_tflop_per_solve": round(dom_flops / 1e12, 4),
                     "all_numeric": {"ms_per_solve": round(ms_num, 3), "launches": launches,
                                     "ms_per_kind": [round(x, 3) for x in ms_kind]}},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(sysm, r.iters, r.useful_flops, args.cpu_sample_iters)
    print(json.dumps(out), flush=True)
    solver.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
