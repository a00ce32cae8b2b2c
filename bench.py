#!/usr/bin/env python3
"""Benchmark of the TC2 + response solve on one MI355X.

One step = one TC2 / TC2-CPSCF update (symbolic pattern, MFMA block
products, drop, reductions and the branch of the next update) of the chosen
precision variant, on the workload's systems with the inputs already
resident in HBM (uploaded by ``tc2_setup`` before timing).  Steps run back to
back through ``tc2_advance``: a solve that finishes within the timed steps
is followed by the next one from H, so K steps are K updates of the solve
sequence.  Batch workloads (many systems in memory-sized units) take one
step = one solve of every unit.

Prints one JSON line.  ``value`` is useful GFLOP/s over the timed steps (the
exact count of useful block products, 2 b^3 each: X0 X0 on X0's stored
blocks and kept outputs, X0 X1_d + X1_d X0 on their own operands and X1_d's
kept outputs); ``ms_per_step`` is the time per update; ``s_per_solve`` is
the device time of a complete solve of the same variant.  The plain FP64
path is timed once and the chosen variant is gated against it on the device
(max |dX1| < 1e-6, relative |d alpha| < 1e-6).
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


def kernel_name(kernel: str, kind: int, D: int, shape: int, b: int, split: bool = False) -> str:
    """Template instance of the numeric kernel of one kind (FP64, FP32, BF16
    operands, FP32 with FP64 sums; with `split`, the FP64-sum kind runs the
    three-way bfloat16 split), as rocprofv3 names it."""
    T = "double" if kind == 0 else "float"
    if kernel == "block":
        return f"k_numeric<{T}, {D}>"
    sp, tq = SHAPES[max(shape, 0)]
    bf = kind == 2 or (split and kind == 3)
    full_k = b > 12 and not bf
    # waves per sub-tile column: four for the 4 x 4 sub-tile with D >= 2 (FP64,
    # and the kinds with FP64 sums), two for the 8 x 8 sub-tile with D <= 1
    # (FP64, FP32 with FP64 sums)
    ws = 1
    if kind in (0, 3) and D >= 2 and (sp, tq) == (4, 4):
        ws = 4
    elif (kind == 0 or (kind == 3 and not split)) and D <= 1 and (sp, tq) == (8, 8):
        ws = 2
    tf = lambda v: "true" if v else "false"
    return (f"k_tile_numeric<{T}, {D}, {sp}, {tq}, {tf(bf)}, {tf(kind == 3)}, {tf(full_k)}, "
            f"{ws}>")

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


def peak_probe() -> int:
    """Attainable peaks on this device, beside the published ones: dense FP32
    and FP64 GEMMs of 8192^3 through the vendor BLAS (torch.matmul), and a
    4 GiB device copy.  One JSON line."""
    import torch
    out = {"mode": "peak_probe", "device": torch.cuda.get_device_name(0)}
    torch.backends.cuda.matmul.allow_tf32 = False
    for name, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        n = 8192
        a = torch.randn(n, n, dtype=dt, device="cuda")
        b = torch.randn(n, n, dtype=dt, device="cuda")
        for _ in range(3):
            torch.matmul(a, b)
        torch.cuda.synchronize()
        reps = 10
        t0 = time.perf_counter()
        for _ in range(reps):
            torch.matmul(a, b)
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t0) / reps
        out[f"gemm_{name}_tflops"] = round(2.0 * n ** 3 / dt_s / 1e12, 1)
        del a, b
    n = (4 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt_s = (time.perf_counter() - t0) / reps
    out["copy_GBps_read_plus_write"] = round(2 * n * 4 / dt_s / 1e9, 1)
    print(json.dumps(out), flush=True)
    return 0


def measured_peaks():
    """Attainable peaks from the committed probe summary, or None."""
    path = os.path.join(ROOT, "profiles", "peaks_measured.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                try:
                    vals[k.strip()] = float(v.strip().strip("`"))
                except ValueError:
                    pass
    return vals or None


def cpu_baseline_dense(sysm, gpu_iters: int, useful_flops: float, iters_sample: int = 1) -> dict:
    """The dense FP64 oracle on the host cores: ``iters_sample`` full-size TC2
    updates (dense products, block drop, band energies) timed, scaled to a
    whole solve by the GPU's update count (systems with N <= 20000)."""
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


def cpu_baseline_bsr(name: str, sysm, useful_flops: float) -> dict:
    """The block-list FP64 oracle on the host (plain numpy, one thread): the
    first three updates of the workload (every row of X_1, the rows of X_2 that
    sampled rows of X_3 need, three sampled rows of X_3), timed.  Its rate of
    block products (each 2 b^3 flops, counting every product it forms) turns
    the useful flops of one solve into an extrapolated solve time."""
    from oracle import bsr_oracle as B
    nb = sysm.H.nb
    rows = sorted({0, nb // 2 + 7 if nb > 20 else nb // 2, nb - 1})
    B.PRODUCTS[0] = 0
    t0 = time.perf_counter()
    B.leading_updates(sysm.H, sysm.H1, sysm.n_occ, sysm.eps, rows, 3)
    dt = time.perf_counter() - t0
    prods = B.PRODUCTS[0]
    rate = prods * 2.0 * sysm.H.b ** 3 / dt
    return {"value": round(rate / 1e9, 3), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "s_per_solve": round(useful_flops / rate, 1), "extrapolated": True,
            "sample": f"block-list FP64 oracle (numpy, one thread), first 3 updates of {name} "
                      f"(all rows of X1, {len(rows)} sampled rows of X3 and the rows of X2 they "
                      f"need): {prods} block products in {dt:.1f} s; a solve of "
                      f"{useful_flops / 1e12:.1f} useful TFLOP extrapolated at that rate"}


def crossover(args) -> int:
    """Seconds per solve of the linear-scaling path (plain FP64, and the default
    variant) and of the dense O(N^3) path over a series of system sizes, with
    the polarizability traces of both (the crossover experiment of Sec. 4)."""
    import torch
    from paper_2009_03551_amd import tc2 as T
    from paper_2009_03551_amd import workloads as W

    stream = torch.cuda.current_stream().cuda_stream
    if args.crossover == "cube":
        sizes = [int(x) for x in (args.sizes or "4,5,6,7,8,10,12").split(",")]
        make = lambda n: W.config_system("cube10", L=n)
    else:
        sizes = [int(x) for x in (args.sizes or "256,512,1024,2048").split(",")]
        make = lambda n: W.config_system("chain64", n=n)
    variants = {"tc2_fp64": dict(precision="fp64", skip="bound", graph=True),
                "tc2_default": dict(precision="fp32", wide=True, fp64_first=args.fp64_first,
                                    closing_fp64=2, skip="bound", graph=True)}
    for n in sizes:
        s = make(n)
        line = {"mode": "crossover", "series": args.crossover, "size": n, "atoms": s.H.nb,
                "N": s.H.n, "b": s.H.b, "dirs": len(s.H1), "eps": s.eps}
        for name, kw in variants.items():
            solver = T.Solver(s, export=False, **kw)
            for _ in range(args.warmup):
                solver.run(stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                r = solver.run(stream=stream)[0]
            torch.cuda.synchronize()
            line[name + "_s"] = (time.perf_counter() - t0) / args.steps
            line[name + "_alpha"] = r.alpha[0] if r.alpha else None
            solver.close()
        if s.H.n > T.DENSE_MAX_N or args.no_dense:
            line["dense_s"] = None  # beyond the dense path's size limit, or not asked for
            print(json.dumps(line), flush=True)
            continue
        T.dense_response(s, stream=stream)  # warm-up (library kernels, workspace)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d = T.dense_response(s, stream=stream)
        torch.cuda.synchronize()
        line.update(dense_s=time.perf_counter() - t0, dense_device_s=d.seconds,
                    dense_ms_eigh=d.ms_eigh, dense_ms_p0=d.ms_p0, dense_ms_p1=d.ms_p1,
                    dense_p1_tflops=(d.flops_p1 / (d.ms_p1 * 1e-3) / 1e12) if d.ms_p1 > 0 else None,
                    dense_alpha=d.alpha[0] if d.alpha else None, gap=d.gap)
        if d.alpha:
            line["rel_dalpha_fp64"] = abs(line["tc2_fp64_alpha"] - d.alpha[0]) / abs(d.alpha[0])
        print(json.dumps(line), flush=True)
    return 0


def decision_latency(args) -> int:
    """Seconds per solve and per update of small, latency-bound FP64 solves
    with the branch and stopping decisions taken on the host after every
    update (graph = 1) and on the device (device_loop = k: the host replays
    k update graphs between two polls of a flag word).  One JSON line per
    workload, with whether every variant took the same branches and reached
    bit-identical traces."""
    import torch
    from paper_2009_03551_amd import tc2 as T
    from paper_2009_03551_amd import workloads as W

    stream = torch.cuda.current_stream().cuda_stream
    cases = {"chain64": lambda: W.config_system("chain64"),
             "chain256": lambda: W.config_system("chain64", n=256),
             "cube4": lambda: W.config_system("cube10", L=4),
             "batch8_chain64": lambda: [W.config_system("chain64", seed=100 + k) for k in range(8)]}
    if args.workload in cases:
        cases = {args.workload: cases[args.workload]}
    ks = [int(x) for x in (args.sizes or "1,4,16").split(",")]
    variants = {"host": {}}
    variants.update({f"device_k{k}": dict(device_loop=k) for k in ks})
    for name, make in cases.items():
        sysm = make()
        first = sysm[0] if isinstance(sysm, list) else sysm
        line = {"mode": "decision_latency", "workload": name, "atoms": first.H.nb, "b": first.H.b,
                "dirs": len(first.H1), "systems": len(sysm) if isinstance(sysm, list) else 1}
        outs = {}
        for vname, kw in variants.items():
            solver = T.Solver(sysm, export=False, graph=True, skip="bound", tune=args.tune,
                              tune_cache=args.tune_cache, **kw)
            for _ in range(args.warmup):
                solver.run(stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                res = solver.run(stream=stream)
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / args.steps
            solver.close()
            upd = max(r.iters for r in res)
            outs[vname] = [(r.branches, r.status, r.alpha, r.e0) for r in res]
            line[vname] = {"s_per_solve": sec, "ms_per_update": 1e3 * sec / max(upd, 1),
                           "updates": upd, "device_updates": res[0].device_loop_updates}
        ref = outs["host"]
        line["identical"] = all(o == ref for o in outs.values())
        line["branches"] = ref[0][0]
        print(json.dumps(line), flush=True)
    return 0


def lowdin_pipeline(args) -> int:
    """Seconds of each stage of the non-orthogonal pipeline (Sec. 2.2): S^-1/2
    and the orthogonal forms, the TC2 / TC2-CPSCF solve on them (the default
    variant), and the back-transforms P = S^-1/2 X S^-1/2."""
    import torch
    from paper_2009_03551_amd import tc2 as T
    from paper_2009_03551_amd import workloads as W

    stream = torch.cuda.current_stream().cuda_stream
    s = W.config_system(args.workload)
    S = W.make_overlap(s, amp=0.2)
    eps = s.eps
    disp = args.displacement
    if disp:  # one displacement of the central atom instead of the field directions
        H1d, S1d = W.make_displacement(s, atom=s.H.nb // 2)
        H1s, S1s = [H1d], [S1d]
    else:
        H1s, S1s = s.H1, None
    line = {"mode": "lowdin_displacement" if disp else "lowdin", "workload": args.workload,
            "atoms": s.H.nb, "N": s.H.n, "b": s.H.b, "dirs": len(H1s), "eps": eps,
            "S_blocks": int(S.row_ptr[-1])}

    def orthogonalise():
        if disp:
            return T.lowdin_response(S, s.H, H1s, S1s, eps=eps, tol=1e-9, max_iter=40,
                                     stream=stream)
        return T.lowdin(S, s.H, H1s, eps=eps, tol=1e-9, max_iter=40, stream=stream)
    for _ in range(args.warmup):
        orthogonalise()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = orthogonalise()
    torch.cuda.synchronize()
    line.update(lowdin_s=time.perf_counter() - t0, lowdin_device_s=g.seconds,
                ns_status=g.status, ns_updates=g.iters, ns_resid=g.resid,
                Z_blocks=int(g.Z.row_ptr[-1]), H_orth_blocks=int(g.H.row_ptr[-1]))
    orth = W.System(H=g.H, H1=g.H1, n_occ=s.n_occ, xyz=s.xyz, eps=eps, tol=s.tol)
    solver = T.Solver(orth, precision="fp32", wide=True, fp64_first=args.fp64_first,
                      closing_fp64=2, skip="bound", graph=True)
    for _ in range(args.warmup):
        solver.run(stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = solver.run(stream=stream)[0]
    torch.cuda.synchronize()
    solver.close()
    line.update(tc2_s=time.perf_counter() - t0, tc2_status=r.status_name, tc2_updates=r.iters,
                trace_x1h1=r.alpha)
    t0 = time.perf_counter()
    P0 = T.congruence(g.Z, r.X0, eps=eps, stream=stream)
    if disp:
        P1 = [T.congruence_response(g.Z, z1, r.X0, x, eps=eps, stream=stream)
              for z1, x in zip(g.Z1, r.X1)]
        line["Z1_blocks"] = [int(z.row_ptr[-1]) for z in g.Z1]
    else:
        P1 = [T.congruence(g.Z, x, eps=eps, stream=stream) for x in r.X1]
    torch.cuda.synchronize()
    line.update(back_transform_s=time.perf_counter() - t0, P0_blocks=int(P0.row_ptr[-1]),
                P1_blocks=[int(p.row_ptr[-1]) for p in P1])
    line["total_s"] = line["lowdin_s"] + line["tc2_s"] + line["back_transform_s"]
    print(json.dumps(line), flush=True)
    return 0


def snapshot(solver, D: int, chunk: int = 1 << 20):
    """Rows, columns and the X1_d values of the current iterate of a context,
    exported to host memory in chunks (the reference side of the gate)."""
    import numpy as np
    n = solver.iterate_size()
    b = solver.systems[0].H.b
    rows = np.empty(n, dtype=np.int32)
    cols = np.empty(n, dtype=np.int32)
    vals = [np.empty((n, b, b)) for _ in range(D)]
    for f in range(0, n, chunk):
        c = min(chunk, n - f)
        r, k, _ = solver.export_entries(1, f, c, values=False)
        rows[f:f + c], cols[f:f + c] = r, k
        for d in range(D):
            vals[d][f:f + c] = solver.export_entries(1 + d, f, c)[2]
    return rows, cols, vals


def export_time(solver, D: int, chunk: int = 1 << 20) -> float:
    """Seconds to copy every entry of X0 and of each X1_d of the current
    iterate (rows, columns, b x b values) to host memory, in chunks."""
    n = solver.iterate_size()
    t0 = time.perf_counter()
    for m in range(1 + D):
        for f in range(0, n, chunk):
            solver.export_entries(m, f, min(chunk, n - f))
    return time.perf_counter() - t0


def gate(solver, snap, res, ref_res, name: str, eps: float) -> dict:
    """max |dX1| over the union of the patterns (on the device) and relative
    |d alpha| of the chosen variant's last solve against a reference.  The
    difference is also split into blocks both runs keep and blocks only one
    run keeps (a block whose norm lies near the drop threshold, kept by one
    run and dropped by the other)."""
    rows, cols, vals = snap
    dx1, det = 0.0, None
    for d, v in enumerate(vals):
        x, dd = solver.compare_entries(1 + d, rows, cols, v, detail=True)
        dx1 = max(dx1, x)
        if det is None:
            det = dd
        else:
            for k in ("max_both", "max_given_only", "max_iterate_only", "max_norm_one_side"):
                det[k] = max(det[k], dd[k])
            det["n_given_only"] += dd["n_given_only"]
            det["n_iterate_only"] += dd["n_iterate_only"]
    dal = max([abs(x - y) / abs(y) for g, f in zip(res, ref_res) for x, y in zip(g.alpha, f.alpha)]
              + [0.0])
    out = {"max_abs_dX1": dx1, "rel_dalpha": dal, "pass": bool(dx1 < 1e-6 and dal < 1e-6),
           "against": name}
    if det:
        out["split"] = {"max_abs_dX1_blocks_both_keep": det["max_both"],
                        "blocks_kept_by_reference_only": det["n_given_only"],
                        "blocks_kept_by_chosen_only": det["n_iterate_only"],
                        "max_abs_in_one_side_blocks": max(det["max_given_only"],
                                                          det["max_iterate_only"]),
                        "max_norm_of_one_side_block_over_eps": det["max_norm_one_side"] / eps
                        if eps > 0 else None}
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed steps: TC2 updates (single-system workloads) or solves (batches)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cube30")
    # default: the fastest variant that passes the gate on cube30 (eps 1e-5):
    # FP64 block products with the exact norm-bound screen and update graphs.
    # Reduced-precision variants (--precision fp32 with --wide 1 and
    # --fp64-first 4, or bf16) are faster per product but move X1 by more
    # than 1e-6 at this drop threshold (blocks near eps kept by one run and
    # dropped by the other); each run reports its own gate.
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--kernel", default="tile", choices=["tile", "block"])
    ap.add_argument("--skip", default="bound", choices=["none", "bound", "mlp"],
                    help="mlp: train the skip network first on logged solves of smaller "
                         "cubes (seeds 500+L, same drop threshold), then skip with it")
    ap.add_argument("--mlp-threshold", type=float, default=0.995)
    ap.add_argument("--mlp-cap", type=float, default=0.0,
                    help="the network skips only candidates whose exact bound is below "
                         "cap * eps (0: the library default, 4)")
    ap.add_argument("--mlp-budget", type=float, default=0.0,
                    help="summed bounds of the network's skips per solve, after which the "
                         "solve continues with the exact screen alone (0: no limit)")
    ap.add_argument("--fp64-first", type=int, default=4)
    ap.add_argument("--wide", type=int, default=1, choices=[0, 1],
                    help="FP32 stages: FP64 sums of the per-block FP32 products")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the sub-tile shapes (timed in the warm-up)")
    ap.add_argument("--tune-cache", default=None, help="tuned-shape cache file (read and appended)")
    ap.add_argument("--graph", type=int, default=1, choices=[0, 1],
                    help="run each update as one captured hipGraph with a persistent "
                         "numeric launch (tiled kernel)")
    ap.add_argument("--group-atoms", type=int, default=16000,
                    help="batch workloads: most atoms per context")
    ap.add_argument("--units", default=None,
                    help="batch workloads: comma-separated indices of the units to run "
                         "(default: all)")
    ap.add_argument("--metrics-log", default=None,
                    help="JSONL file of per-update scalars of the chosen variant")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-reference", action="store_true",
                    help="skip the plain FP64 run and the gate (profiling the chosen variant alone)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--peak-probe", action="store_true",
                    help="only measure attainable peaks (FP32 and FP64 GEMMs, a device copy)")
    ap.add_argument("--crossover", choices=["cube", "chain"], default=None,
                    help="only time the linear-scaling path against the dense O(N^3) path "
                         "over a series of sizes (one JSON line per size)")
    ap.add_argument("--lowdin", action="store_true",
                    help="only time the non-orthogonal pipeline on the workload with a synthetic "
                         "overlap: Loewdin orthogonalisation, the TC2 solve of the orthogonal "
                         "forms, and the back-transform of X0 and X1 (one JSON line)")
    ap.add_argument("--displacement", action="store_true",
                    help="with --lowdin: the perturbation is a displacement of the central atom, "
                         "which moves the overlap too (derivative of S^-1/2, three-term "
                         "back-transform)")
    ap.add_argument("--latency", action="store_true",
                    help="only time small FP64 solves with the branch and stopping decisions on "
                         "the host and on the device (--sizes: poll intervals k, default 1,4,16)")
    ap.add_argument("--no-dense", action="store_true",
                    help="crossover: time the linear-scaling path only")
    ap.add_argument("--sizes", default=None,
                    help="crossover sizes: lattice edges (cube) or atom counts (chain), "
                         "comma-separated")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): this library has "
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
    if args.peak_probe:
        return peak_probe()
    if args.crossover:
        return crossover(args)
    if args.lowdin:
        return lowdin_pipeline(args)
    if args.latency:
        return decision_latency(args)
    stream = torch.cuda.current_stream().cuda_stream

    # workload -> units: lists of systems solved in one context (one merged
    # launch per update).  A batch is packed into units of at most
    # --group-atoms atoms so that each unit's iterates fit in HBM.
    batch = args.workload.startswith("batch")
    if batch:
        n_sys = int(args.workload[5:] or 32)
        systems = W.batch_systems(n_sys=n_sys)
        units = W.pack_units(systems, args.group_atoms)
        if args.units:
            pick = [int(x) for x in args.units.split(",")]
            if any(not 0 <= i < len(units) for i in pick):
                log(f"--units: indices must lie in 0..{len(units) - 1}")
                return 2
            units = [units[i] for i in pick]
            systems = [sy for un in units for sy in un]
    else:
        systems = [W.config_system(args.workload)]
        units = [systems]
    sysm = systems[0]
    D = len(sysm.H1)
    n_atoms = sum(sy.H.nb for sy in systems)
    log(f"workload {args.workload}: {len(systems)} system(s) in {len(units)} unit(s), atoms="
        f"{n_atoms} b={sysm.H.b} N={sum(sy.H.n for sy in systems)} dirs={D} "
        f"eps={sysm.eps} tol={sysm.tol}")

    tile_kw = (dict(tune=args.tune, tune_cache=args.tune_cache, graph=bool(args.graph))
               if args.kernel == "tile" else {})
    # plain FP64 path (every candidate block computed): the reference of the
    # gate and of the speed-up.  Both sides are timed the same way, without
    # kernel events or the useful-product count; those come from a separate,
    # untimed run of the chosen variant over the same (deterministic) updates.
    ref_kw = dict(precision="fp64", kernel=args.kernel, **tile_kw)
    chosen = args.precision
    closing = 0 if chosen == "fp64" else 2
    theta = None
    if args.skip == "mlp":
        from paper_2009_03551_amd import skipnet
        train_sys = [W.config_system("cube10", L=L, seed=500 + L, eps=sysm.eps, n_dir=D)
                     for L in (5, 6, 7)]
        t0 = time.perf_counter()
        x, y = skipnet.collect(train_sys)
        theta, losses = skipnet.train(x, y, epochs=25)
        log(f"skip network: {len(y)} logged candidates ({y.mean():.3f} dropped), loss "
            f"{losses[0]:.4f} -> {losses[-1]:.4f}, {time.perf_counter() - t0:.1f} s")
    variant = dict(precision=chosen, closing_fp64=closing, kernel=args.kernel, skip=args.skip,
                   fp64_first=args.fp64_first if chosen != "fp64" else 0,
                   wide=bool(args.wide and chosen != "fp64"))
    if args.kernel == "tile":
        variant.update(tile_kw)
    if theta is not None:
        variant.update(mlp_weights=theta, mlp_threshold=args.mlp_threshold,
                       mlp_bound_cap=args.mlp_cap, mlp_budget=args.mlp_budget)
    # the measurement run: kernel times by events and the exact useful count
    meas_kw = dict(variant, profile=True, count_useful=True)
    # references solved once per unit, their X1 kept on the host for the gate
    refs = []
    if not args.no_reference:
        refs.append(("plain FP64 GPU path", ref_kw))
    if args.skip == "mlp":
        bkw = dict(variant, skip="bound", count_useful=False)
        for k in ("mlp_weights", "mlp_threshold", "mlp_bound_cap", "mlp_budget"):
            bkw.pop(k)
        refs.append(("exact norm-bound screen, same precision variant", bkw))

    def solve_refs(u):
        """Each reference on unit u: one timed solve, then its X1 on the host."""
        out = []
        for name, kw in refs:
            sv = T.Solver(u, export=False, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = sv.run(stream=stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            t0 = time.perf_counter()
            snap = snapshot(sv, D)
            log(f"  {name}: {res[0].status_name} iters={res[0].iters} {res[0].branches} "
                f"{wall:.2f} s/solve (device {res[0].seconds:.2f} s); X1 snapshot of "
                f"{len(snap[0])} entries in {time.perf_counter() - t0:.1f} s")
            sv.close()
            out.append((name, res, snap, wall))
        return out

    gates, ref_s, ref_useful = {}, {}, {}
    def add_gate(name, g):
        if name not in gates:
            gates[name] = dict(g)
        else:
            cur = gates[name]
            if g["max_abs_dX1"] > cur["max_abs_dX1"]:
                cur["split"] = g.get("split")
            cur["max_abs_dX1"] = max(cur["max_abs_dX1"], g["max_abs_dX1"])
            cur["rel_dalpha"] = max(cur["rel_dalpha"], g["rel_dalpha"])
            cur["pass"] = cur["pass"] and g["pass"]

    results, per_unit = [], []
    if not batch:
        # ---- one system: steps are updates of the solve sequence
        u = units[0]
        for name, res, snap, wall in solve_refs(u):
            ref_s[name] = res[0].seconds
            refs_done = (name, res, snap)
            per_unit.append(refs_done)
        t0 = time.perf_counter()
        sv = T.Solver(u, export=False, metrics_log=args.metrics_log, **variant)
        setup_s = time.perf_counter() - t0  # validation, host set-up, upload
        done = []
        p, r = sv.advance(args.warmup, stream=stream)
        if r:
            done.append(r)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p, r = sv.advance(args.steps, stream=stream)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        if r:
            done.append(r)
        timed_exec = p["executed_flops"]
        assert p["updates"] == args.steps
        # finish the solve in progress (untimed): its iterate is the one gated
        while p["solve_open"] or not done:
            p, r = sv.advance(1, stream=stream)
            if r:
                done.append(r)
        results = done[-1]
        export_s = export_time(sv, D)
        for name, res, snap in per_unit:
            add_gate(name, gate(sv, snap, results, res, name, sysm.eps))
        sv.close()
        # the same updates again, untimed, with the useful-product count and
        # kernel events: the useful flops of the timed updates, kernel times
        mv = T.Solver(u, export=False, **meas_kw)
        mdone = []
        pm, r = mv.advance(args.warmup, stream=stream)
        if r:
            mdone.append(r)
        pm, r = mv.advance(args.steps, stream=stream)
        if r:
            mdone.append(r)
        timed_useful = pm["useful_flops"]
        while pm["solve_open"] or not mdone:
            pm, r = mv.advance(1, stream=stream)
            if r:
                mdone.append(r)
        mv.close()
        assert mdone[-1][0].branches == results[0].branches
        ms_per_step = elapsed / args.steps * 1e3
        value = timed_useful / elapsed / 1e9
        s_solve = sum(x.seconds for x in results[:1])
        log(f"{chosen}: {args.steps} updates in {elapsed:.3f} s ({ms_per_step:.1f} ms/update), "
            f"useful {timed_useful / 1e12:.3f} TF -> {value:.1f} GFLOP/s; solve "
            f"{results[0].iters} updates {results[0].branches} in {s_solve:.2f} s")
        results = mdone[-1]
        per = [[results]]
    else:
        # ---- batches: steps are solves of every unit, one unit at a time
        total_s, per = 0.0, []
        timed_useful = timed_exec = 0.0
        setup_s = export_s = None
        for u in units:
            rdone = solve_refs(u)
            for name, res, snap, wall in rdone:
                ref_s[name] = ref_s.get(name, 0.0) + res[0].seconds
            sv = T.Solver(u, export=False, **variant)
            for _ in range(args.warmup):
                sv.run(stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = [sv.run(stream=stream) for _ in range(args.steps)]
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
            total_s += dt
            timed_exec += sum(x.executed_flops for x in res[-1])
            for name, rres, snap, wall in rdone:
                add_gate(name, gate(sv, snap, res[-1], rres, name, sysm.eps))
            sv.close()
            # one untimed solve with the useful-product count and kernel events
            mv = T.Solver(u, export=False, **meas_kw)
            mres = mv.run(stream=stream)
            mv.close()
            timed_useful += sum(x.useful_flops for x in mres)
            log(f"  unit of {len(u)} systems / {sum(x.H.nb for x in u)} atoms: {dt:.2f} s/solve; "
                f"gate so far {gates}")
            results += mres
            per.append([mres])
        elapsed = total_s * args.steps
        ms_per_step = total_s * 1e3
        s_solve = total_s
        value = timed_useful / total_s / 1e9
        timed_exec = timed_exec

    r = results[0]
    useful = sum(x.useful_flops for x in results)
    executed = sum(x.executed_flops for x in results)
    # roofline of the dominant kernel: the numeric kernel kind (FP64, FP32,
    # BF16 operands, FP32 with FP64 sums) with the most numeric time, over the
    # last complete solve of every unit (the library times a context's launches
    # once, on its first system's result)
    ms_kind = [sum(res[-1][0].ms_numeric_kind[k] for res in per) for k in range(4)]
    dom = max(range(4), key=lambda k: ms_kind[k])
    dom_launches = sum(res[-1][0].numeric_launches_kind[dom] for res in per)
    dom_flops = sum(x.useful_flops_kind[dom] for res in per for x in res[-1])
    achieved = dom_flops / (ms_kind[dom] * 1e-3) / 1e12 if ms_kind[dom] > 0 else 0.0
    split = chosen == "bf16" and variant["wide"]  # FP64-sum kind on bfloat16 MFMAs
    peak = PEAK_TFLOPS["bf16" if split else ("fp64", "fp32", "bf16", "fp32")[dom]]
    pm = measured_peaks() or {}
    pk_meas = None if split else pm.get({0: "gemm_fp64_tflops", 1: "gemm_fp32_tflops",
                                         3: "gemm_fp32_tflops"}.get(dom, ""))
    kname = kernel_name(args.kernel, dom, D, r.tile_shape[dom], sysm.H.b, split)
    traffic = measured_traffic(kname.split("<")[0], args.workload,
                               ("fp64", "fp32", "bf16", "fp32w")[dom])
    plain = refs[0][0] if refs and refs[0][0] == "plain FP64 GPU path" else None
    config = {"workload": args.workload,
              "step": "one solve of every unit" if batch else "one TC2/TC2-CPSCF update",
              "systems": len(systems), "units": len(units),
              "atoms": n_atoms, "b": sysm.H.b, "N": sum(sy.H.n for sy in systems),
              "directions": D, "eps": sysm.eps, "tol": sysm.tol, "precision": chosen,
              "closing_fp64": closing, "iters": r.iters, "branches": r.branches,
              "status": r.status_name,
              "kernel": args.kernel, "skip": args.skip, "fp64_first": variant["fp64_first"],
              "wide_accumulate": variant["wide"], "tuned": bool(args.tune),
              "tile_shape": r.tile_shape, "graph_updates": r.graph_updates,
              "graph_captures": r.graph_captures,
              "screened_blocks": sum(res[-1][0].screened_blocks for res in per),
              "mlp_skipped_blocks": sum(res[-1][0].mlp_skipped_blocks for res in per)}
    if args.skip == "mlp":
        config.update(mlp_threshold=args.mlp_threshold, mlp_cap=args.mlp_cap or 4.0,
                      mlp_budget=args.mlp_budget or None,
                      mlp_updates=sum(res[-1][0].mlp_updates for res in per))
    if args.units:
        config["unit_indices"] = [int(x) for x in args.units.split(",")]
    if len(systems) > 1:
        config["iters_range"] = [min(x.iters for x in results), max(x.iters for x in results)]
    out = {
        "metric": "TC2+response s/solve & useful GFLOP/s, chosen vs plain FP64 at max|dX1|<1e-6",
        "value": round(value, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "s_per_solve": round(s_solve, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[chosen],
        "data": "synthetic",
        "config": config,
        "plain_fp64": None if plain is None else {
            "s_per_solve": round(ref_s[plain], 4)},
        "speedup_vs_plain_fp64": None if plain is None else round(ref_s[plain] / s_solve, 3),
        "gate": gates.get(plain),
        "mlp_vs_bound": gates.get("exact norm-bound screen, same precision variant"),
        "timed_useful_tflop": round(timed_useful / 1e12, 4),
        "timed_executed_tflop": round(timed_exec / 1e12, 4),
        "useful_tflop_per_solve": round(useful / 1e12, 4),
        "union_tflop_per_solve": round(sum(x.union_flops for x in results) / 1e12, 4),
        "nominal_tflop_per_solve": round(sum(x.nominal_flops for x in results) / 1e12, 4),
        "executed_tflop_per_solve": round(executed / 1e12, 4),
        "roofline": {"bound": "mfma",
                     "kernel": kname, "achieved": round(achieved, 3),
                     "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                     "traffic": traffic,
                     "peak_measured": pk_meas,
                     "frac_of_measured": (round(achieved / pk_meas, 4) if pk_meas else None),
                     "launches_per_solve": dom_launches,
                     "avg_launch_ms": round(ms_kind[dom] / max(dom_launches, 1), 4),
                     "useful_tflop_per_solve": round(dom_flops / 1e12, 4),
                     "all_numeric_ms_per_kind": [round(x, 3) for x in ms_kind]},
    }
    if setup_s is not None:
        # from host buffers to host results: tc2_setup (validation, host
        # set-up, upload), one solve, and every entry of X0 and X1 copied back
        tot = setup_s + s_solve + export_s
        out["pcie_inclusive"] = {"setup_s": round(setup_s, 3), "solve_s": round(s_solve, 3),
                                 "export_s": round(export_s, 3), "total_s": round(tot, 3),
                                 "useful_gflops": round(useful / tot / 1e9, 3)}
    if not args.no_cpu_baseline:
        if len(systems) == 1 and sysm.H.n <= 20000:
            log("cpu baseline (dense oracle) ...")
            out["cpu_baseline"] = cpu_baseline_dense(sysm, r.iters, useful)
        elif len(systems) == 1:
            log("cpu baseline (block-list oracle) ...")
            out["cpu_baseline"] = cpu_baseline_bsr(args.workload, sysm, useful)
        else:
            log("cpu baseline skipped: batch workload")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
