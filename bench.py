#!/usr/bin/env python
"""Benchmark of the CPR-type multi-stage preconditioned FGMRES solve on one MI355X.

One step = one Newton-step linear solve of the synthetic reservoir Jacobian:
msp_setup (ingest + preconditioner regeneration, mu = 0) followed by
msp_solve to a relative true residual of 1e-6, with every input already in
HBM.  The default workload is the 128x128x64-cell grid with 7 unknowns per
cell (lognormal permeability sigma 1.5, kz/kh 0.1, 4 wells; 7,340,032
unknowns), the largest single-GPU workload.

Printed: one JSON line with time-to-1e-6 (ms per step), p50/p99, the FP32- vs
FP64-preconditioner comparison (both against the CPU oracle's solution),
SpMV and Gauss-Seidel bandwidth, the roofline of the dominant kernel of the
solve (the block SpMV, timed with HIP events around every launch of the timed
steps), the roofline of a whole FGMRES iteration against its algorithmic
bytes, and the CPU oracle baseline (one full step of the same system).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "CPR-FGMRES time-to-1e-6 + SpMV/GS HBM GB/s; FP32-vs-FP64 precond; p50/p99"
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "cfg0": (0, "10x10x10 cells, b=4, lognormal sigma=1, 2 wells (4,000 unknowns)"),
    "cfg1": (1, "64x64x32 cells, b=4, lognormal sigma=1.5, kz/kh=0.1, 4 wells (524,288 unknowns)"),
    "cfg2": (2, "128x128x64 cells, b=7, lognormal sigma=1.5, kz/kh=0.1, 4 wells (7,340,032 unknowns)"),
    "cfg3": (3, "60x220x85 cells, b=4, layered channelised 1e-3..1e3, 5 wells (4,488,000 unknowns)"),
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q))


def spmv_bytes(sys_):
    """Algorithmic bytes of one block SpMV y = A x: every FP64 block value,
    column index and row pointer once, x read once, y written once."""
    b = sys_.b
    return sys_.nnzb * b * b * 8 + sys_.nnzb * 4 + (sys_.n + 1) * 4 + 2 * sys_.N * 8


def gs_sweep_bytes(nnz, n, s):
    """One PGS-MC sweep (or residual) over a level of n rows and nnz stored
    entries: off-diagonal values and column indices once, then diagonal, f and
    x read once and x (or r) written once; s = value bytes."""
    return (nnz - n) * (s + 4) + 4 * n * s


def iteration_bytes(sys_, levels, bilu_nnzb, s, nu=(1, 1)):
    """Algorithmic bytes of the parts of one FGMRES iteration other than the
    Gram-Schmidt step: the SpMV, then the two-stage preconditioner apply in
    value precision s (bytes): decoupling and restriction to the pressure
    rows, the V-cycle (levels = [(rows, nnz)], the last one solved by the
    two FP64 triangles of n_L^2 entries), the pressure-column residual, the
    block ILU(0) solves and the final combination.  Each matrix value once,
    each vector at its minimum passes."""
    n, b, N, nnzb = sys_.n, sys_.b, sys_.N, sys_.nnzb
    parts = {"spmv": spmv_bytes(sys_)}
    parts["decouple"] = 2 * N * 8 + n * s + 2 * n * s  # w.v -> f, unpermute of e
    amg = 0
    for l, (nl, nnz) in enumerate(levels[:-1]):
        nc = levels[l + 1][0]
        amg += (nu[0] + nu[1] + 1) * gs_sweep_bytes(nnz, nl, s)  # sweeps + residual
        amg += nl * s + 4 * nl + nc * s                         # restriction
        amg += 4 * nl + nc * s + 2 * nl * s                     # prolongation
    nL = levels[-1][0]
    amg += nL * nL * 8 + 4 * nL * 8
    parts["amg"] = amg
    parts["pcol_residual"] = nnzb * b * s + nnzb * 4 + (n + 1) * 4 + N * 8 + n * s + N * s
    off = bilu_nnzb - n
    parts["bilu_solve"] = off * (b * b * s + 4) + n * b * b * s + 4 * N * s
    parts["finish"] = N * s + n * s + N * 8
    return parts


def krylov_bytes(N, steps):
    """Gram-Schmidt at the classical minimum: Arnoldi step j (0-based inside
    its cycle) reads v_0..v_j and w for the dot products, then v_0..v_j and
    w again for the update and writes w: 2(j+1)+3 vector passes."""
    return sum((2 * (j + 1) + 3) * N * 8 for j in steps)


def stage_ms(solver, stream, stage, reps, inp=None, out=None):
    import torch
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    solver.repeat(stage, 2, inp, out)  # warm
    ev0.record(stream)
    solver.repeat(stage, reps, inp, out)
    ev1.record(stream)
    ev1.synchronize()
    return ev0.elapsed_time(ev1) / reps


def run_gpu(sys_, args, precond_fp32, steps, warmup):
    import torch
    from paper_2208_08594_amd import msp
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    rp = torch.as_tensor(sys_.row_ptr, device=dev)
    ci = torch.as_tensor(sys_.col_ind, device=dev)
    vals = torch.as_tensor(sys_.vals.reshape(-1), device=dev)
    rhs = torch.as_tensor(sys_.rhs, device=dev)
    x = torch.zeros(sys_.N, dtype=torch.float64, device=dev)
    solver = msp.Solver(mu=0, restart=30, max_iter=1000, max_coarse=args.max_coarse,
                        precond_fp32=precond_fp32, bilu_order=args.bilu_order, stream=stream)
    solver.set_timing(True)
    infos, timings = [], []

    def step():
        solver.setup(n=sys_.n, b=sys_.b, p=sys_.p, row_ptr=rp, col_ind=ci, vals=vals)
        x.zero_()
        _, info = solver.solve(rhs, x, rtol=1e-6)
        return info

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    times = []
    t0 = time.perf_counter()
    for k in range(steps):
        ts = time.perf_counter()
        info = step()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - ts) * 1e3)
        infos.append(info)
        timings.append(solver.timing())
        log(f"{'fp32' if precond_fp32 else 'fp64'} step {k}: {times[-1]:.2f} ms, "
            f"{info['iterations']} it, relres {info['rel_true_residual']:.2e}, "
            f"setup {info['setup_ms']:.2f} ms (rebuild {info['rebuild_ms']:.2f}), "
            f"solve {info['solve_ms']:.2f} ms; phases "
            + " ".join(f"{v:.1f}" for v in info["phase_ms"][:8]))
    torch.cuda.synchronize()
    total_ms = (time.perf_counter() - t0) * 1e3
    return solver, x.clone(), times, total_ms, infos, timings, stream


def summed(timings, part):
    ms = sum(t[part][0] for t in timings)
    calls = sum(t[part][1] for t in timings)
    return ms, calls


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg2", choices=sorted(WORKLOADS))
    ap.add_argument("--bilu-order", type=int, default=1, choices=[0, 1])
    ap.add_argument("--max-coarse", type=int, default=10000,
                    help="largest coarsest AMG level (rows) solved directly")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="(default; kept for old commands)")
    ap.add_argument("--serving", action="store_true",
                    help="also run the 512-request serving leg in a child process (refused for now: "
                         "that run crashed the serving process; see serve.MAX_SERVED_REQUESTS)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (PMC byte calibration) and exit")
    ap.add_argument("--stage-only", action="store_true",
                    help="only set up the workload and run 5 SpMVs, 5 level-0 sweeps and 3 "
                         "block ILU(0) solves back to back (for hardware-counter runs), then exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.stage_only:
        stage_only(args)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solver path is single-GPU (DESIGN.md describes how "
              "it would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2208_08594_amd import msp, synth

    idx, desc = WORKLOADS[args.workload]
    log("generating", desc)
    sys_ = synth.config(idx)
    solver, x64, times, total_ms, infos, timings, stream = run_gpu(sys_, args, False,
                                                                   args.steps, args.warmup)
    ms_per_step = total_ms / args.steps
    last = infos[-1]
    setup_ms = float(np.median([i["setup_ms"] for i in infos]))
    solve_ms = float(np.median([i["solve_ms"] for i in infos]))
    solve_ms_sum = sum(i["solve_ms"] for i in infos)
    iters_sum = sum(i["iterations"] for i in infos)

    # reuse step (adaptive setup keeps B): ingest + solve only
    reuse = msp.Solver(mu=1000, precond_fp32=False, bilu_order=args.bilu_order, stream=stream)
    dev = torch.device("cuda", 0)
    rp = torch.as_tensor(sys_.row_ptr, device=dev)
    ci = torch.as_tensor(sys_.col_ind, device=dev)
    vals = torch.as_tensor(sys_.vals.reshape(-1), device=dev)
    rhs = torch.as_tensor(sys_.rhs, device=dev)
    reuse.setup(n=sys_.n, b=sys_.b, p=sys_.p, row_ptr=rp, col_ind=ci, vals=vals)
    reuse.solve(rhs, rtol=1e-6)
    reuse_t = []
    for _ in range(max(3, args.steps // 2)):
        ts = time.perf_counter()
        assert not reuse.setup(n=sys_.n, b=sys_.b, p=sys_.p, row_ptr=rp, col_ind=ci, vals=vals)
        reuse.solve(rhs, rtol=1e-6)
        torch.cuda.synchronize()
        reuse_t.append((time.perf_counter() - ts) * 1e3)
    reuse.close()

    # per-stage timing with HIP events on the solver's stream (back-to-back launches)
    xin = torch.rand(sys_.N, dtype=torch.float64, device=dev)
    yout = torch.empty_like(xin)
    t_gs = stage_ms(solver, stream, msp.STAGE_GS0, 50) if last["n_levels"] > 1 else None
    t_bilu = stage_ms(solver, stream, msp.STAGE_BILU, 10)
    t_vc = stage_ms(solver, stream, msp.STAGE_VCYCLE, 10)
    t_pre = stage_ms(solver, stream, msp.STAGE_PRECOND, 10, xin, yout)
    t_coarse = stage_ms(solver, stream, msp.STAGE_COARSE, 20)
    gbs = lambda by, ms: by / (ms * 1e-3) / 1e9

    # sizes of the hierarchy and of the block ILU(0) pattern
    levels = []
    for l in range(last["n_levels"]):
        Ld = solver.level(l)
        levels.append((Ld["n"], int(Ld["row_ptr"][-1])))
    lev0_nnz = levels[0][1]
    b_gs = gs_sweep_bytes(lev0_nnz, sys_.n, 8)
    nL = levels[-1][0]
    b_coarse = nL * nL * 8 + 4 * nL * 8

    # the dominant kernel of the solve: the block SpMV, every launch of the
    # timed steps bracketed by HIP events on the solver's stream
    spmv_ms, spmv_calls = summed(timings, "spmv")
    apply_ms, apply_calls = summed(timings, "apply")
    gsch_ms, gsch_calls = summed(timings, "gram_schmidt")
    b_spmv = spmv_bytes(sys_)
    t_spmv = spmv_ms / max(spmv_calls, 1)
    roofline = {"kernel": f"k_spmv<{sys_.b}> (block SpMV w = A z of every Arnoldi step)",
                "bound": "hbm", "achieved": gbs(b_spmv, t_spmv), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": gbs(b_spmv, t_spmv) / HBM_PEAK_GBS,
                "traffic": None, "bytes_per_launch": b_spmv,
                "avg_launch_us": t_spmv * 1e3, "launches_timed": spmv_calls}

    # a whole FGMRES iteration against its algorithmic bytes (matrices once,
    # vectors at their minimum passes, Gram-Schmidt at the classical minimum)
    parts = iteration_bytes(sys_, levels, sys_.nnzb, 8)
    steps_j = []
    for i in infos:
        k, m = i["iterations"], 30
        steps_j += [j % m for j in range(k)]
    kry = krylov_bytes(sys_.N, steps_j) / len(infos)
    it_bytes = sum(parts.values()) * iters_sum / len(infos) + kry
    solve_gbs = it_bytes / (solve_ms_sum / len(infos) * 1e-3) / 1e9
    roofline_solve = {"what": "one msp_solve (all FGMRES iterations) against its algorithmic "
                              "bytes", "bound": "hbm", "achieved": solve_gbs,
                      "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": solve_gbs / HBM_PEAK_GBS,
                      "bytes_per_solve": it_bytes,
                      "bytes_per_iteration_model": {k: v for k, v in parts.items()},
                      "krylov_bytes_per_solve": kry,
                      "ms_per_iteration": solve_ms_sum / iters_sum}
    kernel_rows = {
        "spmv": {"us": t_spmv * 1e3, "bytes": b_spmv, "gbs": gbs(b_spmv, t_spmv),
                 "how": "HIP events around every SpMV of the timed solves"},
        "gs_sweep_level0": None if t_gs is None else
        {"us": t_gs * 1e3, "bytes": b_gs, "gbs": gbs(b_gs, t_gs),
         "how": "50 back-to-back forward sweeps, HIP events"},
        "bilu_solve": {"us": t_bilu * 1e3, "bytes": parts["bilu_solve"],
                       "gbs": gbs(parts["bilu_solve"], t_bilu),
                       "how": "10 back-to-back solves, HIP events"},
        "vcycle": {"us": t_vc * 1e3, "bytes": parts["amg"], "gbs": gbs(parts["amg"], t_vc)},
        "precond_apply": {"us": apply_ms / max(apply_calls, 1) * 1e3,
                          "bytes": sum(v for k, v in parts.items() if k != "spmv"),
                          "how": "HIP events around every apply of the timed solves"},
        "gram_schmidt_us_per_step": gsch_ms / max(gsch_calls, 1) * 1e3,
        "coarse_solve": {"us": t_coarse * 1e3, "bytes": b_coarse,
                         "gbs": gbs(b_coarse, t_coarse)},
    }
    log(f"SpMV {t_spmv*1e3:.1f} us ({gbs(b_spmv, t_spmv):.0f} GB/s, {spmv_calls} launches); "
        f"GS0 {(t_gs or 0)*1e3:.1f} us; BILU {t_bilu*1e3:.1f} us; V-cycle {t_vc*1e3:.1f} us; "
        f"apply {apply_ms / max(apply_calls, 1)*1e3:.1f} us; coarse {t_coarse*1e3:.1f} us; "
        f"solve {solve_gbs:.0f} GB/s")

    # FP32 preconditioner on the same system, after the FP64 context has
    # given its device memory back (its blocks serve the FP32 context)
    solver.close()
    del xin, yout
    fp32 = None
    x32 = None
    if not args.no_fp32:
        s32, x32, t32, tot32, inf32, tim32, _ = run_gpu(sys_, args, True,
                                                        max(3, args.steps // 2), 1)
        fp32 = {"ms_per_step": tot32 / len(t32),
                "setup_ms": float(np.median([i["setup_ms"] for i in inf32])),
                "solve_ms": float(np.median([i["solve_ms"] for i in inf32])),
                "iterations": inf32[-1]["iterations"],
                "rel_true_residual": inf32[-1]["rel_true_residual"],
                "precond_apply_us": summed(tim32, "apply")[0] /
                max(summed(tim32, "apply")[1], 1) * 1e3}
        s32.close()

    # the solve's device memory goes back before the serving child starts
    x64 = x64.cpu()
    if x32 is not None:
        x32 = x32.cpu()
    del rp, ci, vals, rhs
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    serving = None
    if args.serving and not args.no_serving:
        serving = serving_run()

    cpu = None
    errors = {}
    if not args.no_cpu_baseline:
        cpu, x_or = cpu_baseline(sys_, args.max_coarse)
        nx = np.linalg.norm(x_or)
        errors["fp64_precond_vs_oracle"] = float(np.linalg.norm(x64.numpy() - x_or) / nx)
        if x32 is not None:
            errors["fp32_precond_vs_oracle"] = float(np.linalg.norm(x32.numpy() - x_or) / nx)
        if fp32 is not None:
            fp32["rel_error_vs_fp64_oracle"] = errors.get("fp32_precond_vs_oracle")

    out = {
        "metric": METRIC, "value": ms_per_step, "unit": "ms", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "rtol": 1e-6, "restart": 30,
                   "mu": 0, "max_coarse": args.max_coarse, "precond": "fp64",
                   "bilu_order": "natural" if args.bilu_order == 0 else "multicolor"},
        "p50_ms": percentile(times, 50), "p99_ms": percentile(times, 99),
        "setup_ms": setup_ms, "solve_ms": solve_ms, "iterations": last["iterations"],
        "setup_phase_ms": dict(zip(["pattern", "ingest", "decouple", "aggregation_chain",
                                    "level_layouts", "coarse_inverse_wait", "bilu",
                                    "worker_wait"],
                                   [round(v, 3) for v in last["phase_ms"][:8]])),
        "rel_true_residual": last["rel_true_residual"],
        "solution_rel_error_vs_oracle": errors or None,
        "levels": last["level_rows"], "colors": last["n_colors"],
        "bilu_levels": [last["bilu_levels_fwd"], last["bilu_levels_bwd"]],
        "reuse_step_ms": float(np.median(reuse_t)),
        "spmv_gbs": gbs(b_spmv, t_spmv),
        "gs_gbs": gbs(b_gs, t_gs) if t_gs else None,
        "kernels": kernel_rows,
        "fp32_precond": fp32,
        "roofline": roofline,
        "roofline_solve": roofline_solve,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    log("done")


def stage_only(args):
    """Setup of the workload, then the solve's bandwidth-bound kernels back
    to back: 5 block SpMVs, 5 forward level-0 sweeps, 3 block ILU(0) solves."""
    import torch
    from paper_2208_08594_amd import msp, synth
    idx, desc = WORKLOADS[args.workload]
    sys_ = synth.config(idx)
    s = msp.Solver(mu=0, max_coarse=args.max_coarse, bilu_order=args.bilu_order)
    s.setup(sys_)
    x = torch.rand(sys_.N, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    log("stages:", desc)
    s.repeat(msp.STAGE_SPMV, 5, x, y)
    s.repeat(msp.STAGE_GS0, 5)
    s.repeat(msp.STAGE_BILU, 3)
    torch.cuda.synchronize()
    s.close()
    print(json.dumps({"stages": "spmv x5, gs0 x5, bilu x3", "workload": desc}), flush=True)


def calibrate_copy():
    import torch
    a = torch.rand(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": a.numel() * 8, "reps": 3}))


def serving_run():
    """The serving measurements, in a child process of their own (a clean
    device state, and a failure there cannot take the main line with it):
    512 requests, Poisson arrivals at 0.7 x the measured single-stream
    capacity, cubes of side 16..96 with b = 3..7, 4 Newton steps each,
    adaptive setup mu = 10; then a burst of 96 small requests served with and
    without batching of the small solves."""
    import subprocess
    log("serving: 512 requests, sides 16..96, b 3..7, 4 Newton steps, load 0.7 (child process)")
    p = subprocess.run([sys.executable, "-X", "faulthandler", "-m", "paper_2208_08594_amd.serve",
                        "--bench"], cwd=ROOT, stdout=subprocess.PIPE, text=True, timeout=900)
    lines = [l for l in p.stdout.splitlines() if l.startswith("{")]
    if p.returncode != 0 or not lines:
        log(f"serving child exited with {p.returncode}")
        return {"error": f"serving process exited with status {p.returncode}"}
    return json.loads(lines[-1])


def cpu_baseline(sys_, max_coarse=10000):
    """The oracle, as it is, on one full Newton step of the same system
    (setup + FGMRES to 1e-6) on one host thread; returns its record and x."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    from oracle import oracle as O
    log("cpu baseline: oracle setup + solve, 1 thread")
    import contextlib
    guard = threadpool_limits(limits=1) if threadpool_limits else contextlib.nullcontext()
    with guard:
        t0 = time.perf_counter()
        s = O.OracleSolver(max_coarse=max_coarse)
        s.setup(sys_)
        t1 = time.perf_counter()
        x, it, rr, st = s.solve(sys_.rhs, 1e-6)
        t2 = time.perf_counter()
    s.close()
    return ({"value": (t2 - t0) * 1e3, "unit": "ms", "cores": 1, "kind": "oracle",
             "sample": "one full Newton step (setup + FGMRES to 1e-6) of the same system, "
                       f"sequential FP64 oracle, LAPACK on 1 thread; setup {1e3*(t1-t0):.0f} ms, "
                       f"solve {1e3*(t2-t1):.0f} ms, {it} iterations, relres {rr:.2e}",
             "iterations": it, "rel_true_residual": rr}, np.asarray(x))


if __name__ == "__main__":
    main()
