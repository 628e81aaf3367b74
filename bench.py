#!/usr/bin/env python
"""Benchmark of the CPR-type multi-stage preconditioned FGMRES solve on one MI355X.

One step = one Newton-step linear solve of the synthetic reservoir Jacobian:
msp_setup (ingest + preconditioner regeneration, mu = 0) followed by
msp_solve to a relative true residual of 1e-6, with every input already in
HBM.  The default workload is the 64x64x32-cell grid with 4 unknowns per cell
(lognormal permeability sigma 1.5, kz/kh 0.1, 4 wells; 524,288 unknowns).

Printed: one JSON line with time-to-1e-6 (ms per step), p50/p99, the FP32- vs
FP64-preconditioner comparison, SpMV and Gauss-Seidel bandwidth, the roofline
of the dominant kernel (HIP events on the solver's stream) and the CPU oracle
baseline on a bounded sample of the same workload.
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
FP64_MFMA_PEAK_TFLOPS = 78.6
KERNEL_SRC = os.path.join(ROOT, "paper_2208_08594_amd", "csrc", "msp_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "tri_sweep_traffic.md")
KERNEL_HDR = os.path.join(ROOT, "paper_2208_08594_amd", "csrc", "msp_kernels.h")


def lu_block():
    """Block size of the coarsest-level solver's block LU (kLuBlock)."""
    import re
    m = re.search(r"constexpr int kLuBlock = (\d+);", open(KERNEL_HDR).read())
    return int(m.group(1))


LU_BLOCK = lu_block()
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
    b = sys_.b
    return sys_.nnzb * b * b * 8 + sys_.nnzb * 4 + (sys_.n + 1) * 4 + 2 * sys_.N * 8


def gs_sweep_bytes(level0_nnz, n, val_bytes):
    # off-diagonal values + column indices, diagonal, f, x read once and written once
    off = level0_nnz - n
    return off * (val_bytes + 4) + n * val_bytes * 4


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
    solver = msp.Solver(mu=0, restart=30, max_iter=1000, max_coarse=10000,
                        precond_fp32=precond_fp32, bilu_order=args.bilu_order, stream=stream)
    infos = []

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
        log(f"{'fp32' if precond_fp32 else 'fp64'} step {k}: {times[-1]:.2f} ms, "
            f"{info['iterations']} it, relres {info['rel_true_residual']:.2e}, "
            f"setup {info['setup_ms']:.2f} ms (rebuild {info['rebuild_ms']:.2f}), "
            f"solve {info['solve_ms']:.2f} ms; phases "
            + " ".join(f"{v:.1f}" for v in info["phase_ms"][:8]))
    torch.cuda.synchronize()
    total_ms = (time.perf_counter() - t0) * 1e3
    return solver, x.clone(), times, total_ms, infos, stream


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg1", choices=sorted(WORKLOADS))
    ap.add_argument("--bilu-order", type=int, default=1, choices=[0, 1])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (PMC byte calibration) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solver path is single-GPU (see DESIGN.md for how "
              "it would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2208_08594_amd import msp, synth

    idx, desc = WORKLOADS[args.workload]
    log("generating", desc)
    sys_ = synth.config(idx)
    solver, x64, times, total_ms, infos, stream = run_gpu(sys_, args, False, args.steps,
                                                          args.warmup)
    ms_per_step = total_ms / args.steps
    last = infos[-1]
    setup_ms = float(np.median([i["setup_ms"] for i in infos]))
    solve_ms = float(np.median([i["solve_ms"] for i in infos]))

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

    # kernel timing with HIP events on the solver's stream
    xin = torch.rand(sys_.N, dtype=torch.float64, device=dev)
    yout = torch.empty_like(xin)
    reps = 50
    t_spmv = stage_ms(solver, stream, msp.STAGE_SPMV, reps, xin, yout)
    t_gs = stage_ms(solver, stream, msp.STAGE_GS0, reps) if last["n_levels"] > 1 else None
    t_bilu = stage_ms(solver, stream, msp.STAGE_BILU, 10)
    t_vc = stage_ms(solver, stream, msp.STAGE_VCYCLE, 10)
    t_pre = stage_ms(solver, stream, msp.STAGE_PRECOND, 10, xin, yout)
    t_coarse = stage_ms(solver, stream, msp.STAGE_COARSE, 20)
    t_upd = stage_ms(solver, stream, msp.STAGE_TRI_SWEEP, 10)
    b_spmv = spmv_bytes(sys_)
    lev0_nnz = int(solver.level(0)["row_ptr"][-1])
    b_gs = gs_sweep_bytes(lev0_nnz, sys_.n, 8)
    nL = last["level_rows"][-1]
    # the two triangles of the coarsest solve read n_L^2 entries in all
    b_coarse = nL * nL * 8 + 4 * nL * 8
    gbs = lambda by, ms: by / (ms * 1e-3) / 1e9
    log(f"SpMV {t_spmv*1e3:.1f} us ({gbs(b_spmv, t_spmv):.0f} GB/s); "
        f"GS0 {(t_gs or 0)*1e3:.1f} us; BILU {t_bilu*1e3:.1f} us; V-cycle {t_vc*1e3:.1f} us; "
        f"precond {t_pre*1e3:.1f} us; coarse {t_coarse*1e3:.1f} us ({gbs(b_coarse, t_coarse):.0f} GB/s)")

    # FP32 preconditioner on the same system
    fp32 = None
    if not args.no_fp32:
        s32, x32, t32, tot32, inf32, _ = run_gpu(sys_, args, True, max(3, args.steps // 2), 1)
        d = (x32 - x64).norm().item() / x64.norm().item()
        fp32 = {"ms_per_step": tot32 / len(t32),
                "setup_ms": float(np.median([i["setup_ms"] for i in inf32])),
                "solve_ms": float(np.median([i["solve_ms"] for i in inf32])),
                "iterations": inf32[-1]["iterations"],
                "rel_true_residual": inf32[-1]["rel_true_residual"],
                "rel_diff_vs_fp64_solution": d,
                "precond_apply_us": stage_ms(s32, stream, msp.STAGE_PRECOND, 10, xin, yout) * 1e3}
        s32.close()

    # dominant kernel of a step: the GEMM steps of the triangular-inverse
    # sweeps of the coarsest-level solver (FP64 matrix cores); the timed
    # launch is the largest one, W's last block column: C = -A B with A
    # (J P) x k and B k x P (P = LU_BLOCK, J the last block, k = sweep_depth):
    # algorithmic work 2 J P P k flops
    P = LU_BLOCK
    mr = max((nL - 1) // P * P, 1)
    kd = sweep_depth(solver.level(len(last["level_rows"]) - 1), P)
    upd_flops = 2.0 * mr * P * kd
    achieved = upd_flops / (t_upd * 1e-3) / 1e12
    roofline = {"kernel": f"k_dgemm_s (largest triangular-inverse sweep step of the coarsest-level "
                          f"solver, {mr}x{P}x{kd}, n_L={nL})", "bound": "mfma",
                "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_MFMA_PEAK_TFLOPS,
                "traffic": stored_traffic(f"{mr}x{P}x{kd}"),
                "flops_per_launch": upd_flops, "avg_launch_us": t_upd * 1e3,
                "algorithmic_bytes_per_launch": (mr * kd + kd * P + mr * P) * 8}
    roofline_spmv = {"kernel": f"k_spmv<{sys_.b}>", "bound": "hbm",
                     "achieved": gbs(b_spmv, t_spmv), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs(b_spmv, t_spmv) / HBM_PEAK_GBS, "bytes_per_launch": b_spmv,
                     "avg_launch_us": t_spmv * 1e3}
    serving = None
    if not args.no_serving:
        serving = serving_sample()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(sys_)

    out = {
        "metric": METRIC, "value": ms_per_step, "unit": "ms", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "rtol": 1e-6, "restart": 30,
                   "mu": 0, "max_coarse": 10000, "precond": "fp64",
                   "bilu_order": "natural" if args.bilu_order == 0 else "multicolor"},
        "p50_ms": percentile(times, 50), "p99_ms": percentile(times, 99),
        "setup_ms": setup_ms, "solve_ms": solve_ms, "iterations": last["iterations"],
        "setup_phase_ms": dict(zip(["pattern", "ingest", "decouple", "aggregation_chain",
                                    "level_layouts", "coarse_inverse_wait", "bilu",
                                    "worker_wait"],
                                   [round(v, 3) for v in last["phase_ms"][:8]])),
        "rel_true_residual": last["rel_true_residual"],
        "levels": last["level_rows"], "colors": last["n_colors"],
        "bilu_levels": [last["bilu_levels_fwd"], last["bilu_levels_bwd"]],
        "reuse_step_ms": float(np.median(reuse_t)),
        "spmv_gbs": gbs(b_spmv, t_spmv),
        "gs_gbs": gbs(b_gs, t_gs) if t_gs else None,
        "stage_us": {"spmv": t_spmv * 1e3, "gs_sweep_level0": t_gs and t_gs * 1e3,
                     "bilu_solve": t_bilu * 1e3, "vcycle": t_vc * 1e3,
                     "precond_apply": t_pre * 1e3, "coarse_solve": t_coarse * 1e3},
        "fp32_precond": fp32,
        "roofline": roofline,
        "roofline_spmv": roofline_spmv,
        "coarse_solve_gbs": gbs(b_coarse, t_coarse),
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    solver.close()
    torch.cuda.synchronize()
    log("done")


def sweep_depth(level, P):
    """Depth k of the largest sweep step of the coarsest solver, W's last block
    column J: J P minus the first row of U's band there.  U's block row s
    reaches columns below max(1 + the last column whose first stored row lies
    in blocks <= s, the end of block s + 1)."""
    rp, ci = level["row_ptr"], level["col_ind"]
    n = len(rp) - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    first_row = np.full(n, n)
    np.minimum.at(first_row, ci, rows)
    steps = (n + P - 1) // P
    ends = np.zeros(steps, dtype=np.int64)
    np.maximum.at(ends, first_row // P, np.arange(n) + 1)
    ends = np.maximum.accumulate(ends)
    J = steps - 1
    K = J * P
    us = 0
    while us < J and max(int(ends[us]), min(n, us * P + 2 * P)) <= K:
        us += 1
    return max(K - us * P, 1)


def source_hash():
    """sha256[:16] of the dominant kernel's source: the FP64 GEMM tile code
    (from its header comment to the end of the small-tile kernel), its
    launcher and the block size (which fixes the timed shape), so edits elsewhere in the
    file keep the stored counters valid."""
    import hashlib
    src = open(KERNEL_SRC).read()
    a = src.index("// C = alpha * A B + beta * C (row-major, FP64) on the matrix cores.")
    b = src.index("dgemm_tile<kGTs, kGTs, 2, 2>", a)
    b = src.index("\n}\n", b) + 3
    c = src.index("hipError_t launch_dgemm(")
    d = src.index("\n}\n", c) + 3
    key = src[a:b] + src[c:d] + f"tri_sweep W-last-column block={LU_BLOCK}"
    return hashlib.sha256(key.encode()).hexdigest()[:16]


def stored_traffic(shape):
    """HBM bytes per launch of the dominant kernel from the committed PMC
    summary, only if it was taken on the current kernel source and at the
    launch shape timed here (M x N x K)."""
    try:
        txt = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    vals = {}
    for line in txt.splitlines():
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].rsplit(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel source sha256[:16]") != source_hash():
        return None
    if vals.get("launch shape") != shape:
        return None
    try:
        return float(vals["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def calibrate_copy():
    import torch
    a = torch.rand(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": a.numel() * 8, "reps": 3}))


def serving_sample():
    """A short continuous-batching run (reported beside the main metric)."""
    from paper_2208_08594_amd import serve
    log("serving sample: 16 requests, sides 16..32, 4 slots, mu=10")
    cal = serve.make_requests(2, rate=0.0, steps=4, sides=[16, 24, 32])
    t = time.perf_counter()
    serve.Server(slots=1, mu=10).run(cal)
    per_req = (time.perf_counter() - t) / len(cal)
    rate = 0.7 * 4 / per_req
    reqs = serve.make_requests(16, rate=rate, steps=4, sides=[16, 24, 32])
    res = serve.Server(slots=4, mu=10).run(reqs)
    res.update({"arrival_rate_per_s": rate, "slots": 4, "mu": 10,
                "sample": "16 requests x 4 Newton steps, cubes 16^3..32^3, b 3..7"})
    res.pop("errors", None)
    return res


def cpu_baseline(sys_):
    """The oracle, as it is, on one full Newton step of the same workload."""
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
        s = O.OracleSolver()
        s.setup(sys_)
        t1 = time.perf_counter()
        x, it, rr, st = s.solve(sys_.rhs, 1e-6)
        t2 = time.perf_counter()
    s.close()
    return {"value": (t2 - t0) * 1e3, "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": "one full Newton step (setup + FGMRES to 1e-6) of the same system, "
                      f"sequential FP64 oracle, LAPACK on 1 thread; setup {1e3*(t1-t0):.0f} ms, "
                      f"solve {1e3*(t2-t1):.0f} ms, {it} iterations",
            "iterations": it}


if __name__ == "__main__":
    main()
