"""Studies on synthetic inputs, run through the libmsp C-ABI (GPU).

* Smoother comparison (the analogue of Table 1, Sec. 6): the AMG smoother of
  the MSP preconditioner is PGS-MC (Alg. 4.3) or weighted point Jacobi
  (PJAC); a Newton sequence of systems is solved with mu = 0 and the total
  FGMRES iterations and time are reported.  (The iteration counts of the
  CPU oracle on the same sequence, including sequential Gauss-Seidel in
  natural row order, come from oracle/smoother_iterations.py, which is test
  infrastructure and not part of this package.)
* Stages: the two-stage preconditioner (pressure, then R) against the
  paper's three stages (concentration, pressure, R; eq. MSP), with block
  ILU(0) or block Jacobi as R.
* Adaptive-setup sweep (the analogue of Tables 2/4/6, Sec. 6): the same
  sequence is solved with mu in {0, 10, 20, 30, 40}; reported are the number
  of preconditioner regenerations (SetupCalls), the fraction of time spent in
  setup (SetupRatio), the total iterations and the total time.

The Newton sequence is the request model of the serving loop: system s is
the base Jacobian with every stored value outside the Dirichlet rows scaled
by (1 + 0.05 u), u ~ U[-1, 1] drawn per step, and a fresh right-hand side.

    python -m paper_2208_08594_amd.studies --smoothers --mu-sweep --stages [--workload cfg1]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import msp, synth


def newton_sequence(base, steps, seed=77):
    return [base] + [synth.newton_step(base, s, seed) for s in range(1, steps)]


def _upload(seq, dev):
    import torch
    rp = torch.as_tensor(seq[0].row_ptr, device=dev)
    ci = torch.as_tensor(seq[0].col_ind, device=dev)
    vals = [torch.as_tensor(s.vals.reshape(-1), device=dev) for s in seq]
    rhs = [torch.as_tensor(s.rhs, device=dev) for s in seq]
    return rp, ci, vals, rhs


def run_sequence(seq, dev_arrays, rtol=1e-6, **opts):
    """Solve the sequence on the GPU with one context; per-step infos and the
    host wall time of setup and solve."""
    import torch
    rp, ci, vals, rhs = dev_arrays
    base = seq[0]
    g = msp.Solver(**opts)
    out = []
    try:
        for k in range(len(seq)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.setup(n=base.n, b=base.b, p=base.p, row_ptr=rp, col_ind=ci, vals=vals[k])
            t1 = time.perf_counter()
            x, info = g.solve(rhs[k], rtol=rtol)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            info = dict(info)
            info["setup_wall_ms"] = (t1 - t0) * 1e3
            info["solve_wall_ms"] = (t2 - t1) * 1e3
            out.append(info)
    finally:
        g.close()
    return out


def _summary(infos):
    setup = sum(i["setup_wall_ms"] for i in infos)
    solve = sum(i["solve_wall_ms"] for i in infos)
    return {"systems": len(infos), "iterations": sum(i["iterations"] for i in infos),
            "setup_calls": infos[-1]["setup_calls"],
            "time_ms": setup + solve, "setup_ratio": setup / (setup + solve),
            "max_rel_residual": max(i["rel_true_residual"] for i in infos),
            "all_converged": all(i["status"] == 0 for i in infos)}


def smoother_study(seq, dev_arrays):
    variants = [("PGS-MC", dict(smoother=0)),
                ("PJAC w=1", dict(smoother=1, jacobi_weight=1.0)),
                ("PJAC w=2/3", dict(smoother=1, jacobi_weight=2.0 / 3.0))]
    res = {}
    run_sequence(seq[:1], dev_arrays)  # warm-up
    for name, opts in variants:
        res[name] = _summary(run_sequence(seq, dev_arrays, **opts))
    return res


def stage_study(seq, dev_arrays):
    """Two stages (P, R; the default) against the paper's three (N, P, R),
    with block ILU(0) or block Jacobi as R."""
    run_sequence(seq[:1], dev_arrays)  # warm-up
    variants = [("P,R  R=BILU(0)", dict()), ("N,P,R  R=BILU(0)", dict(n_stage=1)),
                ("P,R  R=block Jacobi", dict(full_smoother=1)),
                ("N,P,R  R=block Jacobi", dict(full_smoother=1, n_stage=1))]
    return {name: _summary(run_sequence(seq, dev_arrays, **opts)) for name, opts in variants}


def mu_sweep(seq, dev_arrays, mus=(0, 10, 20, 30, 40)):
    run_sequence(seq[:1], dev_arrays)  # warm-up
    return {str(mu): _summary(run_sequence(seq, dev_arrays, mu=mu)) for mu in mus}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="cfg1", choices=["cfg0", "cfg1", "cfg2", "cfg3"])
    ap.add_argument("--systems", type=int, default=12, help="length of the Newton sequence")
    ap.add_argument("--smoothers", action="store_true")
    ap.add_argument("--mu-sweep", action="store_true")
    ap.add_argument("--stages", action="store_true", help="two versus three stages")
    args = ap.parse_args()
    import torch
    dev = torch.device("cuda", 0)
    base = synth.config(int(args.workload[3:]))
    seq = newton_sequence(base, args.systems)
    arrays = _upload(seq, dev)
    out = {"workload": f"{args.workload}: {base.name} n={base.n} b={base.b}",
           "systems": args.systems, "rtol": 1e-6,
           "sequence": "5% multiplicative perturbation per step, fresh rhs"}
    if args.smoothers:
        out["smoothers"] = smoother_study(seq, arrays)
    if args.mu_sweep:
        out["mu_sweep"] = mu_sweep(seq, arrays)
    if args.stages:
        out["stages"] = stage_study(seq, arrays)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
