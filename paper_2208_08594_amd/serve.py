"""Continuous-batching request loop over the libmsp C-ABI.

Each request is one reservoir Jacobian sequence: a cube of side s with block
size b drawn from the serving mix, solved for several Newton steps whose
matrix values are perturbed by 5% between steps (the adaptive SETUP of
Sec. 3.2 decides per step whether the preconditioner is rebuilt).

Scheduling:
  * requests arrive by a Poisson process (precomputed arrival times);
  * a request is admitted as soon as a slot is free AND its device footprint
    (msp_footprint + its input arrays) fits the remaining HBM budget; it waits
    otherwise (never fails for lack of memory);
  * every admitted request runs on its own HIP stream with its own solver
    context (kept resident across its Newton steps), on a worker thread, so
    the work of concurrent requests overlaps on the device;
  * when a request finishes its slot and memory are released and the next
    waiting request is admitted immediately.

Reported: per-request latency (arrival -> last Newton step done), p50/p99,
solves per second, admitted concurrency and the rebuild (reuse) rate.
"""
from __future__ import annotations

import argparse
import json
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import msp, synth


@dataclass
class Request:
    rid: int
    side: int
    b: int
    steps: int
    arrival: float                 # seconds after the start of the run
    seed: int
    footprint: int = 0
    admitted: float = -1.0
    done: float = -1.0
    infos: list = field(default_factory=list)
    x_norms: list = field(default_factory=list)
    x_last: object = None
    base: object = None            # the request's first Jacobian (host), built before the clock
    error: str | None = None


def make_requests(n_req, rate, seed=0, steps=4, sides=None, blocks=None):
    """n_req requests with exponential inter-arrival times of mean 1/rate."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n_req):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        side, b = synth.serving_request(r)
        if sides is not None:
            side = sides[r % len(sides)] if side not in sides else side
        if blocks is not None:
            b = blocks[r % len(blocks)] if b not in blocks else b
        out.append(Request(rid=r, side=side, b=b, steps=steps, arrival=t, seed=1000 + r))
    return out


class Server:
    def __init__(self, slots=4, hbm_budget=None, mu=10, rtol=1e-6, precond_fp32=False,
                 keep_x=False, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.slots = slots
        if hbm_budget is None:
            free, _total = torch.cuda.mem_get_info(self.device)
            hbm_budget = int(0.8 * free)
        self.hbm_budget = int(hbm_budget)
        self.mu = mu
        self.rtol = rtol
        self.precond_fp32 = precond_fp32
        self.keep_x = keep_x
        self.lock = threading.Condition()
        self.in_use = 0
        self.active = 0
        self.max_active = 0

    # -- one request on its own stream and context ----------------------------
    def _run(self, req: Request, t0: float):
        torch = self.torch
        try:
            base = req.base if req.base is not None else synth.serving_system(req.rid, req.side,
                                                                                 req.b)
            stream = torch.cuda.Stream(self.device)
            with torch.cuda.stream(stream):
                dev = self.device
                rp = torch.as_tensor(base.row_ptr, device=dev)
                ci = torch.as_tensor(base.col_ind, device=dev)
                vals0 = torch.as_tensor(base.vals.reshape(-1), device=dev)
                rhs0 = torch.as_tensor(base.rhs, device=dev)
                keep = torch.as_tensor(
                    np.repeat(base.dirichlet_row_mask(), base.b, axis=1).reshape(-1), device=dev)
                solver = msp.Solver(mu=self.mu, precond_fp32=self.precond_fp32, stream=stream,
                                    device=dev)
                x = torch.zeros(base.N, dtype=torch.float64, device=dev)
                for t in range(req.steps):
                    if t == 0:
                        vals, rhs = vals0, rhs0
                    else:
                        g = torch.Generator(device=dev)
                        g.manual_seed(req.seed * 1000 + t)
                        u = torch.rand(vals0.shape, generator=g, device=dev, dtype=torch.float64)
                        vals = torch.where(keep, vals0, vals0 * (1.0 + 0.05 * (2.0 * u - 1.0)))
                        rhs = 2.0 * torch.rand(rhs0.shape, generator=g, device=dev,
                                               dtype=torch.float64) - 1.0
                    solver.setup(n=base.n, b=base.b, p=base.p, row_ptr=rp, col_ind=ci, vals=vals)
                    x.zero_()
                    _, info = solver.solve(rhs, x, rtol=self.rtol)
                    req.infos.append(info)
                    req.x_norms.append(float(x.norm().item()))
                if self.keep_x:
                    req.x_last = x.detach().cpu().numpy()
                req.base = None
                stream.synchronize()
                solver.close()
        except Exception as e:  # recorded, the loop goes on
            req.error = repr(e)
        finally:
            req.done = time.perf_counter() - t0
            with self.lock:
                self.in_use -= req.footprint
                self.active -= 1
                self.lock.notify_all()

    def footprint(self, req: Request) -> int:
        n = req.side ** 3
        nnzb = n + 2 * 3 * (req.side - 1) * req.side ** 2
        inputs = nnzb * req.b * req.b * 8 * 3 + (n + 1 + nnzb) * 4 + n * req.b * 8 * 4
        return msp.footprint(n, nnzb, req.b, mu=self.mu, precond_fp32=self.precond_fp32) + inputs

    def run(self, requests):
        """Serve the requests; returns a summary dict."""
        for r in requests:
            r.footprint = self.footprint(r)
            if r.footprint > self.hbm_budget:
                raise ValueError(f"request {r.rid} needs {r.footprint} B, budget {self.hbm_budget}")
            # Jacobian assembly is the simulator's job: inputs exist before arrival
            r.base = synth.serving_system(r.rid, r.side, r.b)
        pending = sorted(requests, key=lambda r: r.arrival)
        threads = []
        t0 = time.perf_counter()
        i = 0
        while i < len(pending):
            req = pending[i]
            now = time.perf_counter() - t0
            if now < req.arrival:
                time.sleep(min(req.arrival - now, 0.05))
                continue
            with self.lock:
                while not (self.active < self.slots and self.in_use + req.footprint <= self.hbm_budget):
                    self.lock.wait(0.05)
                self.in_use += req.footprint
                self.active += 1
                self.max_active = max(self.max_active, self.active)
            req.admitted = time.perf_counter() - t0
            th = threading.Thread(target=self._run, args=(req, t0), daemon=True)
            th.start()
            threads.append(th)
            i += 1
        for th in threads:
            th.join()
        makespan = time.perf_counter() - t0
        return summarize(requests, makespan, self.max_active)


def summarize(requests, makespan, max_active):
    ok = [r for r in requests if r.error is None]
    lat = [r.done - r.arrival for r in ok]
    solves = sum(len(r.infos) for r in ok)
    rebuilt = sum(int(i["rebuilt"]) for r in ok for i in r.infos)
    return {
        "requests": len(requests), "failed": len(requests) - len(ok), "solves": solves,
        "makespan_s": makespan, "solves_per_s": solves / makespan if makespan > 0 else 0.0,
        "p50_latency_ms": 1e3 * float(np.percentile(lat, 50)) if lat else None,
        "p99_latency_ms": 1e3 * float(np.percentile(lat, 99)) if lat else None,
        "mean_queue_ms": 1e3 * float(np.mean([r.admitted - r.arrival for r in ok])) if ok else None,
        "max_concurrent": max_active,
        "rebuild_rate": rebuilt / solves if solves else None,
        "mean_iterations": float(np.mean([i["iterations"] for r in ok for i in r.infos])) if ok else None,
        "max_rel_residual": max((i["rel_true_residual"] for r in ok for i in r.infos), default=None),
        "errors": [r.error for r in requests if r.error][:3],
    }


def main():
    ap = argparse.ArgumentParser(description="continuous-batching serving benchmark")
    ap.add_argument("--requests", type=int, default=32)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--mu", type=int, default=10)
    ap.add_argument("--max-side", type=int, default=96)
    ap.add_argument("--load", type=float, default=0.7, help="arrival rate / 1-slot capacity")
    ap.add_argument("--fp32", action="store_true")
    args = ap.parse_args()
    sides = [s for s in synth.SERVING_SIDES if s <= args.max_side]
    cal = make_requests(4, rate=0.0, steps=args.steps, sides=sides)
    t = time.perf_counter()
    Server(slots=1, mu=args.mu, precond_fp32=args.fp32).run(cal)
    per_req = (time.perf_counter() - t) / len(cal)
    rate = args.load / per_req
    reqs = make_requests(args.requests, rate=rate, steps=args.steps, sides=sides)
    res = Server(slots=args.slots, mu=args.mu, precond_fp32=args.fp32).run(reqs)
    res.update({"arrival_rate_per_s": rate, "single_slot_s_per_request": per_req,
                "slots": args.slots, "mu": args.mu, "max_side": args.max_side})
    print(json.dumps(res))


if __name__ == "__main__":
    main()
