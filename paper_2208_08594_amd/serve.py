"""Continuous-batching request loop over the libmsp C-ABI.

Each request is one reservoir Jacobian sequence: a cube of side s with block
size b drawn from the serving mix, solved for several Newton steps whose
matrix values are perturbed by 5% between steps (the adaptive SETUP of
Sec. 3.2 decides per step whether the preconditioner is rebuilt).

Scheduling (one host thread owns every framework and library call; the
concurrency is on the device):
  * requests arrive by a Poisson process (precomputed arrival times);
  * a request is admitted as soon as a slot is free AND its device footprint
    (msp_footprint + its input arrays) fits the remaining HBM budget; it waits
    otherwise (never fails for lack of memory);
  * an admitted request's Jacobian is drawn on the GPU (the simulator's
    assembly stands outside the solver; a 96^3, b = 7 request holds 2.4 GB of
    values) on a stream of its own, and its solver context is kept resident
    across its Newton steps;
  * the loop runs in rounds: every admitted request gets its next Newton
    step's matrix and its setup (the adaptive SETUP may keep its
    preconditioner), then ONE msp_solve_batch solves all of them together,
    queuing every solve's next Arnoldi step as soon as its previous one ends,
    so the solves of all active requests overlap on the device.  Requests
    join at the next round after their admission and leave when their last
    step is done (continuous batching at the Newton-step boundary);
  * when a request finishes, its slot and memory are released and waiting
    requests are admitted before the next round.

Reported: per-request latency (arrival -> last Newton step done), p50/p99,
solves per second, admitted concurrency, batch sizes and the rebuild
(reuse) rate.
"""
from __future__ import annotations

import argparse
import json
import sys
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
    last_system: object = None     # (row_ptr, col_ind, vals, rhs) of the last step, if kept
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


class _Live:
    """A request being served: its stream, context and device inputs."""

    def __init__(self, server, req: Request):
        torch = server.torch
        self.req = req
        self.stream = torch.cuda.Stream(server.device)
        with torch.cuda.stream(self.stream):
            self.sys = synth.serving_system_device(req.rid, req.side, req.b, server.patterns)
            self.x = torch.zeros(self.sys["rhs"].numel(), dtype=torch.float64,
                                 device=server.device)
        self.solver = msp.Solver(mu=server.mu, precond_fp32=server.precond_fp32,
                                 stream=self.stream, device=server.device)
        self.step = 0
        self.rhs = None
        self.vals = None

    def values(self, server):
        """Matrix and rhs of the current Newton step (on the request's stream):
        step 0 is the drawn system, later steps scale every stored value
        outside the Dirichlet rows by (1 + 0.05 u), u ~ U[-1, 1], and draw a
        fresh rhs."""
        torch = server.torch
        s = self.sys
        with torch.cuda.stream(self.stream):
            if self.step == 0:
                self.vals, self.rhs = s["vals"], s["rhs"]
            else:
                g = torch.Generator(device=server.device)
                g.manual_seed(self.req.seed * 1000 + self.step)
                u = torch.rand(s["vals"].shape, generator=g, device=server.device,
                               dtype=torch.float64)
                self.vals = torch.where(s["keep"], s["vals"],
                                        s["vals"] * (1.0 + 0.05 * (2.0 * u - 1.0)))
                self.rhs = 2.0 * torch.rand(s["rhs"].shape, generator=g,
                                            device=server.device, dtype=torch.float64) - 1.0

    def setup(self):
        s = self.sys
        self.solver.setup(n=s["n"], b=s["b"], p=s["p"], row_ptr=s["row_ptr"],
                          col_ind=s["col_ind"], vals=self.vals)
        with self.solver.torch.cuda.stream(self.stream):
            self.x.zero_()

    def record(self, server, info):
        req = self.req
        req.infos.append(info)
        with server.torch.cuda.stream(self.stream):
            req.x_norms.append(float(self.x.norm().item()))
        self.step += 1
        if self.step == req.steps and server.keep_x:
            s = self.sys
            req.x_last = self.x.detach().cpu().numpy()
            req.last_system = (s["row_ptr"].cpu().numpy(), s["col_ind"].cpu().numpy(),
                               self.vals.detach().cpu().numpy().reshape(-1, s["b"], s["b"]),
                               self.rhs.detach().cpu().numpy())

    def close(self):
        try:
            self.stream.synchronize()
        finally:
            self.solver.close()
            self.sys = self.vals = self.rhs = self.x = None


class Server:
    def __init__(self, slots=16, hbm_budget=None, mu=10, rtol=1e-6, precond_fp32=False,
                 keep_x=False, device="cuda:0", batch=True):
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
        self.batch = batch  # False: one msp_solve per request, one after another
        self.patterns = synth.DevicePatterns(self.device)
        self.in_use = 0
        self.max_active = 0
        self.batch_sizes = []

    def footprint(self, req: Request) -> int:
        n = req.side ** 3
        nnzb = n + 2 * 3 * (req.side - 1) * req.side ** 2
        inputs = nnzb * req.b * req.b * 8 * 3 + (n + 1 + nnzb) * 4 + n * req.b * 8 * 4
        return msp.footprint(n, nnzb, req.b, mu=self.mu, precond_fp32=self.precond_fp32) + inputs

    def _retire(self, lv: _Live, t0: float):
        try:
            lv.close()
        except Exception as e:
            lv.req.error = lv.req.error or repr(e)
        lv.req.done = time.perf_counter() - t0
        self.in_use -= lv.req.footprint

    def _round(self, live):
        """One Newton step of every live request: matrices and setups, then
        the solves (together, or one by one without batching)."""
        ready = []
        for lv in live:
            try:
                lv.values(self)
                lv.setup()
                ready.append(lv)
            except Exception as e:
                lv.req.error = repr(e)
        if not ready:
            return
        self.batch_sizes.append(len(ready))
        if self.batch:
            try:
                infos = msp.solve_batch([lv.solver for lv in ready], [lv.rhs for lv in ready],
                                        [lv.x for lv in ready], rtol=self.rtol)
            except Exception as e:
                for lv in ready:
                    lv.req.error = repr(e)
                return
        else:
            infos = []
            for lv in ready:
                try:
                    infos.append(lv.solver.solve(lv.rhs, lv.x, rtol=self.rtol)[1])
                except Exception as e:
                    lv.req.error = repr(e)
                    infos.append(None)
        for lv, info in zip(ready, infos):
            if info is None:
                continue
            if info["status"] < 0:
                lv.req.error = msp.STATUS.get(info["status"], info["status"])
            else:
                lv.record(self, info)

    def run(self, requests, progress=False):
        """Serve the requests; returns a summary dict.  progress: a line on
        stderr every 10 s (admitted and finished requests)."""
        for r in requests:
            r.footprint = self.footprint(r)
            if r.footprint > self.hbm_budget:
                raise ValueError(f"request {r.rid} needs {r.footprint} B, budget {self.hbm_budget}")
        for side in sorted({r.side for r in requests}):
            self.patterns.get(side)  # the grid patterns exist before the clock starts
        pending = sorted(requests, key=lambda r: r.arrival)
        live = []
        t0 = time.perf_counter()
        i = 0
        last_note = 0.0
        while i < len(pending) or live:
            now = time.perf_counter() - t0
            if progress and now - last_note >= 10.0:
                last_note = now
                fin = sum(1 for r in requests if r.done >= 0)
                print(f"[serve] {now:.0f} s: admitted {i}/{len(pending)}, finished {fin}",
                      file=sys.stderr, flush=True)
            # admission: arrived requests, while a slot and memory are free
            while (i < len(pending) and pending[i].arrival <= now and len(live) < self.slots
                   and self.in_use + pending[i].footprint <= self.hbm_budget):
                req = pending[i]
                i += 1
                req.admitted = now
                self.in_use += req.footprint
                try:
                    live.append(_Live(self, req))
                except Exception as e:
                    req.error = repr(e)
                    req.done = time.perf_counter() - t0
                    self.in_use -= req.footprint
            self.max_active = max(self.max_active, len(live))
            if not live:
                if i < len(pending):
                    time.sleep(max(0.0, min(pending[i].arrival - now, 0.05)))
                continue
            self._round(live)
            keep = []
            for lv in live:
                if lv.req.error is not None or lv.step >= lv.req.steps:
                    self._retire(lv, t0)
                else:
                    keep.append(lv)
            live = keep
        makespan = time.perf_counter() - t0
        res = summarize(requests, makespan, self.max_active)
        bs = self.batch_sizes
        res["rounds"] = len(bs)
        res["mean_batch_size"] = float(np.mean(bs)) if bs else 0.0
        res["max_batch_size"] = max(bs) if bs else 0
        return res


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


def calibrate(n_req=12, steps=4, sides=None, mu=10, precond_fp32=False):
    """Mean service time of one request alone (one slot, no batching), over
    the first n_req requests of the mix: the single-stream capacity is its
    inverse."""
    cal = make_requests(n_req, rate=0.0, steps=steps, sides=sides)
    srv = Server(slots=1, mu=mu, precond_fp32=precond_fp32, batch=False)
    t = time.perf_counter()
    srv.run(cal)
    return (time.perf_counter() - t) / len(cal)


# Runs of the full mix ended with a segmentation fault of the serving
# process after about 150 requests (at a torch call that draws a request's
# matrix); its cause is not yet found, so runs longer than the largest one
# that has completed are refused.
MAX_SERVED_REQUESTS = 128


def serve_mix(n_req=512, load=0.7, steps=4, slots=16, mu=10, max_side=96, precond_fp32=False,
              seed=0):
    """The serving workload: n_req requests with Poisson arrivals at `load`
    times the measured single-stream capacity, cubes of side in the serving
    set up to max_side, b in 3..7, `steps` Newton steps each."""
    if n_req > MAX_SERVED_REQUESTS:
        raise RuntimeError(f"serving runs of more than {MAX_SERVED_REQUESTS} requests are "
                           "disabled: the 512-request mix crashed the serving process after "
                           "about 150 requests and the cause is not yet found")
    sides = [s for s in synth.SERVING_SIDES if s <= max_side]
    per_req = calibrate(steps=steps, sides=sides, mu=mu, precond_fp32=precond_fp32)
    rate = load / per_req
    reqs = make_requests(n_req, rate=rate, steps=steps, sides=sides, seed=seed)
    res = Server(slots=slots, mu=mu, precond_fp32=precond_fp32).run(reqs, progress=True)
    res.update({"arrival_rate_per_s": rate, "single_stream_s_per_request": per_req,
                "load": load, "slots": slots, "mu": mu, "max_side": max_side,
                "steps_per_request": steps})
    return res


def serve_bench():
    """The serving measurements reported beside the main benchmark: the
    512-request mix of serve_mix, then a burst of 96 small requests (sides
    16..32) all arriving at once, served with and without batching of the
    small solves."""
    res = serve_mix(n_req=512, load=0.7, steps=4, slots=16, mu=10, max_side=96)
    res.pop("errors", None)
    res["workload"] = ("512 requests x 4 Newton steps, cubes of side 16..96, b 3..7, "
                       "Poisson arrivals at 0.7 x single-stream capacity, mu = 10")
    burst = {}
    for name, batched in (("batched", True), ("one_request_at_a_time", False)):
        print(f"[serve] burst: 96 small requests at once, {name}", file=sys.stderr, flush=True)
        reqs = make_requests(96, rate=0.0, steps=4, sides=[16, 24, 32], seed=5)
        r = Server(slots=16 if batched else 1, mu=10, batch=batched).run(reqs)
        burst[name] = {k: r[k] for k in ("solves", "makespan_s", "solves_per_s", "p50_latency_ms",
                                         "p99_latency_ms", "max_concurrent", "mean_batch_size",
                                         "max_batch_size", "failed")}
    res["burst_small"] = burst
    return res


def main():
    ap = argparse.ArgumentParser(description="continuous-batching serving benchmark")
    ap.add_argument("--bench", action="store_true",
                    help="the 512-request mix and the small-request burst, one JSON line")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--mu", type=int, default=10)
    ap.add_argument("--max-side", type=int, default=96)
    ap.add_argument("--load", type=float, default=0.7, help="arrival rate / 1-slot capacity")
    ap.add_argument("--fp32", action="store_true")
    args = ap.parse_args()
    if args.bench:
        print(json.dumps(serve_bench()), flush=True)
        return
    res = serve_mix(args.requests, args.load, args.steps, args.slots, args.mu, args.max_side,
                    args.fp32)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
