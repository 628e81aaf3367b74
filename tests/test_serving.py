"""Serving loop: request generation and summaries on the CPU; admission,
overlap, batching, per-request determinism and served solutions against the
oracle on the GPU."""
import numpy as np
import pytest

from paper_2208_08594_amd import msp, serve, synth


def test_request_stream_is_seeded():
    a = serve.make_requests(16, rate=5.0, seed=3)
    b = serve.make_requests(16, rate=5.0, seed=3)
    assert [(r.side, r.b, r.arrival) for r in a] == [(r.side, r.b, r.arrival) for r in b]
    assert all(r.side in synth.SERVING_SIDES and 3 <= r.b <= 7 for r in a)
    assert all(x.arrival < y.arrival for x, y in zip(a, a[1:]))
    capped = serve.make_requests(16, rate=5.0, sides=[16, 24])
    assert {r.side for r in capped} <= {16, 24}


def test_summary_statistics():
    reqs = serve.make_requests(4, rate=0.0)
    for k, r in enumerate(reqs):
        r.admitted = 0.0
        r.done = 0.1 * (k + 1)
        r.infos = [{"rebuilt": t == 0, "iterations": 5, "rel_true_residual": 1e-7}
                   for t in range(r.steps)]
    s = serve.summarize(reqs, makespan=0.4, max_active=2)
    assert s["solves"] == 16 and s["failed"] == 0
    assert abs(s["solves_per_s"] - 40.0) < 1e-9
    assert abs(s["p50_latency_ms"] - 250.0) < 1e-6 and s["rebuild_rate"] == 0.25


class _Replay:
    """Stands in for numpy's Generator in synth.assemble, handing out given
    draws (the coupling, then the rhs) in the order assemble asks for them."""

    def __init__(self, draws):
        self.draws = list(draws)

    def uniform(self, lo, hi, size=None):
        return self.draws.pop(0)


def test_device_generator_follows_the_host_law():
    """The torch generator of serving Jacobians (run here on the CPU) gives
    exactly the system synth.assemble builds from the same random draws."""
    import torch
    side, b, r = 5, 4, 7
    pats = synth.DevicePatterns(torch.device("cpu"))
    d = synth.serving_system_device(r, side, b, pats)
    gen = torch.Generator(device="cpu")
    gen.manual_seed(1000 + r)
    n = side ** 3
    f64 = torch.float64
    logk = torch.randn(n, generator=gen, dtype=f64).numpy()
    acc = (0.5 + 1.5 * torch.rand(n, generator=gen, dtype=f64)).numpy()
    C = (-0.1 + 0.2 * torch.rand((n, b, b), generator=gen, dtype=f64)).numpy()
    rhs = (2.0 * torch.rand(n * b, generator=gen, dtype=f64) - 1.0).numpy()
    k = np.exp(logk)
    ref = synth.assemble("replay", side, side, side, b, k, k, acc, _Replay([C, rhs]),
                         synth.corner_wells(side, side, side))
    assert np.array_equal(d["row_ptr"].numpy(), ref.row_ptr)
    assert np.array_equal(d["col_ind"].numpy(), ref.col_ind)
    assert np.allclose(d["vals"].numpy().reshape(ref.vals.shape), ref.vals, rtol=1e-14, atol=0)
    assert np.array_equal(d["rhs"].numpy(), ref.rhs)
    keep = d["keep"].numpy().reshape(ref.vals.shape)
    assert np.array_equal(keep, np.repeat(ref.dirichlet_row_mask()[:, :, None], b, axis=2))


def _small_requests(n, rate):
    reqs = serve.make_requests(n, rate=rate, steps=3, sides=[16, 24], seed=5)
    return reqs


@pytest.mark.gpu
def test_request_result_same_alone_and_in_mix():
    print("[case] serving determinism", flush=True)
    alone = _small_requests(6, rate=0.0)
    serve.Server(slots=1, mu=5, keep_x=True).run(alone)
    mixed = _small_requests(6, rate=0.0)
    res = serve.Server(slots=4, mu=5, keep_x=True).run(mixed)
    assert res["failed"] == 0 and res["max_concurrent"] > 1
    for a, m in zip(alone, mixed):
        assert [i["iterations"] for i in a.infos] == [i["iterations"] for i in m.infos]
        assert np.array_equal(a.x_last, m.x_last)
        assert all(i["rel_true_residual"] <= 1e-6 for i in m.infos)


@pytest.mark.gpu
def test_admission_waits_for_memory():
    print("[case] serving admission", flush=True)
    reqs = _small_requests(4, rate=0.0)
    srv = serve.Server(slots=4, mu=5)
    one = max(srv.footprint(r) for r in reqs)
    srv.hbm_budget = one  # room for a single request at a time
    res = srv.run(reqs)
    assert res["failed"] == 0 and res["max_concurrent"] == 1 and res["solves"] == 12


@pytest.mark.gpu
def test_adaptive_reuse_in_serving():
    print("[case] serving reuse", flush=True)
    reqs = _small_requests(3, rate=0.0)
    res = serve.Server(slots=2, mu=1000).run(reqs)
    assert res["failed"] == 0
    for r in reqs:
        assert [bool(i["rebuilt"]) for i in r.infos] == [True, False, False]


@pytest.mark.gpu
def test_batched_solve_equals_single_solves():
    """msp_solve_batch over contexts of different sizes gives each system
    exactly the result of msp_solve on its own."""
    import torch
    print("[case] msp_solve_batch vs msp_solve", flush=True)
    systems = [synth.lognormal_grid(12, 10, 8, 3, 31, 1.0, 1.0, "corners2"),
               synth.lognormal_grid(16, 16, 16, 5, 32, 1.0, 1.0, "corners2"),
               synth.config(0)]
    alone, batch = [], []
    for s in systems:
        a = msp.Solver(max_coarse=100)
        a.setup(s)
        xa, ia = a.solve(s.rhs, rtol=1e-6)
        alone.append((xa.cpu().numpy(), ia))
        a.close()
    sols = []
    for s in systems:
        g = msp.Solver(max_coarse=100)
        g.setup(s)
        sols.append(g)
    rhs = [torch.as_tensor(s.rhs, device="cuda") for s in systems]
    xs = [torch.zeros(s.N, dtype=torch.float64, device="cuda") for s in systems]
    infos = msp.solve_batch(sols, rhs, xs, rtol=1e-6)
    for (xa, ia), xb, ib in zip(alone, xs, infos):
        assert ib["status"] == 0 and ib["iterations"] == ia["iterations"]
        assert np.array_equal(xb.cpu().numpy(), xa)
    for g in sols:
        g.close()


@pytest.mark.gpu
def test_served_solutions_match_the_oracle():
    """A mix of requests served in batched rounds: every
    served solution of the last Newton step satisfies the true residual bound
    on the served matrix, and equals the oracle's FP64 solve of that matrix
    to within what two solves to rtol 1e-6 can differ."""
    from oracle import oracle as O
    print("[case] served solutions vs oracle", flush=True)
    reqs = serve.make_requests(8, rate=0.0, steps=3, sides=[16, 24, 48], seed=9)
    res = serve.Server(slots=6, mu=5, keep_x=True).run(reqs)
    assert res["failed"] == 0 and res["rounds"] > 0 and res["max_batch_size"] > 1
    for r in reqs:
        rp, ci, vals, rhs = r.last_system
        n, b = len(rp) - 1, vals.shape[1]
        A = None
        import scipy.sparse as sp
        A = sp.bsr_matrix((vals, ci, rp), shape=(n * b, n * b))
        res_norm = np.linalg.norm(rhs - A @ r.x_last) / np.linalg.norm(rhs)
        assert res_norm <= 1e-6, (r.rid, res_norm)
        o = O.OracleSolver(max_coarse=10000)
        o.setup(n=n, b=b, p=0, row_ptr=rp, col_ind=ci, vals=vals)
        xo, it, rr, st = o.solve(rhs, 1e-6)
        o.close()
        err = np.linalg.norm(r.x_last - xo) / np.linalg.norm(xo)
        print(f"[case] request {r.rid} side {r.side} b {r.b}: "
              f"iterations {r.infos[-1]['iterations']} (oracle {it}), |x-xo|/|xo| {err:.1e}",
              flush=True)
        assert st == 0 and err <= 1e-4
        if r.infos[-1]["rebuilt"]:
            assert abs(r.infos[-1]["iterations"] - it) <= 1
