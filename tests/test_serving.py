"""Serving loop: request generation and summaries on the CPU; admission,
overlap and per-request determinism on the GPU."""
import numpy as np
import pytest

from paper_2208_08594_amd import serve, synth


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
