"""Continuous-batching loop: admission by footprint (CPU), overlap and
"same result alone and in the mix" (GPU)."""
import numpy as np
import pytest

from paper_2607_00755_amd import inputs, serving


def small_requests(count, rate=400.0, seed=31, ns=(32, 48)):
    g = inputs.rng(seed)
    t, out = 0.0, []
    for _ in range(count):
        lam = float(np.exp(g.uniform(np.log(1e-2), np.log(10.0))))
        pl = float(np.exp(g.uniform(np.log(0.05), np.log(0.5))))
        ph = float(np.exp(g.uniform(np.log(1.0), np.log(5.0))))
        ratio = float(g.uniform(0.1, 10.0))
        n = ns[int(g.integers(0, len(ns)))]
        t += float(g.exponential(1.0 / rate))
        out.append(inputs.Solve(lam, pl, ph, ratio, n=n, t_end=float(g.uniform(2.0, 4.0)),
                                arrival=t))
    return out


def test_u_end_radiation_era():
    assert abs(serving.u_end_of(1e2) - 0.5 * np.log(200.0)) < 1e-15
    assert abs(np.exp(serving.u_end_of(1e4)) - np.sqrt(2e4)) < 1e-9


def test_admission_refuses_when_budget_too_small():
    srv = serving.Server(budget_bytes=1000)
    done = srv.run(small_requests(3), realtime=False)
    assert len(done) == 3 and all(r.status == -4 for r in done)
    assert srv.refused == 3 and srv.used_bytes == 0


def test_stats_per_grid_size():
    """Latency percentiles overall and per grid size, warm-up and failed
    requests left out (host logic only)."""
    srv = serving.Server()
    done = []
    for rid, (n, lat, st) in enumerate([(64, 1.0, 1), (64, 3.0, 1), (128, 2.0, 1), (128, 9.0, -1),
                                        (64, 100.0, 1)]):
        r = serving.Request(rid, inputs.Solve(1.0, 0.1, 2.0, 0.5, n=n), arrival=0.0)
        r.finished, r.status, r.steps = lat, st, 10 * (rid + 1)
        done.append(r)
    s = srv.stats(done, warm=0)
    assert s["completed"] == 4 and s["failed"] == 1
    assert s["per_n"]["64"]["completed"] == 3 and s["per_n"]["128"]["completed"] == 1
    assert s["per_n"]["64"]["p50_s"] == 3.0 and s["per_n"]["128"]["p99_s"] == 2.0
    assert s["per_n"]["64"]["mean_steps"] == (10 + 20 + 50) / 3
    w = srv.stats(done, warm=4)
    assert w["completed"] == 1 and set(w["per_n"]) == {"64"}


@pytest.mark.gpu
def test_serving_overlap_and_mix_invariance():
    reqs = small_requests(14)
    srv = serving.Server(b_cap=16, rtol=1e-4, iters_per_tick=8, keep_results=True)
    done = srv.run(reqs)
    assert len(done) == 14 and all(r.status == 1 for r in done), [r.status for r in done]
    st = srv.stats(done)
    assert st["completed"] == 14 and st["p99_s"] >= st["p50_s"] > 0
    # requests were admitted while others were in flight
    assert max(st["mean_batch"].values()) > 1.5, st
    mixed = {r.rid: r for r in done}
    for rid in (0, 5, 11):
        alone = serving.Server(b_cap=16, rtol=1e-4, iters_per_tick=8, keep_results=True)
        one = reqs[rid]
        solo = alone.run([inputs.Solve(one.lam, one.p_low, one.p_high, one.ratio, n=one.n,
                                       t_end=one.t_end, arrival=0.0)])[0]
        a, b = solo.result, mixed[rid].result
        assert solo.steps == mixed[rid].steps
        assert np.max(np.abs(a - b)) <= 1e-5 * np.max(np.abs(b)), rid
