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
    requests left out; step-capped (2), cancelled (-5) and refused (-4)
    requests counted apart, not as completed (host logic only)."""
    srv = serving.Server()
    done = []
    for rid, (n, lat, st) in enumerate([(64, 1.0, 1), (64, 3.0, 1), (128, 2.0, 1), (128, 9.0, -1),
                                        (64, 100.0, 1), (64, 7.0, 2), (128, 4.0, -5),
                                        (128, 0.0, -4), (64, 5.0, -2)]):
        r = serving.Request(rid, inputs.Solve(1.0, 0.1, 2.0, 0.5, n=n), arrival=0.0)
        r.finished, r.status, r.steps = lat, st, 10 * (rid + 1)
        done.append(r)
    s = srv.stats(done, warm=0)
    assert s["completed"] == 4 and s["failed"] == 2
    assert s["truncated"] == 1 and s["cancelled"] == 1 and s["refused"] == 1
    assert s["per_n"]["64"]["completed"] == 3 and s["per_n"]["128"]["completed"] == 1
    assert s["per_n"]["64"]["p50_s"] == 3.0 and s["per_n"]["128"]["p99_s"] == 2.0
    assert s["per_n"]["64"]["mean_steps"] == (10 + 20 + 50) / 3
    assert s["per_n"]["64"]["max_steps"] == 50 and s["max_steps"] == 50
    w = srv.stats(done, warm=4)
    assert w["completed"] == 1 and set(w["per_n"]) == {"64"}


def test_cancel_waiting_requests():
    """Cancelled requests that have not been admitted leave the queue with
    status -5 (host logic only; no group exists)."""
    srv = serving.Server()
    waiting = [serving.Request(rid, inputs.Solve(1.0, 0.1, 2.0, 0.5, n=64), arrival=0.0)
               for rid in range(4)]
    srv.cancel(1)
    srv.cancel(3)
    done = []
    left = srv._apply_cancellations(waiting, 2.5, done)
    assert [r.rid for r in left] == [0, 2]
    assert [(r.rid, r.status, r.finished) for r in done] == [(1, -5, 2.5), (3, -5, 2.5)]
    assert srv._apply_cancellations(left, 3.0, done) == left


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


@pytest.mark.gpu
def test_serving_cancel_leaves_others_unchanged():
    """Three requests cancelled while running (or waiting) leave with status
    -5; every other request ends bit for bit as in a run without the
    cancellations (same steps, same final state)."""
    reqs = small_requests(12, seed=37)
    base = serving.Server(b_cap=16, rtol=1e-4, iters_per_tick=8, keep_results=True)
    ref = {r.rid: r for r in base.run(reqs, realtime=False)}
    srv = serving.Server(b_cap=16, rtol=1e-4, iters_per_tick=8, keep_results=True)
    cancel = (2, 5, 9)
    ticks = [0]

    def on_tick(ndone, ntotal):
        ticks[0] += 1
        if ticks[0] == 3:
            for rid in cancel:
                srv.cancel(rid)

    done = {r.rid: r for r in srv.run(reqs, realtime=False, on_tick=on_tick)}
    assert len(done) == 12
    assert all(done[rid].status == -5 for rid in cancel), [done[r].status for r in cancel]
    st = srv.stats(list(done.values()))
    assert st["cancelled"] == 3 and st["completed"] == 9
    for rid, r in done.items():
        if rid in cancel:
            continue
        assert r.status == 1 and r.steps == ref[rid].steps, rid
        assert np.array_equal(r.result, ref[rid].result), rid


@pytest.mark.gpu
def test_served_solves_match_oracle():
    """Served solves (FP64 contraction, adaptive Heun in ln a with drift,
    config-5 grid p in [1e-4, 20]) against the oracle's free-running adaptive
    Heun of the same solve: one request per grid size N = 64 and 128 at the
    shortest end time of the workload (t_end H_i = 100), run through the
    serving loop together.  Both sides take the same controller (rtol 1e-6)
    in FP64, so they agree to rtol level: 1e-5 max-norm, and step counts
    within 0.1 % (over some 2e4 steps a rounding difference may flip an
    accept decision now and then)."""
    import oracle
    reqs = [inputs.Solve(0.3, 0.12, 2.2, 0.8, n=64, t_end=100.0, arrival=0.0),
            inputs.Solve(0.02, 0.07, 1.6, 3.0, n=128, t_end=100.0, arrival=0.0)]
    srv = serving.Server(prec=serving.kxg.F64, b_cap=4, iters_per_tick=64, keep_results=True)
    done = {r.rid: r for r in srv.run(reqs, realtime=False)}
    for rid, sv in enumerate(reqs):
        r = done[rid]
        assert r.status == 1, r.status
        p = inputs.log_grid(sv.n, inputs.SERVING_PMIN, inputs.SERVING_PMAX)
        f0 = sv.f0(p)
        op = oracle.Operator(p)
        u_end = serving.u_end_of(sv.t_end)
        ref = op.heun(f0 * p ** 3, sv.lam, op.gamma0(f0), u_end, 1e-3, expansion=True,
                      rtol=1e-6, max_steps=200000)
        assert abs(r.steps - len(ref["dt"])) <= max(2, 1e-3 * len(ref["dt"])), \
            (sv.n, r.steps, len(ref["dt"]))
        want = ref["x"] / (np.exp(3 * u_end) * p ** 3)
        err = float(np.max(np.abs(r.result - want)) / np.max(np.abs(want)))
        assert err <= 1e-5, (sv.n, err)
