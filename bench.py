#!/usr/bin/env python3
"""Benchmark of the collision-operator hot path on one MI355X.

Step = one RK4 step of the batched FP32 workload (N = 256 log grid on
p/m in [1e-3, 20], B = 512 seeded bimodal distributions, lambda log-uniform in
[1e-3, 1e3]): four evaluations of C[f] (MFMA GEMM gain + FP64 loss,
projection) and the FP64 state update, all on the device.  value = C[f]
evaluations per second (4 B / step time), inputs resident in HBM.

Also reported: the plain FP64 single-distribution path at N = 256 (B = 1,
one HBM stream over the dense tensor) and the ratio, the 16-bit split path at
B = 4096, the roofline of the dominant kernel (GEMM duration from HIP events
on its own stream over the timed region) and the FP64 CPU oracle timed on the
host cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "C[f] evals/s at N=256 batched vs plain FP64; p50/p99 solve latency"
PEAK = {"f32": 157.3, "bf16": 2500.0, "f16": 2500.0, "f64": 78.6}   # TFLOP/s dense
HBM_PEAK = 8000.0                                                    # GB/s


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=800,
                    help="measured serving requests (after --serve-warm warm-up ones); 0 = skip")
    ap.add_argument("--serve-warm", type=int, default=200)
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--serve-check", type=int, default=32,
                    help="measured requests re-run alone and compared with their result in the mix")
    ap.add_argument("--serve-sweep", default="25,50,80,110,140",
                    help="comma-separated arrival rates of a saturation sweep; empty = none")
    ap.add_argument("--serve-sweep-requests", type=int, default=400,
                    help="measured requests per sweep rate, at least (see --serve-sweep-seconds)")
    ap.add_argument("--serve-sweep-seconds", type=float, default=12.0,
                    help="each sweep rate also runs at least this many seconds of arrivals, "
                         "several solve lifetimes, so that a queue can build up")
    ap.add_argument("--cpu-full", action="store_true",
                    help="time the oracle's 16-solve subsamples in full (minutes) instead of "
                         "extrapolating from a bounded part of each")
    ap.add_argument("--profile-run", nargs="?", const="gemm", default=None,
                    choices=("gemm", "stream384", "streamx384", "x3", "serve"),
                    help="short run for profilers: 'gemm' = the timed RK4 steps, the plain "
                         "FP64 path and a 1 GiB device copy (the calibration kernel); "
                         "'stream384' = 50 plain FP64 evaluations at N = 384 and the copy; "
                         "'streamx384' = 50 exact-form evaluations (Bose-Einstein, log "
                         "interpolation) at N = 384 in FP64 and in FP32, and the copy; "
                         "'x3' = --steps 16-bit RK4 steps (BF16x3, FP16x3, then FP16x2) at N = 256, "
                         "B = 4096 and the copy; 'serve' = 300 requests of the serving "
                         "workload at 60 req/s")
    return ap.parse_args()


def kernel_source_sha1(sources):
    """sha1 over the kernel's source files, concatenated in the given order."""
    import hashlib
    h = hashlib.sha1()
    for src in sources:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return h.hexdigest()


GEMM_F32_SOURCES = ("paper_2607_00755_amd/csrc/kxg_gemm_f32.hip",
                    "paper_2607_00755_amd/csrc/kxg_device.h",
                    "paper_2607_00755_amd/csrc/kxg_geom.h")
GEMM_X3_SOURCES = ("paper_2607_00755_amd/csrc/kxg_gemm16.hip",
                   "paper_2607_00755_amd/csrc/kxg_device.h",
                   "paper_2607_00755_amd/csrc/kxg_geom.h",
                   "paper_2607_00755_amd/csrc/kxg_plan.cpp")


def counted_traffic(profile_md, sources, key="traffic_bytes_per_launch"):
    """HBM bytes per launch (field `key`) from a committed counter summary, if
    it was taken on the current kernel sources (sha1 recorded in the
    summary), else None."""
    try:
        text = open(os.path.join(ROOT, "profiles", profile_md)).read()
        sha = kernel_source_sha1(sources)
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line and line.split(":")[0].strip() in ("kernel_source_sha1", key):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.split()[0].strip("`")   # first token; a remark may follow
    if fields.get("kernel_source_sha1") != sha or key not in fields:
        return None
    return int(float(fields[key]))


def serving_alone_check(serving, reqs, done, warm, count):
    """Re-run `count` measured requests alone (fresh server, same path) and
    compare their final state with the one they reached in the mix."""
    import numpy as np
    from paper_2607_00755_amd import inputs, kxg
    mixed = {r.rid: r for r in done if r.rid >= warm and r.status == 1}
    ids = sorted(mixed)
    sample = ids[::max(1, len(ids) // count)][:count]
    worst, same_steps = 0.0, True
    for rid in sample:
        one = reqs[rid]
        alone = serving.Server(prec=kxg.F32, b_cap=512, iters_per_tick=64, keep_results=True)
        solo = alone.run([inputs.Solve(one.lam, one.p_low, one.p_high, one.ratio, n=one.n,
                                       t_end=one.t_end, arrival=0.0)])[0]
        a, b = solo.result, mixed[rid].result
        worst = max(worst, float(np.max(np.abs(a - b)) / np.max(np.abs(b))))
        same_steps = same_steps and solo.steps == mixed[rid].steps
        del alone
    return {"requests": len(sample), "max_rel_diff": worst, "same_steps": same_steps}


def sustainable(rows):
    """The sweep row of the highest rate the loop keeps up with (rows in
    increasing rate): solves complete at least at 0.9 x the arrival rate
    while requests arrive (keep_up >= 0.9) and no queue builds up (the
    median latency of the last quarter of the arrivals is at most 1.5 x that
    of the first quarter); None if even the lowest rate is not kept up with.
    Continuous batching admits a burst into the batch rather than a queue,
    so latency alone grows slowly past capacity: the completion rate is the
    test.  The completed solves/s of a finite burst include the drain after
    the last arrival, so they sit below the offered rate even when the loop
    keeps up; a kept-up rate is itself the sustained throughput."""
    best = None
    for r in rows:
        if r["keep_up"] >= 0.9 and r["queue_growth"] <= 1.5:
            best = r
    return best


def serving_sweep(serving, args):
    """Arrival-rate sweep of the serving loop: p50/p99 latency, solves/s and
    the completion-to-arrival rate ratio per rate; the largest sustainable
    rate by `sustainable`."""
    from paper_2607_00755_amd import inputs, kxg
    rows = []
    for rate in [float(x) for x in args.serve_sweep.split(",") if x.strip()]:
        nr = max(args.serve_sweep_requests, int(round(args.serve_sweep_seconds * rate)))
        nw = max(1, nr // 5)
        reqs = inputs.serving_requests(nw + nr, rate=rate)
        srv = serving.Server(prec=kxg.F32, b_cap=512, iters_per_tick=64)
        t0 = time.perf_counter()
        done = srv.run(reqs)
        st = srv.stats(done, warm=nw)
        rows.append({"rate_req_per_s": rate, "requests": nr, "warmup": nw, "p50_s": round(st["p50_s"], 3),
                     "p99_s": round(st["p99_s"], 3), "solves_per_s": round(st["solves_per_s"], 2),
                     "queue_growth": round(st["queue_growth"], 3), "keep_up": round(st["keep_up"], 3),
                     "completion_rate_per_s": round(st["keep_up"] * rate, 1),
                     "completed": st["completed"], "truncated": st["truncated"],
                     "failed": st["failed"], "wall_s": round(time.perf_counter() - t0, 1)})
        log("serving sweep %.1f req/s: p50 %.3f s p99 %.3f s, %.2f solves/s, queue growth %.2f, "
            "keep-up %.2f" % (rate, st["p50_s"], st["p99_s"], st["solves_per_s"], st["queue_growth"],
                              st["keep_up"]))
        del srv
    best = sustainable(rows)
    return {"rates": rows, "min_requests_per_rate": args.serve_sweep_requests,
            "min_arrival_seconds_per_rate": args.serve_sweep_seconds,
            "max_sustainable_rate_req_per_s": None if best is None else best["rate_req_per_s"],
            "completion_rate_at_sustainable_per_s": None if best is None else best["completion_rate_per_s"],
            "rule": "highest rate at which solves complete at >= 0.9 x the arrival rate while "
                    "requests arrive (from one median latency after the first arrival to the "
                    "last) and late arrivals wait no longer than early ones (median latency of "
                    "the last quarter <= 1.5 x the first quarter's)"}


def packed_k(n):
    nb = (n + 15) // 16
    return nb * (nb + 1) // 2 * 256


import numpy as np


def single_paths(args, dev):
    """The plain single-distribution paths: FP64 stream at N = 384 (A is
    453 MB, larger than the 256 MB Infinity Cache, so the stream comes from
    HBM), the N = 32 FP64 RK4 run (100 steps, launch-bound, graph replay) and
    the N = 128 FP32 drift run (adaptive Heun until 1e4 accepted steps)."""
    import torch
    from paper_2607_00755_amd import inputs, kxg
    out = {}
    # HBM stream, N = 384 FP64
    n = 384
    p = inputs.log_grid(n, 1e-3, 20.0)
    k = kxg.Kernel(p, precs=(kxg.F64,), b_cap=1)
    f = torch.tensor(inputs.draw_solves(1)[0].f0(p)[None, :], device=dev)
    C = torch.empty_like(f)
    for _ in range(3):
        k.eval(f, prec=kxg.F64, out=C, diagnostics=False)
    torch.cuda.synchronize()
    reps = 100
    kxg.profile_begin(reps + 2)
    t0 = time.perf_counter()
    for _ in range(reps):
        k.eval(f, prec=kxg.F64, out=C, diagnostics=False)
    torch.cuda.synchronize()
    wl = (time.perf_counter() - t0) / reps
    ms, cnt = kxg.profile_end()
    us = 1e3 * ms / max(cnt, 1)
    # bytes of one launch: the packed kept blocks of A' (64 KiB each)
    nbytes = 65536 * k.stats()["blocks64"]
    gbps = nbytes / (us * 1e-6) / 1e9
    out["plain_fp64_n384"] = {"evals_per_s": round(1.0 / wl, 1), "stream_kernel_us": round(us, 2),
                              "stream_GBps": round(gbps, 1), "hbm_frac": round(gbps / HBM_PEAK, 4),
                              "bytes_per_launch": nbytes, "dense_tensor_bytes": 8 * n ** 3}
    log("plain fp64 N=384 stream: %.1f us, %.0f GB/s of packed blocks" % (us, gbps))
    del k
    # HBM stream, N = 416 FP32 (single-distribution handle: the packed kept
    # blocks in FP32, 32 KiB each; the dense A32 would be 288 MB)
    n = 416
    p = inputs.log_grid(n, 1e-3, 20.0)
    k = kxg.Kernel(p, precs=(kxg.F32,), b_cap=1)
    f = torch.tensor(inputs.draw_solves(1)[0].f0(p)[None, :], device=dev)
    C = torch.empty_like(f)
    for _ in range(3):
        k.eval(f, prec=kxg.F32, out=C, diagnostics=False)
    torch.cuda.synchronize()
    kxg.profile_begin(reps + 2)
    for _ in range(reps):
        k.eval(f, prec=kxg.F32, out=C, diagnostics=False)
    torch.cuda.synchronize()
    ms, cnt = kxg.profile_end()
    us = 1e3 * ms / max(cnt, 1)
    nbytes = 32768 * k.stats()["blocks64"]
    gbps = nbytes / (us * 1e-6) / 1e9
    out["plain_fp32_n416"] = {"stream_kernel_us": round(us, 2), "stream_GBps": round(gbps, 1),
                              "hbm_frac": round(gbps / HBM_PEAK, 4), "bytes_per_launch": nbytes,
                              "dense_tensor_bytes": 4 * n ** 3}
    log("plain fp32 N=416 stream: %.1f us, %.0f GB/s of packed blocks" % (us, gbps))
    del k
    # N = 32 FP64, RK4, 100 steps on a side stream (captured graph)
    w = inputs.single_fp64_n32()
    p = w.grid()
    k = kxg.Kernel(p, precs=(kxg.F64,), b_cap=1)
    side = torch.cuda.Stream()
    f0 = torch.tensor(w.f0()[0], device=dev)
    times = []
    for rep in range(3):
        st = kxg.Stepper(k, kind=kxg.RK4, prec=kxg.F64, b_cap=1)
        st.set(0, f0, lam=1.0, t_end=1e30, h_i=1.0, max_steps=100, stream=side)
        st.advance(1, stream=side)          # capture
        side.synchronize()
        st.set(0, f0, lam=1.0, t_end=1e30, h_i=1.0, max_steps=100, stream=side)
        side.synchronize()
        t0 = time.perf_counter()
        st.advance(100, stream=side)
        side.synchronize()
        times.append(time.perf_counter() - t0)
    best = min(times)
    out["single_fp64_n32_rk4"] = {"steps": 100, "ms_total": round(1e3 * best, 3),
                                  "us_per_step": round(1e6 * best / 100, 2),
                                  "us_per_eval": round(1e6 * best / 400, 2)}
    log("N=32 fp64 RK4: %.1f us/step" % (1e6 * best / 100))
    del k
    # N = 128 FP32, adaptive Heun with radiation drift, until 1e4 accepted steps
    w = inputs.single_fp32_n128()
    p = w.grid()
    s = w.solves[0]
    k = kxg.Kernel(p, precs=(kxg.F32,), b_cap=1)
    st = kxg.Stepper(k, kind=kxg.HEUN, prec=kxg.F32, b_cap=1, expansion=kxg.EXP_RADIATION)
    st.set(0, torch.tensor(w.f0()[0], device=dev), lam=s.lam, t_end=0.5 * np.log(2e4), dt=1e-3,
           h_i=0.0, max_steps=10000, stream=side)
    side.synchronize()
    t0 = time.perf_counter()
    it = 0
    while True:
        st.advance(256, stream=side)
        it += 256
        q = st.query(stream=side)[0]
        if q["status"] != 0 or it > 60000:
            break
    el = time.perf_counter() - t0
    out["single_fp32_n128_drift"] = {"accepted": q["steps"], "rejected": q["rejected"],
                                     "u_reached": round(q["t"], 4), "status": q["status"],
                                     "wall_s": round(el, 3),
                                     "us_per_attempt": round(1e6 * el / (q["steps"] + q["rejected"]), 2),
                                     "lambda": s.lam}
    log("N=128 fp32 drift: %d steps in %.2f s" % (q["steps"], el))
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_config_rows(full):
    """Wall time of the FP64 CPU oracle on the workloads' own inputs: the
    N = 32 single solve in full (one evaluation plus 100 RK4 steps), the
    N = 128 expanding solve (adaptive Heun until 1e4 accepted steps) and the
    seeded 16-solve subsample of the N = 256 batches (2000 RK4 steps each;
    the oracle is FP64 whatever precision the device path uses, so the FP32
    and 16-bit batches share it).  Without `full` the last two are timed on a
    bounded part (1000 of the 1e4 steps; 20 of the 2000 steps) and scaled up
    by the step ratio (the cost per step is the same throughout)."""
    import oracle
    from paper_2607_00755_amd import inputs
    rows = []
    w = inputs.single_fp64_n32()
    p = w.grid()
    f0 = w.f0()[0]
    t0 = time.perf_counter()
    op = oracle.Operator(p)
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    op.collision(f0, project=True)
    op.rk4(f0, 1.0, 0.1 / op.gamma0(f0), 100)
    rows.append({"workload": w.name, "work": "1 evaluation + 100 RK4 steps", "build_s": round(tb, 4),
                 "wall_s": round(time.perf_counter() - t0, 4), "extrapolated": False})
    w = inputs.single_fp32_n128()
    p = w.grid()
    f0 = w.f0()[0]
    s0 = w.solves[0]
    op = oracle.Operator(p)
    steps = 10000 if full else 1000
    t0 = time.perf_counter()
    r = op.heun(f0 * p ** 3, s0.lam, op.gamma0(f0), 0.5 * np.log(2e4), 1e-3, expansion=True,
                max_steps=steps)
    el = time.perf_counter() - t0
    done = len(r["dt"])
    rows.append({"workload": w.name, "work": "adaptive Heun in ln a, 1e4 accepted steps",
                 "measured_steps": done, "measured_s": round(el, 3),
                 "wall_s": round(el * 10000 / max(done, 1), 2), "extrapolated": done != 10000})
    w = inputs.batched_fp32_n256(512)
    p = w.grid()
    op = oracle.Operator(p)
    picks = np.linspace(0, 511, 16).astype(int)
    f0 = w.f0()
    steps = 2000 if full else 20
    t0 = time.perf_counter()
    for b in picks:
        sv = w.solves[b]
        op.rk4(f0[b], sv.lam, 0.1 / (sv.lam * op.gamma0(f0[b])), steps)
    el = time.perf_counter() - t0
    rows.append({"workload": "n256 batches, 16-solve subsample", "work": "16 solves x 2000 RK4 steps",
                 "measured_steps": steps, "measured_s": round(el, 3),
                 "wall_s": round(el * 2000 / steps, 1), "extrapolated": steps != 2000})
    return rows


def freeze_in_workload(dev, iters=400):
    """The two-source freeze-in evolution (Sec. 3 sources, Sec. 4.2 regimes)
    as a batch: 256 solves on an N = 128 FP32 grid, each a seeded lambda of a
    coupling scan with a condensate (N0 = 1, Gamma = 0.5 H_i, p0 = 0.8) and a
    Higgs-like decay source (kappa = 1, m_h = 5 m, T_i = 2 m), starting from
    f = 0 in the source-only regime (du = 0.01).  Times `iters` iterations
    (one source RK4 step or one Heun attempt per slot each) and the same
    batch on a plain expanding-run stepper (no sources, elastic operator on)
    for the cost of the freeze-in machinery (loss rates, sources, switch)."""
    import torch
    from paper_2607_00755_amd import inputs, kxg
    n, B = 128, 256
    p = inputs.log_grid(n, 1e-3, 20.0)
    rng = np.random.default_rng(20261202)
    lam = 10 ** rng.uniform(1.0, 3.0, B)
    k = kxg.Kernel(p, precs=(kxg.F32,), b_cap=B)
    out = {"workload": "freeze_in_fp32_n128_b256", "iterations": iters}
    f0 = torch.tensor(np.stack([s.f0(p) * 1e-2 for s in inputs.draw_solves(B, seed=3)]),
                      device=dev)
    zero = torch.zeros((B, n), dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()
    for label, fi in (("freeze_in", True), ("plain_expanding", False)):
        st = kxg.Stepper(k, kind=kxg.HEUN, prec=kxg.F32, b_cap=B, expansion=kxg.EXP_RADIATION,
                         freeze_in=fi)
        if fi:
            st.set_many(0, zero, lam, 4.0, dt=1e-3, h_i=1.0, src_n0=1.0, src_gamma=0.5,
                        src_p0=0.8, src_kappa=1.0, src_mh=5.0, src_ti=2.0, du_src=0.01,
                        eps_switch=1e-2)
        else:
            st.set_many(0, f0, lam * 1e-2, 4.0, dt=1e-3, h_i=1.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            st.advance(8, stream=stream)         # graph capture and warm-up
            stream.synchronize()
            t0 = time.perf_counter()
            st.advance(iters, stream=stream)
            stream.synchronize()
        el = time.perf_counter() - t0
        q = st.query()
        row = {"ms_per_iteration": round(1e3 * el / iters, 4),
               "slot_iterations_per_s": round(B * iters / el, 1)}
        if fi:
            row["slots_switched"] = sum(1 for r in q if r["phase"] == 1)
            row["mean_source_steps"] = round(float(np.mean([r["n_src"] for r in q])), 1)
        out[label] = row
        del st
    out["freeze_in_overhead"] = round(out["freeze_in"]["ms_per_iteration"] /
                                      out["plain_expanding"]["ms_per_iteration"], 3)
    log("freeze-in batch: %s" % out)
    return out


def paper_timing_curve(dev):
    """The paper's own timing workload (Sec. 5, Fig. run_time): one full-grid
    evaluation of the contact operator for the two-bump input of
    eq. benchmark_two_bump on q in [1e-3, 1e2] (m = lambda = a = 1), log grid,
    N_mu = 18, Bose-Einstein factors and log interpolation, no projection;
    FP64 and FP32, per N.  The kernel build (done once per grid here, per
    call in the paper's formulation) is timed separately."""
    import torch
    from paper_2607_00755_amd import inputs, kxg
    rows = []
    for n in (32, 64, 96, 128, 192, 256, 384):
        q = inputs.log_grid(n, 1e-3, 1e2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = kxg.Kernel(q, precs=(kxg.F64, kxg.F32), b_cap=1, brackets=True)
        build_ms = 1e3 * (time.perf_counter() - t0)
        f = torch.tensor(inputs.two_bump_benchmark(q)[None, :], device=dev)
        C = torch.empty_like(f)
        d = torch.empty((1, kxg.NDIAG), dtype=torch.float64, device=dev)
        # bytes one FP64 (FP32) evaluation streams: the weights and brackets
        # of the blocks that hold a weight, in both (kb, mb) orders
        nbx = k.stats()["blocks_exact"]
        row = {"n": n, "build_ms": round(build_ms, 2), "stream_bytes_f64": nbx * (65536 + 16384),
               "stream_bytes_f32": nbx * (32768 + 16384), "dense_bytes_f64": 10 * n ** 3}
        for prec in (kxg.F64, kxg.F32):
            for _ in range(3):
                k.eval(f, prec=prec, project=False, log_interp=True, eta=1, out=C, diag=d)
            torch.cuda.synchronize()
            reps = 30
            t0 = time.perf_counter()
            for _ in range(reps):
                k.eval(f, prec=prec, project=False, log_interp=True, eta=1, out=C, diag=d)
            torch.cuda.synchronize()
            row["us_per_eval_" + kxg.PREC_NAMES[prec]] = round(1e6 * (time.perf_counter() - t0) / reps, 2)
        rows.append(row)
        del k
        log("paper workload N=%d: %s" % (n, row))
    return rows


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the hot path runs on one GPU only (--gpus 1); how it would shard "
              "over several GPUs is described in the design notes, not implemented.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2607_00755_amd import inputs, kxg

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    if args.profile_run == "stream384":
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        n = 384
        p = inputs.log_grid(n, 1e-3, 20.0)
        k = kxg.Kernel(p, precs=(kxg.F64,), b_cap=1)
        f = torch.tensor(inputs.draw_solves(1)[0].f0(p)[None, :], device=dev)
        C = torch.empty_like(f)
        for _ in range(50):
            k.eval(f, prec=kxg.F64, out=C, diagnostics=False)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": "stream384", "evals": 50}), flush=True)
        return
    if args.profile_run == "streamx384":
        # the exact-form stream (eq. app_dense_collision with Bose-Einstein
        # factors and log interpolation, the paper's timing workload) at
        # N = 384 in FP64 and FP32, 50 evaluations each, then the
        # calibration copy
        n = 384
        p = inputs.log_grid(n, 1e-3, 1e2)
        k = kxg.Kernel(p, precs=(kxg.F64, kxg.F32), b_cap=1, brackets=True)
        f = torch.tensor(inputs.two_bump_benchmark(p)[None, :], device=dev)
        C = torch.empty_like(f)
        for prec in (kxg.F64, kxg.F32):
            for _ in range(50):
                k.eval(f, prec=prec, out=C, diagnostics=False, project=False, log_interp=True, eta=1)
        torch.cuda.synchronize()
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": "streamx384", "evals": 50}), flush=True)
        return
    if args.profile_run == "serve":
        # the serving loop under a moderate load: 60 req/s, 300 requests
        from paper_2607_00755_amd import serving
        reqs = inputs.serving_requests(300, rate=60.0)
        srv = serving.Server(prec=kxg.F32, b_cap=512, iters_per_tick=64)
        done = srv.run(reqs)
        st = srv.stats(done, warm=50)
        print(json.dumps({"profile_run": "serve", "p50_s": st["p50_s"], "p99_s": st["p99_s"],
                          "completed": st["completed"]}), flush=True)
        return
    if args.profile_run == "x3":
        # the 16-bit workload: N = 256, B = 4096 RK4 steps in BF16x3, FP16x3
        # and FP16x2 (graph replays on a side stream), then the calibration copy
        w4 = inputs.mixed_n256(4096)
        p4 = w4.grid()
        f4 = torch.tensor(w4.f0(), device=dev)
        k4 = kxg.Kernel(p4, precs=(kxg.BF16X3, kxg.F16X3, kxg.F16X2), b_cap=4096)
        side = torch.cuda.Stream()
        for prec in (kxg.BF16X3, kxg.F16X3, kxg.F16X2):
            st4 = kxg.Stepper(k4, kind=kxg.RK4, prec=prec, b_cap=4096)
            st4.set_many(0, f4, lam=[s.lam for s in w4.solves], t_end=1e30, h_i=1.0)
            torch.cuda.synchronize()       # sets on the default stream, steps on side
            st4.advance(args.steps, stream=side)
            side.synchronize()
            del st4
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": "x3", "steps": args.steps}), flush=True)
        return

    # ---------------- batched FP32 RK4 (the timed step) ----------------
    w = inputs.batched_fp32_n256(512)
    n, B = w.n, w.batch
    p = w.grid()
    f0 = torch.tensor(w.f0(), device=dev)
    t0 = time.time()
    ker = kxg.Kernel(p, precs=(kxg.F64, kxg.F32), b_cap=B)
    log("kernel build N=%d: %.3f s" % (n, time.time() - t0))
    st = kxg.Stepper(ker, kind=kxg.RK4, prec=kxg.F32, b_cap=B)
    st.set_many(0, f0, lam=[s.lam for s in w.solves], t_end=1e30, h_i=1.0)
    torch.cuda.synchronize()               # sets on the default stream, steps on run_stream
    # the timed steps run as they do in production: on a stream of their own,
    # each step one replay of the captured iteration (HIP graph)
    run_stream = torch.cuda.Stream()
    st.advance(args.warmup, stream=run_stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.advance(args.steps, stream=run_stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    value = 4 * B / (wall / args.steps)
    q = st.query()
    bad = sum(1 for x in q[:B] if x["status"] < 0)
    log("batched f32 RK4: %.3f ms/step, %.3e C-evals/s, %d failed slots" % (ms_step, value, bad))
    # GEMM launch times for the roofline: a further run of the same steps
    # with timing events around every GEMM launch (direct launches)
    prof_steps = min(args.steps, 100)
    kxg.profile_begin(4 * prof_steps + 8)
    st.advance(prof_steps, stream=run_stream)
    torch.cuda.synchronize()
    gemm_ms, gemm_n = kxg.profile_end()
    gemm_avg_ms = gemm_ms / max(gemm_n, 1)
    # algorithmic work of one launch: 2 flops per distribution and non-zero
    # entry of the symmetric (k <= m) packing of A' = A - delta_ik R_im (gain
    # and loss in one contraction); the MFMAs execute the kept 32 x 16 x 16
    # blocks, zeros inside them included
    info = ker.stats()
    flops_alg = 2.0 * B * info["nnz_packed"]
    flops_exec = 2.0 * B * 32 * 256 * info["nonzero_blocks"]
    flops_packed = 2.0 * B * n * packed_k(n)
    flops_dense = 2.0 * B * n * n * n
    achieved = flops_alg / (gemm_avg_ms * 1e-3) / 1e12
    achieved_exec = flops_exec / (gemm_avg_ms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK["f32"],
                "unit": "TFLOP/s", "frac": round(achieved / PEAK["f32"], 4),
                "traffic": counted_traffic("gemm_f32_n256_b512.md", GEMM_F32_SOURCES),
                "kernel": "k_gemm_f32<4>", "avg_launch_us": round(gemm_avg_ms * 1e3, 2),
                "launches": gemm_n, "flops_per_launch": flops_alg,
                "nnz_packed": info["nnz_packed"],
                "executed_flops_per_launch": flops_exec,
                "executed_tflops": round(achieved_exec, 2),
                "executed_frac": round(achieved_exec / PEAK["f32"], 4),
                "packed_flops_per_launch": flops_packed,
                "dense_equiv_flops_per_launch": flops_dense,
                "blocks_kept": "%d of %d" % (info["nonzero_blocks"], info["packed_blocks"])}

    extras = {}
    if args.profile_run:
        # calibration kernel for the HBM byte counters: a plain 1 GiB copy
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        args.no_extras, args.no_cpu_baseline, args.serve_requests = True, True, 0
    peaks = None
    if not args.profile_run:
        # what this chip sustains (independent MFMA loops on every SIMD, a
        # plain vector copy), beside the datasheet peaks
        peaks = kxg.peak_probe()
        extras["measured_peaks"] = {k: round(v, 1) for k, v in peaks.items()}
        roofline["measured_peak"] = round(peaks["mfma_f32_tflops"], 1)
        roofline["frac_of_measured"] = round(achieved / peaks["mfma_f32_tflops"], 4)
        roofline["executed_frac_of_measured"] = round(achieved_exec / peaks["mfma_f32_tflops"], 4)
        log("measured peaks: %s" % extras["measured_peaks"])
    # ---------------- plain FP64 single distribution ----------------
    # (projected C, no diagnostics: the same output as the batched step)
    f1 = f0[:1].contiguous()
    C1 = torch.empty_like(f1)
    for _ in range(5):
        ker.eval(f1, prec=kxg.F64, out=C1, diagnostics=False)
    torch.cuda.synchronize()
    reps = 200
    kxg.profile_begin(reps + 2)
    t0 = time.perf_counter()
    for _ in range(reps):
        ker.eval(f1, prec=kxg.F64, out=C1, diagnostics=False)
    torch.cuda.synchronize()
    plain_wall = (time.perf_counter() - t0) / reps
    s_ms, s_n = kxg.profile_end()
    stream_us = 1e3 * s_ms / max(s_n, 1)
    plain = 1.0 / plain_wall
    # the plain FP64 stream reads the kept blocks of the packed A' (the same
    # blocks as the FP32 operand, FP64, 64 KiB each), not the dense tensor
    bytes_stream = 65536.0 * ker.stats()["blocks64"]
    extras["plain_fp64"] = {"evals_per_s": round(plain, 1), "us_per_eval": round(1e6 * plain_wall, 2),
                            "stream_kernel_us": round(stream_us, 2),
                            "stream_GBps": round(bytes_stream / (stream_us * 1e-6) / 1e9, 1),
                            "hbm_frac": round(bytes_stream / (stream_us * 1e-6) / 1e9 / HBM_PEAK, 4),
                            "bytes_per_launch": int(bytes_stream), "dense_tensor_bytes": 8 * n ** 3}
    extras["batched_vs_plain_fp64"] = round(value / plain, 1)
    log("plain fp64 N=256: %.1f us/eval (stream kernel %.1f us, %.0f GB/s of packed blocks)" %
        (1e6 * plain_wall, stream_us, bytes_stream / (stream_us * 1e-6) / 1e9))
    if not args.no_extras:
        # the same evaluation with the packed operand evicted from the 256 MB
        # MALL first (a 1 GiB buffer written between evaluations)
        scratch = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        cold = []
        for r in range(20):
            scratch.fill_(float(r))
            kxg.profile_begin(2)
            ker.eval(f1, prec=kxg.F64, out=C1, diagnostics=False)
            torch.cuda.synchronize()
            c_ms, c_n = kxg.profile_end()
            cold.append(1e3 * c_ms / max(c_n, 1))
        del scratch
        cold_us = sorted(cold)[len(cold) // 2]
        extras["plain_fp64"]["cold_stream_kernel_us"] = round(cold_us, 2)
        extras["plain_fp64"]["cold_stream_GBps"] = round(bytes_stream / (cold_us * 1e-6) / 1e9, 1)
        extras["plain_fp64"]["cold_hbm_frac"] = round(bytes_stream / (cold_us * 1e-6) / 1e9 / HBM_PEAK, 4)
        log("plain fp64 N=256 cold: stream kernel %.1f us (median of 20), %.0f GB/s" %
            (cold_us, bytes_stream / (cold_us * 1e-6) / 1e9))

    if not args.no_extras:
        # ---------------- 16-bit split at B = 4096: RK4 steps ----------------
        w4 = inputs.mixed_n256(4096)
        f4 = torch.tensor(w4.f0(), device=dev)
        k4 = kxg.Kernel(p, precs=(kxg.BF16X3, kxg.F16X3, kxg.F16X2), b_cap=4096)
        info4 = k4.stats()
        blocks16 = info4["blocks16"]
        lams4 = [s.lam for s in w4.solves]
        for prec, name in ((kxg.BF16X3, "bf16x3"), (kxg.F16X3, "f16x3"), (kxg.F16X2, "f16x2")):
            st4 = kxg.Stepper(k4, kind=kxg.RK4, prec=prec, b_cap=4096)
            st4.set_many(0, f4, lam=lams4, t_end=1e30, h_i=1.0)
            torch.cuda.synchronize()       # sets on the default stream, steps on run_stream
            st4.advance(3, stream=run_stream)
            torch.cuda.synchronize()
            steps4 = 20
            t0 = time.perf_counter()
            st4.advance(steps4, stream=run_stream)
            torch.cuda.synchronize()
            wl = (time.perf_counter() - t0) / steps4
            kxg.profile_begin(4 * 5 + 8)
            st4.advance(5, stream=run_stream)
            torch.cuda.synchronize()
            g_ms, g_n = kxg.profile_end()
            g_us = 1e3 * g_ms / max(g_n, 1)
            # algorithmic work per GEMM: one product over the non-zero packed
            # entries; executed: the split products (3, or 2 for FP16 x2) over
            # the blocks multiplied (the group's i-blocks up to the last
            # non-zero one of each kept pair)
            fa = 2.0 * 4096 * info4["nnz_packed"]
            fl = (2 if prec == kxg.F16X2 else 3) * 2.0 * 4096 * 32 * 256 * blocks16
            extras[name + "_b4096"] = {
                "evals_per_s": round(4 * 4096 / wl, 1), "ms_per_rk4_step": round(1e3 * wl, 3),
                "gemm_us": round(g_us, 1),
                "alg_tflops": round(fa / (g_us * 1e-6) / 1e12, 1),
                "alg_frac": round(fa / (g_us * 1e-6) / 1e12 / PEAK["bf16"], 4),
                "executed_mfma_tflops": round(fl / (g_us * 1e-6) / 1e12, 1),
                "executed_mfma_frac": round(fl / (g_us * 1e-6) / 1e12 / PEAK["bf16"], 4),
                "executed_frac_of_measured": (round(fl / (g_us * 1e-6) / 1e12 / peaks["mfma_bf16_tflops"], 4)
                                              if peaks else None),
                "blocks": blocks16, "blocks_staged": info4["staged16"],
                "traffic": counted_traffic("gemm_x3_n256_b4096.md", GEMM_X3_SOURCES,
                                           "traffic_bytes_per_launch" + {kxg.BF16X3: "",
                                                                         kxg.F16X3: "_f16x3",
                                                                         kxg.F16X2: "_f16x2"}[prec])}
            log("%s B=4096 RK4: %.3f ms/step, gemm %.1f us" % (name, 1e3 * wl, g_us))
            del st4
        # split ablations: error of 256 rows against the FP64 path, GEMM time at B = 4096
        k64 = kxg.Kernel(p, precs=(kxg.F64,), b_cap=256)
        rows = f4[:256].contiguous()
        ref, _ = k64.eval(rows, prec=kxg.F64, diagnostics=False)
        abl = {}
        for prec, name in ((kxg.BF16X3, "bf16"), (kxg.F16X3, "f16")):
            for split, sname in ((3, "x3"), (2, "f_only_split"), (1, "no_split")):
                C, _ = k4.eval(rows, prec=prec, diagnostics=False, split=split)
                err = ((C - ref).abs().max(dim=1).values / ref.abs().max(dim=1).values).max().item()
                C4 = torch.empty_like(f4)
                k4.eval(f4, prec=prec, out=C4, diagnostics=False, split=split)
                torch.cuda.synchronize()
                kxg.profile_begin(8)
                for _ in range(5):
                    k4.eval(f4, prec=prec, out=C4, diagnostics=False, split=split)
                torch.cuda.synchronize()
                a_ms, a_n = kxg.profile_end()
                abl["%s_%s" % (name, sname)] = {"max_rel_err": float("%.3g" % err),
                                                "gemm_us": round(1e3 * a_ms / max(a_n, 1), 1)}
                del C4
        extras["split_ablation_b4096"] = abl
        log("split ablations: %s" % abl)
        del k4, k64

    if not args.no_extras:
        # ---------------- single-distribution paths ----------------
        extras.update(single_paths(args, dev))
        if peaks:
            for key in ("plain_fp64_n384", "plain_fp32_n416"):
                if key in extras:
                    extras[key]["frac_of_measured_read"] = round(extras[key]["stream_GBps"] / peaks["read_GBps"], 4)
        extras["paper_timing_workload_be_log"] = paper_timing_curve(dev)
        extras["freeze_in_fp32_n128_b256"] = freeze_in_workload(dev)

    # ---------------- serving loop (continuous batching) ----------------
    serve = None
    if args.serve_requests > 0:
        from paper_2607_00755_amd import serving
        reqs = inputs.serving_requests(args.serve_warm + args.serve_requests, rate=args.serve_rate)
        srv = serving.Server(prec=kxg.F32, b_cap=512, iters_per_tick=64, keep_results=args.serve_check > 0)
        t0 = time.perf_counter()
        done = srv.run(reqs)
        el = time.perf_counter() - t0
        serve = srv.stats(done, warm=args.serve_warm)
        serve.update({"requests": args.serve_requests, "warmup_requests": args.serve_warm,
                      "rate_req_per_s": args.serve_rate, "wall_s": round(el, 2), "prec": "f32",
                      "stepper": "adaptive Heun in ln a, rtol 1e-6, radiation drift",
                      "regime": "overload: the offered rate exceeds what the device completes, "
                                "so p50/p99 grow with the number of requests (see serving_sweep)"})
        serve["mean_batch"] = {str(k): round(v, 1) for k, v in serve["mean_batch"].items()}
        serve["per_n"] = {k: {q: round(v, 3) for q, v in d.items()} for k, d in serve["per_n"].items()}
        log("serving: p50 %.3f s p99 %.3f s, %.2f solves/s" %
            (serve["p50_s"], serve["p99_s"], serve["solves_per_s"]))
        del srv
        if args.serve_check > 0:
            serve["alone_check"] = serving_alone_check(serving, reqs, done, args.serve_warm, args.serve_check)
            log("serving: %d requests re-run alone, max rel diff %.2e, same steps %s" %
                (serve["alone_check"]["requests"], serve["alone_check"]["max_rel_diff"],
                 serve["alone_check"]["same_steps"]))
        done = None
        if args.serve_sweep:
            extras["serving_sweep"] = serving_sweep(serving, args)
            log("serving: largest sustainable rate %s req/s" %
                extras["serving_sweep"]["max_sustainable_rate_req_per_s"])

    # ---------------- CPU oracle baseline ----------------
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        threads = oracle.max_threads()
        op = oracle.Operator(p)
        fb = w.f0()[0]
        op.collision(fb, project=True)
        cnt, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds:
            op.collision(fb, project=True)
            cnt += 1
        el = time.perf_counter() - t0
        cpu = {"value": round(cnt / el, 2), "unit": "C-evals/s", "cores": threads, "kind": "oracle",
               "sample": "%d evaluations of one N=256 distribution (FP64 A/R contraction + "
                         "projection) in %.1f s" % (cnt, el),
               "cpu_model": cpu_model(), "nproc": os.cpu_count()}
        log("cpu oracle: %.2f C-evals/s on %d threads (%s)" % (cnt / el, threads, cpu["cpu_model"]))
        if not args.no_extras:
            # further rows: one thread at N = 256, all threads at N = 32, 128, 384
            rows = []
            for nn, th, secs in ((256, 1, 3.0), (32, threads, 1.5), (128, threads, 1.5), (384, threads, 3.0)):
                oracle.set_threads(th)
                pp = inputs.log_grid(nn, 1e-3, 20.0)
                o2 = oracle.Operator(pp)
                fx = inputs.draw_solves(1)[0].f0(pp)
                o2.collision(fx, project=True)
                c2, t1 = 0, time.perf_counter()
                while time.perf_counter() - t1 < secs:
                    o2.collision(fx, project=True)
                    c2 += 1
                e2 = time.perf_counter() - t1
                rows.append({"n": nn, "threads": th, "C_evals_per_s": round(c2 / e2, 2), "evals": c2})
                del o2
            oracle.set_threads(threads)
            extras["cpu_oracle_rows"] = rows
            log("cpu oracle rows: %s" % rows)
            extras["cpu_oracle_workloads"] = cpu_config_rows(args.cpu_full)
            log("cpu oracle workloads: %s" % extras["cpu_oracle_workloads"])

    out = {"metric": METRIC, "value": round(value, 1), "unit": "C-evals/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": w.name + " RK4 step (4 evals, projected, FP64 state)",
                      "n_grid": n, "batch": B, "p_range": [w.pmin, w.pmax], "n_mu": 18,
                      "parallelism": "1 GPU"},
           "roofline": roofline, "cpu_baseline": cpu,
           "p50_solve_latency_s": None if serve is None else round(serve["p50_s"], 4),
           "p99_solve_latency_s": None if serve is None else round(serve["p99_s"], 4),
           "serving": serve}
    out.update(extras)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
