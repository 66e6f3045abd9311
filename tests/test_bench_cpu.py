"""Host-side checks of bench.py: the JSON contract fields it computes without
a GPU (counter lookup, --gpus guard)."""
import os
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_counted_traffic_matches_current_sources(tmp_path, monkeypatch):
    """The committed counter summary is used only while the GEMM sources are
    the ones it was taken on."""
    sha = bench.kernel_source_sha1(bench.GEMM_F32_SOURCES)
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "x.md").write_text("kernel_source_sha1: `%s`  (a remark)\ntraffic_bytes_per_launch: 123\n" % sha)
    (prof / "y.md").write_text("kernel_source_sha1: `%s`\ntraffic_bytes_per_launch: 123\n" % ("0" * 40))
    src = tmp_path / "paper_2607_00755_amd" / "csrc"
    src.mkdir(parents=True)
    for s in bench.GEMM_F32_SOURCES:
        (tmp_path / s).write_bytes(open(os.path.join(ROOT, s), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counted_traffic("x.md", bench.GEMM_F32_SOURCES) == 123
    assert bench.counted_traffic("y.md", bench.GEMM_F32_SOURCES) is None
    assert bench.counted_traffic("missing.md", bench.GEMM_F32_SOURCES) is None
    # a changed kernel source invalidates the summary
    (tmp_path / bench.GEMM_F32_SOURCES[0]).write_bytes(b"changed")
    assert bench.counted_traffic("x.md", bench.GEMM_F32_SOURCES) is None


def test_committed_gemm_profile_is_parseable():
    text = open(os.path.join(ROOT, "profiles", "gemm_f32_n256_b512.md")).read()
    assert "kernel_source_sha1:" in text and "traffic_bytes_per_launch:" in text


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


def test_oracle_thread_control_takes_effect():
    """The CPU baseline rows time the oracle at a given thread count; the
    count must reach the OpenMP runtime even after it has started."""
    import oracle
    from paper_2607_00755_amd import inputs
    before = oracle.max_threads()
    op = oracle.Operator(inputs.log_grid(12, 1e-2, 5.0))
    op.collision(np.ones(12))          # OpenMP runtime started
    try:
        oracle.set_threads(1)
        assert oracle.max_threads() == 1
        oracle.set_threads(2)
        assert oracle.max_threads() == 2
    finally:
        oracle.set_threads(before)


def test_sustainable_rate_rule():
    rows = [{"rate_req_per_s": 10.0, "queue_growth": 1.0, "keep_up": 1.0, "p99_s": 4.0},
            {"rate_req_per_s": 20.0, "queue_growth": 1.1, "keep_up": 0.98, "p99_s": 5.0},
            {"rate_req_per_s": 40.0, "queue_growth": 1.4, "keep_up": 0.93, "p99_s": 5.9},
            {"rate_req_per_s": 60.0, "queue_growth": 1.2, "keep_up": 0.7, "p99_s": 8.0}]
    # 60 req/s: completions fall behind arrivals although latency grew little
    assert bench.sustainable(rows)["rate_req_per_s"] == 40.0
    rows[2]["keep_up"] = 0.85
    assert bench.sustainable(rows)["rate_req_per_s"] == 20.0
    rows[2]["keep_up"] = 0.95
    rows[2]["queue_growth"] = 1.6   # late arrivals wait longer: a queue builds up
    assert bench.sustainable(rows)["rate_req_per_s"] == 20.0
    assert bench.sustainable([]) is None


def test_keep_up_ratio():
    """stats' keep_up: completions per second while requests arrive over the
    arrival rate, about 1 when the loop keeps up and capacity / offered rate
    when it does not (synthetic request records, no GPU)."""
    from types import SimpleNamespace as NS
    from paper_2607_00755_amd import serving

    def run(rate, capacity, n=400, lat=1.0):
        done, t_free = [], 0.0
        for j in range(n):
            a = j / rate
            start = max(a, t_free)              # one server of the given capacity
            t_free = start + 1.0 / capacity
            done.append(NS(rid=j, arrival=a, finished=start + lat, latency=start + lat - a,
                           status=1, steps=1, solve=NS(n=64)))
        srv = serving.Server.__new__(serving.Server)
        srv.groups = {}
        return srv.stats(done)["keep_up"]

    assert abs(run(20.0, 50.0) - 1.0) < 0.05
    assert abs(run(100.0, 50.0) - 0.5) < 0.05


def test_cpu_oracle_workload_rows():
    """Bounded oracle timings of the workloads: config-1 solve in full, the
    others scaled from a bounded part by the step ratio."""
    rows = bench.cpu_config_rows(full=False)
    assert [r["extrapolated"] for r in rows] == [False, True, True]
    assert rows[1]["measured_steps"] == 1000
    assert abs(rows[1]["wall_s"] - 10 * rows[1]["measured_s"]) <= 0.02 * rows[1]["wall_s"] + 0.01
    assert abs(rows[2]["wall_s"] - 100 * rows[2]["measured_s"]) <= 0.1 + 0.01 * rows[2]["wall_s"]
    assert bench.cpu_model()
