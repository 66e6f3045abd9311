"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU: the oracle (gcc), libkxg's host-only planning code (GEMM work units,
Gauss-Legendre rule; property checks in tests/sanitize/plan_check.cpp) and
the host side of the whole library (argument checks, error paths; hipcc with
the sanitizers on the host pass only) under the CPU tests that call it.  A
planted overrun in a copy of the oracle shows that the harness reports."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLEAN = ("ERROR: AddressSanitizer", "runtime error:", "LeakSanitizer")


def _gcc_asan():
    return subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()


def _clang_asan():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def _run(cmd, preload, extra_env=None, timeout=900):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", LD_PRELOAD=preload)
    env.update(extra_env or {})
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=timeout)


def _assert_clean(r):
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    for bad in CLEAN:
        assert bad not in out, out[-4000:]


def test_planning_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", exe,
                    os.path.join(ROOT, "tests", "sanitize", "plan_check.cpp"),
                    os.path.join(ROOT, "paper_2607_00755_amd", "csrc", "kxg_plan.cpp")],
                   check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    _assert_clean(r)
    assert r.stdout.strip() == "ok"


def test_oracle_under_sanitizers(tmp_path):
    import oracle
    lib = oracle.build(sanitize=True, out=str(tmp_path / "liboracle_san.so"))
    r = _run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
              "tests/test_oracle_pins.py", "-k",
              "closed_form or projection or drift or freeze_in or condensate or gamma22 "
              "or cuts or direct_equals or quadratic or heun_step_size"],
             _gcc_asan(), {"ORACLE_LIBRARY": lib, "OMP_NUM_THREADS": "2"})
    _assert_clean(r)
    assert " passed" in r.stdout


@pytest.mark.skipif(_clang_asan() is None, reason="no clang ASan runtime in /opt/rocm/llvm")
def test_library_host_code_under_sanitizers(tmp_path):
    from paper_2607_00755_amd import build
    lib = build.build(sanitize=True, out_dir=str(tmp_path))
    r = _run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
              "tests/test_lib_cpu.py"], _clang_asan(), {"KXG_LIBRARY": lib})
    _assert_clean(r)
    assert " passed" in r.stdout


def test_sanitizer_reports_a_planted_overrun(tmp_path):
    """A copy of the oracle with one loop reading past its array: the
    sanitized build must report it (the harness above is not blind)."""
    src = open(os.path.join(ROOT, "oracle", "kxg_oracle.c")).read()
    good = "    for (int i = 0; i < n; ++i) {\n        N += h[i] * f[i];"
    assert good in src
    planted = src.replace(good, "    for (int i = 0; i <= n; ++i) {\n        N += h[i] * f[i];")
    c = tmp_path / "planted.c"
    c.write_text(planted)
    lib = str(tmp_path / "libplanted.so")
    subprocess.run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fopenmp", "-shared", "-fPIC", "-o", lib, str(c), "-lm"], check=True)
    prog = ("import ctypes, numpy as np\n"
            "L = ctypes.CDLL(%r)\n"
            "p = ctypes.POINTER(ctypes.c_double)\n"
            "h = np.ones(8); E = np.ones(8); f = np.ones(8); out = np.zeros(3)\n"
            "L.or_moments(ctypes.c_int(8), h.ctypes.data_as(p), E.ctypes.data_as(p),\n"
            "             f.ctypes.data_as(p), out.ctypes.data_as(p))\n" % lib)
    r = _run([sys.executable, "-c", prog], _gcc_asan())
    assert r.returncode != 0
    assert "AddressSanitizer" in r.stderr
