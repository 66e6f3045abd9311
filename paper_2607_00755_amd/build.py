"""Build libkxg.so in-tree with hipcc for gfx950.

Every translation unit is compiled with packed-FP32 instructions disabled;
the kernel-tensor build additionally with FMA contraction off, so that its
kinematic decisions do not depend on contraction.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libkxg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]
UNITS = {
    "kxg_api.cpp": ["-x", "hip"],
    "kxg_build.hip": ["-ffp-contract=off"],
    "kxg_eval.hip": [],
    "kxg_gemm_f32.hip": [],
    "kxg_gemm16.hip": [],
    "kxg_probe.hip": [],
    "kxg_step.hip": [],
    "kxg_plan.cpp": [],
}


# host-side AddressSanitizer + UndefinedBehaviorSanitizer (the device code is
# built as usual; each flag goes to the host pass only)
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-shared-libsan"]


def _compile(unit: str, build_dir: str = BUILD, extra=()) -> str:
    src = os.path.join(CSRC, unit)
    obj = os.path.join(build_dir, unit + ".o")
    cmd = [HIPCC] + COMMON + UNITS[unit] + list(extra) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in (r.stderr or "").splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (unit, err))
    if err.strip():
        sys.stderr.write(err + "\n")
    return obj


def build(verbose: bool = False, sanitize: bool = False, out_dir: str = None) -> str:
    """Compile and link libkxg.so (in-tree, or into out_dir; with sanitize,
    the host code carries ASan and UBSan, whose runtime the loading process
    must preload)."""
    build_dir = os.path.join(out_dir, "_build") if out_dir else BUILD
    lib = os.path.join(out_dir, "libkxg.so") if out_dir else LIB
    extra = SANITIZE if sanitize else []
    os.makedirs(build_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(lambda u: _compile(u, build_dir, extra), sorted(UNITS)))
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + extra + ["-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
