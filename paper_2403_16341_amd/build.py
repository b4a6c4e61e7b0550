"""Build step of the HIP library ``_lib/libnls.so`` (gfx950).

Every translation unit under ``csrc/`` is compiled with hipcc in parallel and
linked into one shared library exposing the C ABI of ``include/nls.h``.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libnls.so")
BUILD_DIR = os.path.join(ROOT, "_build")

ARCH = os.environ.get("NLS_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", CSRC, "-I", INCLUDE,
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
# device code: no packed FP32 instructions (some of their forms have given
# wrong results on gfx950 without any error); FMA contraction allowed
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=fast",
          # the group kernels unroll their LU fully up to n = 64 (row arrays in
          # registers); the default limit for requested unrolling stops at 40
          "-mllvm", "-pragma-unroll-threshold=1000000",
          # atomics here are issued by one lane for its wavefront; the
          # compiler's cross-lane rewrite would wait for each result at once
          # instead of where it is used
          "-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]

GROUP_BUCKETS = (16, 24, 32, 40, 48, 56, 64)
SOURCES = [
    # (file, is_device)
    ("nls_host.cpp", False),
    ("nls_serve.cpp", False),
    ("nls_util.hip", True),
    ("nls_poly.hip", True),
    ("nls_sens.hip", True),
    ("nls_noalloc.hip", True),
    ("nls_lane_f64.hip", True),
    ("nls_lane_f32.hip", True),
] + [("nls_group_%s_nb%d.hip" % (p, nb), True) for p in ("f64", "f32") for nb in GROUP_BUCKETS]
HOST_CXX = os.environ.get("CXX", shutil.which("g++") or "g++")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _compile(src: str, device: bool) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    if device:
        cmd = [HIPCC, *COMMON, *DEVICE]
    else:
        # host-only runtime: plain C++ against the HIP runtime API headers
        cmd = [HOST_CXX, *COMMON, "-I", os.path.join(ROCM, "include"), "-D__HIP_PLATFORM_AMD__"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if res.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), msgs))
    return obj


def build(verbose: bool = True, jobs: int | None = None) -> str:
    """Compile every translation unit and link ``_lib/libnls.so``."""
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        futs = {ex.submit(_compile, s, d): s for s, d in SOURCES}
        objs = []
        for f in concurrent.futures.as_completed(futs):
            objs.append(f.result())
            if verbose:
                print("[nls build] compiled", futs[f], flush=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp, *sorted(objs),
           "-Wl,--no-undefined", "-pthread", "-L", os.path.join(ROCM, "lib"), "-lamdhip64"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed: %s\n%s%s" % (" ".join(cmd), res.stdout, res.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("[nls build] linked", LIB, flush=True)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
