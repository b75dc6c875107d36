"""Build libcfsim.so (HIP for gfx950) in-tree with hipcc.

Packed FP32 instructions are disabled (``-packed-fp32-ops``); every kernel is
plain FP32 VALU code. Multiply-add contraction is decided per source expression
(``-ffp-contract=on``), never across statements by the backend, so a drone's
arithmetic is the same in every kernel instantiation (lane, tile, work-queue,
mixed or per-model launches, forward and adjoint recompute) and the results do
not depend on the launch configuration.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["cf_api.hip", "cf_step.hip", "cf_rollout.hip", "cf_rollout_bwd.hip", "cf_mppi.hip", "cf_probe.hip"]
# host-only runtime pieces (no device code), compiled by the host compiler
HOST_SOURCES = ["cf_host.cpp"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-I", os.path.join(ROOT, "include")]
LIB = os.path.join(HERE, "libcfsim.so")
ARCH = os.environ.get("CFSIM_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=on",
         "-I", os.path.join(ROOT, "include")]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def cxx() -> str:
    for cand in (os.environ.get("CXX"), shutil.which("g++"), shutil.which("c++")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("no host C++ compiler found")


def _stale(obj: str, src: str) -> bool:
    """An object is stale if it is missing or older than its source or any header."""
    if not os.path.exists(obj):
        return True
    deps = [src] + [os.path.join(HERE, "csrc", f) for f in os.listdir(os.path.join(HERE, "csrc"))
                    if f.endswith((".hpp", ".h"))] + [os.path.join(ROOT, "include", "cfsim.h")]
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, extra_flags=(), incremental: bool = False) -> str:
    """Compile every HIP source and link the shared library; returns its path.
    ``incremental`` recompiles only sources whose object is older than the
    source or a header (the default compiles everything)."""
    cc = hipcc()
    bdir = os.path.join(ROOT, "_build")
    os.makedirs(bdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        if incremental and not extra_flags and not _stale(obj, os.path.join(HERE, "csrc", src)):
            return obj
        cmd = [cc, *FLAGS, *extra_flags, "-c", os.path.join(HERE, "csrc", src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        return obj

    def compile_host(src):
        obj = os.path.join(bdir, src.replace(".cpp", ".o"))
        if incremental and not _stale(obj, os.path.join(HERE, "csrc", src)):
            return obj
        cmd = [cxx(), *HOST_FLAGS, "-c", os.path.join(HERE, "csrc", src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"host compiler failed on {src}:\n{r.stderr}")
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES) + len(HOST_SOURCES)) as ex:
        futs = [ex.submit(compile_one, s) for s in SOURCES] + [ex.submit(compile_host, s) for s in HOST_SOURCES]
        objs = [f.result() for f in futs]
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build(verbose=True, incremental="--incremental" in sys.argv))
