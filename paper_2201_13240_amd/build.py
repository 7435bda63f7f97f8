"""Builds libwos.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwos.so")
ARCH = os.environ.get("WOS_OFFLOAD_ARCH", "gfx950")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

# The walker is instantiated per precision and dimension in four translation units, which
# compile in parallel with the rest.
SOURCES = ["wos_walker_f64_3d.hip", "wos_walker_f64_2d.hip", "wos_walker_f32_3d.hip", "wos_walker_f32_2d.hip",
           "wos_kernels.hip", "wos_api.cpp", "bvh.cpp"]
HEADERS = ["wos_walker.h", "wos_device.h", "wos_types.h", "wos_launch.h", "bvh.h", "bessel_tables.h",
           "proposal_bound.h"]

# Packed FP32 instructions are disabled for all device code (the compiler forms them
# from scalar float code on its own otherwise).
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics", "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compiles every source (always, `jobs` at a time; 0: up to 8) and links libwos.so
    next to this file."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmd = [hipcc()] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            # host-only C++ (HIP runtime API only)
            cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-c", os.path.join(CSRC, src), "-o", obj,
                   "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include"]
        cmds.append(cmd)
        objs.append(obj)
    jobs = jobs or min(8, os.cpu_count() or 1)
    running, pending = [], list(cmds)
    while pending or running:
        while pending and len(running) < jobs:
            cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((subprocess.Popen(cmd, cwd="/tmp"), cmd))
        proc, cmd = running.pop(0)
        if proc.wait() != 0:
            for q, _ in running:
                q.wait()
            raise subprocess.CalledProcessError(proc.returncode, cmd)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd="/tmp")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
