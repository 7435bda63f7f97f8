"""The host builders of the candidate grids and the BVH (paper_2201_13240_amd/csrc/bvh.cpp)
under the compilers' sanitizers, on CPU: the grid check driver (tests/host/grid_check.cpp)
is built with AddressSanitizer and UndefinedBehaviorSanitizer, and separately with
ThreadSanitizer, and runs the same inputs as tests/test_host_grid.py. The triangle grid
is built with 4 threads and with 1 there, so ThreadSanitizer sees the threaded build
(parts filled by worker threads, exceptions carried back, the merge after the joins).
Any report ends the driver with a non-zero status (halt_on_error)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2201_13240_amd import workloads as WL

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2201_13240_amd", "csrc")

SANITIZERS = {
    "address_undefined": (["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
                          {"ASAN_OPTIONS": "halt_on_error=1:detect_leaks=1:verify_asan_link_order=0",
                           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}),
    "thread": (["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"}),
}


def _inputs():
    g = WL.icosphere(np.random.default_rng(3), 3, 0.1)
    V, T = np.asarray(g["vertices"]), np.asarray(g["triangles"])
    tris = np.zeros((len(T), 12))
    tris[:, :9] = V[T].reshape(len(T), 9)
    S = np.asarray(WL.star_polygon(np.random.default_rng(5), 512)["vertices"])
    segs = np.c_[S, np.roll(S, -1, axis=0)]
    rng = np.random.default_rng(6)
    P = rng.uniform(-1, 1, size=(40, 3, 3))
    P[:, :, 2] = 0.0
    flat = np.zeros((40, 12))
    flat[:, :9] = P.reshape(40, 9)
    return [("tri", tris), ("seg", segs), ("tri", flat)]


@pytest.mark.parametrize("name", sorted(SANITIZERS))
def test_grid_builders_under_sanitizer(name, tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    flags, env_add = SANITIZERS[name]
    exe = str(tmp_path / f"grid_check_{name}")
    cmd = ["g++", "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-pthread", *flags, f"-I{CSRC}",
           os.path.join(HERE, "host", "grid_check.cpp"), os.path.join(CSRC, "bvh.cpp"), "-o", exe]
    subprocess.check_call(cmd)
    env = dict(os.environ)
    env.update(env_add)
    for i, (kind, arr) in enumerate(_inputs()):
        path = str(tmp_path / f"in{i}.bin")
        np.ascontiguousarray(arr, np.float64).tofile(path)
        r = subprocess.run([exe, kind, path], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, f"{name} {kind}: status {r.returncode}\n{r.stderr[-4000:]}"
        assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
        out = r.stdout.split()
        res = {out[k]: int(out[k + 1]) for k in range(0, len(out), 2)}
        assert res["bad_exact"] == 0 and res["bad_bound"] == 0, res
        if kind == "tri":
            assert res["threads_equal"] == 1, res
