"""Host logic of the candidate grids (paper_2201_13240_amd/csrc/bvh.cpp), on CPU: a small
C++ driver (tests/host/grid_check.cpp) builds the triangle grid of a perturbed icosphere
and the segment grid of a star polygon with truncated lists, samples points in the cells
and checks the walker's scan against brute force: the scan returns the exact nearest
distance, or, where a truncated list cannot decide, a lower bound of it (the bounded
ball of the walk stays inside the domain, Sec. 3). The triangle grid must not depend on
the number of build threads."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2201_13240_amd import workloads as WL

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2201_13240_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("grid_check")
    exe = str(d / "grid_check")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-pthread", f"-I{CSRC}",
                           os.path.join(HERE, "host", "grid_check.cpp"), os.path.join(CSRC, "bvh.cpp"), "-o", exe])
    return d, exe


def _run(driver, kind, arr):
    d, exe = driver
    path = str(d / f"{kind}.bin")
    np.ascontiguousarray(arr, np.float64).tofile(path)
    out = subprocess.run([exe, kind, path], capture_output=True, text=True, check=True).stdout.split()
    return {out[i]: int(out[i + 1]) for i in range(0, len(out), 2)}


def test_triangle_grid_scan_is_exact_or_a_lower_bound(driver):
    g = WL.icosphere(np.random.default_rng(3), 3, 0.1)
    V, T = np.asarray(g["vertices"]), np.asarray(g["triangles"])
    tris = np.zeros((len(T), 12))
    tris[:, :9] = V[T].reshape(len(T), 9)
    r = _run(driver, "tri", tris)
    assert r["points"] > 1000 and r["exact"] > 0 and r["bounded"] > 0, r
    assert r["bad_exact"] == 0 and r["bad_bound"] == 0, r
    assert r["threads_equal"] == 1


def test_segment_grid_truncated_lists(driver):
    V = np.asarray(WL.star_polygon(np.random.default_rng(5), 512)["vertices"])
    segs = np.c_[V, np.roll(V, -1, axis=0)]
    r = _run(driver, "seg", segs)
    assert r["points"] > 5000 and r["exact"] > 0 and r["bounded"] > 0, r
    assert r["bad_exact"] == 0 and r["bad_bound"] == 0, r


def test_flat_input_keeps_the_grid_bounded(driver):
    """A flat triangle set (degenerate input, zero volume) and a flat zigzag of segments:
    the grids stay within twice their target of 16 cells per primitive."""
    rng = np.random.default_rng(6)
    P = rng.uniform(-1, 1, size=(40, 3, 3))
    P[:, :, 2] = 0.0
    tris = np.zeros((40, 12))
    tris[:, :9] = P.reshape(40, 9)
    r = _run(driver, "tri", tris)
    assert 0 < r["cells"] <= 2 * 16 * 40 and r["bad_exact"] == 0 and r["bad_bound"] == 0, r
    x = np.linspace(-1, 1, 41)
    V = np.c_[x, 1e-9 * (np.arange(41) % 2)]
    segs = np.c_[V[:-1], V[1:]]
    r = _run(driver, "seg", segs)
    assert 0 < r["cells"] <= 2 * 16 * 40 and r["bad_exact"] == 0 and r["bad_bound"] == 0, r
