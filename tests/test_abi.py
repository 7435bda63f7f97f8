"""CPU checks of the C ABI: the library loads, exports every symbol declared in
include/wos.h, and rejects invalid descriptors with the documented status codes
before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "wos.h")).read()
    return sorted(set(re.findall(r"\b(wos_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def W():
    from paper_2201_13240_amd import wos
    if not os.path.exists(wos.LIB_PATH):
        pytest.fail("libwos.so is not built (run __graft_entry__.build())")
    wos.lib()
    return wos


def test_exports_every_declared_symbol(W):
    L = W.lib()
    declared = _declared()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(W.EXPORTS) == declared


def test_version_and_struct_sizes(W):
    assert W.lib().wos_version() >= 100
    # wos_options / wos_batch_item layouts as declared in the header
    assert C.sizeof(W.Options) == 80
    assert C.sizeof(W.BatchItem) == 88


def _base_problem():
    from paper_2201_13240_amd import workloads as WL
    return WL.config1()["problems"][0]


def _create(W, prob, **kw):
    with pytest.raises(W.WosError) as e:
        W.Problem(prob, **kw)
    return e.value.status


def test_invalid_descriptors_are_rejected(W):
    from paper_2201_13240_amd import workloads as WL
    p = dict(_base_problem())
    p["epsilon"] = 0.0
    assert _create(W, p) == 1                      # WOS_ERR_INVALID_ARG
    c = WL.field_const(1.0)
    p = WL.make_problem(4, WL.geom_ball([0, 0], 1.0), c, c, c, c, c)
    assert _create(W, p) == 1
    p = dict(_base_problem())
    p["geometry"] = WL.geom_ball([0, 0], -1.0)
    assert _create(W, p) == 2                      # WOS_ERR_GEOMETRY
    p = dict(_base_problem())
    p["geometry"] = WL.geom_polygon(np.zeros((2, 2)))
    assert _create(W, p) == 2
    p = dict(_base_problem())
    p["alpha"] = WL.field_bumps([[0, 0]], [0.0], [1.0])   # zero width
    assert _create(W, p) == 1
    p = dict(_base_problem())
    p["alpha"] = WL.field_manufactured("expcos")   # manufactured only for f and g
    assert _create(W, p) == 1
    c = WL.field_const(1.0)
    p = WL.make_problem(3, WL.geom_trimesh(np.zeros((4, 3)), np.array([[0, 1, 9]] * 4)), c, c, c, c, c)
    assert _create(W, p) == 2                      # triangle index out of range


def test_invalid_sdf_programs_are_rejected(W):
    from paper_2201_13240_amd import workloads as WL
    c = WL.field_const(1.0)
    ball = WL.sdf_row(WL.SDF_UNION, "ball", [0, 0], [1.0])

    def prob(rows, lo=(-1, -1), hi=(1, 1)):
        return WL.make_problem(2, WL.geom_sdf(rows, lo, hi), c, c, c, c, c)

    first_not_union = ball.copy()
    first_not_union[0] = WL.SDF_INTERSECT
    bad_op, bad_shape, bad_radius = ball.copy(), ball.copy(), ball.copy()
    bad_op[0], bad_shape[1], bad_radius[5] = 3, 7, 0.0
    bad_box = WL.sdf_row(WL.SDF_UNION, "box", [0, 0], [1.0, 0.0])
    zero_normal = WL.sdf_row(WL.SDF_INTERSECT, "halfspace", [0, 0], [0.5])
    for rows in ([first_not_union], [ball, bad_op], [bad_shape], [bad_radius], [bad_box], [ball, zero_normal],
                 [ball] * 257, np.zeros((0, 8))):
        assert _create(W, prob(rows)) == 2
    assert _create(W, prob([ball], lo=(1, -1), hi=(1, 1))) == 2   # empty bounding box
    nan = ball.copy()
    nan[2] = np.nan
    assert _create(W, prob([nan])) == 2


def test_solve_rejects_bad_batches_without_device(W):
    o = W.options(walks=0)
    assert W.lib().wos_solve(None, 0, C.byref(o), None) == 1
    items = (W.BatchItem * 1)()
    assert W.lib().wos_solve(items, 1, C.byref(o), None) == 1   # null problem / zero walks
    assert W.lib().wos_last_error()
    # weight-window options are checked before any problem is touched
    for kw in ({"ww_hi": -1.0}, {"ww_hi": 1.5, "variant": 2}, {"ww_hi": 0.4, "russian_roulette": True, "ww_lo": 0.5},
               {"variant": 2, "russian_roulette": True}, {"variant": 3}):
        o = W.options(walks=16, **kw)
        assert W.lib().wos_solve(items, 1, C.byref(o), None) == 1, kw
        assert W.lib().wos_last_error()


def test_tune_cache_rejects_bad_files(W, tmp_path):
    """A malformed tuned-shape file or a path that cannot be read is rejected before any
    shape is set (no device call is made)."""
    bad = tmp_path / "bad.txt"
    bad.write_text("# header\ngfx950 256 0 0 2 2 0 0 100 64\n")      # block size not a multiple of 64
    with pytest.raises(W.WosError) as e:
        W.tune_cache_load(bad)
    assert e.value.status == 1 and "line 2" in str(e.value)
    bad.write_text("gfx950 256 0 0 4 2 0 0 256 64\n")                  # no such dimension
    with pytest.raises(W.WosError):
        W.tune_cache_load(bad)
    with pytest.raises(W.WosError):
        W.tune_cache_load(tmp_path / "missing.txt")
