"""Python binding of libwos.so (the C ABI in include/wos.h): argument marshalling only.

Every step of the walk runs in the HIP kernels of the library. PyTorch provides device
memory and streams. If the library is missing, every entry point raises; there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwos.so")

WOS_FP32, WOS_FP32_COMPENSATED, WOS_FP64, WOS_FP64_FP32_DRAWS = 0, 1, 2, 3
_GEOM = {"ball": 0, "box": 1, "polygon": 2, "trimesh": 3, "sdf": 4}
_BASE = {"none": 0, "fourier": 1, "bumps": 2, "tanh": 3, "tanh_drift": 4, "manufactured": 5}
_TRANSFORM = {"affine": 0, "exp": 1}
_SOLUTION = {"expcos": 1, "quadratic": 2}
PRECISIONS = {"fp32": WOS_FP32, "fp32c": WOS_FP32_COMPENSATED, "fp64": WOS_FP64, "fp64_fp32draws": WOS_FP64_FP32_DRAWS}


class WosError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"wos status {status}: {msg}")
        self.status = status


class GeometryDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad", C.c_int32), ("vertices", C.POINTER(C.c_double)),
                ("n_vertices", C.c_int64), ("triangles", C.POINTER(C.c_int32)), ("n_triangles", C.c_int64),
                ("center", C.c_double * 3), ("radius", C.c_double), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3)]


class FieldDesc(C.Structure):
    _fields_ = [("base", C.c_int32), ("transform", C.c_int32), ("c0", C.c_double), ("c1", C.c_double),
                ("n_terms", C.c_int32), ("solution_id", C.c_int32), ("terms", C.POINTER(C.c_double)),
                ("params", C.c_double * 8)]


class ProblemDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("allow_negative_sigma", C.c_int32), ("geometry", GeometryDesc),
                ("alpha", FieldDesc), ("psi", FieldDesc), ("sigma", FieldDesc), ("source", FieldDesc),
                ("boundary", FieldDesc), ("epsilon", C.c_double), ("sigma_bar", C.c_double),
                ("sigma_bar_grid", C.c_int32), ("pad", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("variant", C.c_int32), ("seed", C.c_uint64),
                ("walks_per_point", C.c_uint64), ("walk_offset", C.c_uint64), ("russian_roulette", C.c_int32),
                ("pad", C.c_int32), ("ww_lo", C.c_double), ("ww_hi", C.c_double), ("max_steps", C.c_uint64),
                ("block_size", C.c_int32), ("tile_walks", C.c_int32), ("workspace_bytes", C.c_uint64)]


class BatchItem(C.Structure):
    _fields_ = [("problem", C.c_void_p), ("points", C.c_void_p), ("n_points", C.c_int64),
                ("problem_index", C.c_uint32), ("pad", C.c_uint32), ("sum", C.c_void_p), ("sum_sq", C.c_void_p),
                ("n_walks", C.c_void_p), ("n_steps", C.c_void_p), ("counters", C.c_void_p),
                ("grad_sum", C.c_void_p), ("grad_sum_sq", C.c_void_p)]


# Every symbol declared in include/wos.h.
EXPORTS = ["wos_last_error", "wos_version", "wos_problem_create", "wos_problem_info", "wos_problem_bvh_info", "wos_problem_grid_info",
           "wos_problem_destroy", "wos_solve", "wos_solve_static", "wos_count_events", "wos_finalize", "wos_finalize_grad", "wos_plan_create", "wos_plan_launch",
           "wos_plan_time", "wos_plan_info", "wos_plan_destroy", "wos_eval_coefficients", "wos_eval_distance", "wos_eval_ball",
           "wos_sample_radius", "wos_philox", "wos_eval_bessel", "wos_eval_offcentred", "wos_classify",
           "wos_problem_setup_times", "wos_plan_setup_times", "wos_tune_cache_save", "wos_tune_cache_load"]

_lib = None


def lib():
    """Loads libwos.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2201_13240_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i64, u64, i32, u32 = C.c_void_p, C.c_int64, C.c_uint64, C.c_int32, C.c_uint32
        dp = C.POINTER(C.c_double)
        L.wos_last_error.restype = C.c_char_p
        L.wos_problem_create.argtypes = [C.POINTER(ProblemDesc), C.c_int, C.POINTER(vp)]
        L.wos_problem_info.argtypes = [vp, dp, dp, dp]
        L.wos_problem_bvh_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i32), C.POINTER(i64)]
        L.wos_problem_grid_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i64)]
        L.wos_problem_destroy.argtypes = [vp]
        L.wos_solve.argtypes = [C.POINTER(BatchItem), i32, C.POINTER(Options), vp]
        L.wos_solve_static.argtypes = [C.POINTER(BatchItem), i32, C.POINTER(Options), vp]
        L.wos_count_events.argtypes = [C.POINTER(BatchItem), i32, C.POINTER(Options), vp, vp]
        L.wos_finalize.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.wos_finalize_grad.argtypes = [vp, vp, vp, i64, i32, vp, vp, vp]
        L.wos_plan_create.argtypes = [C.POINTER(BatchItem), i32, C.POINTER(Options), vp, C.POINTER(vp)]
        L.wos_plan_launch.argtypes = [vp, u64, u64, vp]
        L.wos_plan_time.argtypes = [vp, u64, u64, vp, dp, dp]
        L.wos_plan_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.wos_plan_destroy.argtypes = [vp]
        L.wos_problem_setup_times.argtypes = [vp, dp, dp, dp]
        L.wos_plan_setup_times.argtypes = [vp, dp, dp, C.POINTER(i32)]
        L.wos_tune_cache_save.argtypes = [C.c_char_p, C.POINTER(i32)]
        L.wos_tune_cache_load.argtypes = [C.c_char_p, C.POINTER(i32)]
        L.wos_eval_coefficients.argtypes = [vp, vp, i64, i32, vp, vp]
        L.wos_eval_distance.argtypes = [vp, vp, i64, i32, vp, vp, vp]
        L.wos_eval_ball.argtypes = [i32, i32, vp, i64, vp, vp]
        L.wos_sample_radius.argtypes = [i32, i32, C.c_double, i64, u64, vp, vp, vp]
        L.wos_philox.argtypes = [vp, u64, i64, vp, vp]
        L.wos_eval_bessel.argtypes = [i32, i32, vp, i64, vp, vp]
        L.wos_eval_offcentred.argtypes = [i32, i32, i32, C.c_double, C.c_double, vp, vp, i64, vp, vp]
        L.wos_classify.argtypes = [vp, vp, i64, vp, vp]
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise WosError(status, lib().wos_last_error().decode())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


# ----------------------------------------------------------------------------- problems

class Problem:
    """A compiled problem (wos_problem_create). `prob` is a workload dict (see workloads.py)."""

    def __init__(self, prob: dict, device: int = 0, sigma_bar: float | None = None, sigma_bar_grid: int = 0,
                 allow_negative_sigma: bool = False):
        self._keep = []
        d = ProblemDesc()
        d.dim = prob["dim"]
        d.allow_negative_sigma = int(allow_negative_sigma)
        d.epsilon = prob["epsilon"]
        d.sigma_bar = -1.0 if sigma_bar is None else float(sigma_bar)
        d.sigma_bar_grid = int(sigma_bar_grid)
        self._geometry(d.geometry, prob["geometry"])
        for name in ("alpha", "psi", "sigma", "source", "boundary"):
            self._field(getattr(d, name), prob[name], prob["dim"])
        h = C.c_void_p()
        _check(lib().wos_problem_create(C.byref(d), device, C.byref(h)))
        self.handle = h
        self.dim = prob["dim"]
        self.device = device
        del self._keep

    def _arr(self, a, dtype=np.float64):
        a = np.ascontiguousarray(np.asarray(a, dtype))
        self._keep.append(a)
        return a

    def _geometry(self, G, g):
        G.kind = _GEOM[g["kind"]]
        if g["kind"] == "ball":
            for i, v in enumerate(g["center"]):
                G.center[i] = v
            G.radius = g["radius"]
        elif g["kind"] == "box":
            for i in range(len(g["lo"])):
                G.lo[i] = g["lo"][i]
                G.hi[i] = g["hi"][i]
        elif g["kind"] == "sdf":
            V = self._arr(g["rows"])
            if V.ndim != 2 or V.shape[1] != 8:
                raise ValueError("SDF rows must be [n][8]")
            G.vertices = V.ctypes.data_as(C.POINTER(C.c_double))
            G.n_vertices = V.shape[0]
            for i in range(len(g["lo"])):
                G.lo[i] = g["lo"][i]
                G.hi[i] = g["hi"][i]
        else:
            V = self._arr(g["vertices"])
            G.vertices = V.ctypes.data_as(C.POINTER(C.c_double))
            G.n_vertices = V.shape[0]
            if g["kind"] == "trimesh":
                T = self._arr(g["triangles"], np.int32)
                G.triangles = T.ctypes.data_as(C.POINTER(C.c_int32))
                G.n_triangles = T.shape[0]

    def _field(self, F, f, dim):
        F.base = _BASE[f["base"]]
        F.transform = _TRANSFORM[f["transform"]]
        F.c0 = f["c0"]
        F.c1 = f["c1"]
        b = f["base"]
        if b in ("fourier", "bumps"):
            if b == "fourier":
                packed = np.concatenate([f["k"], f["a"][:, None], f["phi"][:, None]], 1)
            else:
                packed = np.concatenate([f["centers"], f["widths"][:, None], f["amps"][:, None]], 1)
            if packed.shape[1] != dim + 2:
                raise ValueError(f"field terms have {packed.shape[1] - 2} coordinates, problem dim is {dim}")
            P = self._arr(packed)
            F.terms = P.ctypes.data_as(C.POINTER(C.c_double))
            F.n_terms = P.shape[0]
        elif b == "tanh":
            F.params[0], F.params[1], F.params[2] = f["axis"], f["x0"], f["width"]
        elif b == "tanh_drift":
            for i, v in enumerate([f["axis"], f["x0"], f["width"], f["low"], f["high"], f["omega"]]):
                F.params[i] = v
        elif b == "manufactured":
            F.solution_id = _SOLUTION[f["u"]]

    def setup_times(self):
        g, s, u = C.c_double(), C.c_double(), C.c_double()
        _check(lib().wos_problem_setup_times(self.handle, C.byref(g), C.byref(s), C.byref(u)))
        return {"geometry_ms": g.value, "sigma_bar_ms": s.value, "upload_ms": u.value}

    def info(self):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        _check(lib().wos_problem_info(self.handle, C.byref(a), C.byref(b), C.byref(c)))
        return {"sigma_prime_min": a.value, "sigma_prime_max": b.value, "sigma_bar": c.value}

    def bvh_info(self):
        n, dpt, p = C.c_int64(), C.c_int32(), C.c_int64()
        _check(lib().wos_problem_bvh_info(self.handle, C.byref(n), C.byref(dpt), C.byref(p)))
        return {"nodes": n.value, "depth": dpt.value, "prims": p.value}

    def grid_info(self):
        nx, ny, nz, nc = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
        _check(lib().wos_problem_grid_info(self.handle, C.byref(nx), C.byref(ny), C.byref(nz), C.byref(nc)))
        return {"nx": nx.value, "ny": ny.value, "nz": nz.value, "candidates": nc.value}

    @property
    def sigma_bar(self):
        return self.info()["sigma_bar"]

    def close(self):
        if getattr(self, "handle", None):
            lib().wos_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- solving

class Accumulators:
    """Per-point device accumulators of one batch item (added into by every solve)."""

    def __init__(self, n, device="cuda", grad_dim=0):
        """grad_dim > 0 adds gradient sums [n][grad_dim] (supplemental Sec. 2)."""
        import torch
        self.sum = torch.zeros(n, dtype=torch.float64, device=device)
        self.sum_sq = torch.zeros(n, dtype=torch.float64, device=device)
        self.n_walks = torch.zeros(n, dtype=torch.int64, device=device)
        self.n_steps = torch.zeros(n, dtype=torch.int64, device=device)
        self.counters = torch.zeros(4, dtype=torch.int64, device=device)
        self.grad_sum = torch.zeros((n, grad_dim), dtype=torch.float64, device=device) if grad_dim else None
        self.grad_sum_sq = torch.zeros_like(self.grad_sum) if grad_dim else None


VARIANTS = {"alg1": 0, "eq28": 1, "next_flight": 2}


def options(precision="fp32", walks=128, seed=0, walk_offset=0, variant=0, russian_roulette=False, ww_lo=0.5,
            ww_hi=0.0, max_steps=0, block_size=0, tile_walks=0, workspace_bytes=0):
    o = Options()
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    o.seed = seed
    o.walks_per_point = walks
    o.walk_offset = walk_offset
    o.russian_roulette = int(bool(russian_roulette))
    o.ww_lo = ww_lo
    o.ww_hi = ww_hi
    o.max_steps = max_steps
    o.block_size = block_size
    o.tile_walks = tile_walks
    o.workspace_bytes = workspace_bytes
    return o


def _items(entries):
    arr = (BatchItem * len(entries))()
    for i, (prob, pts, acc, pidx) in enumerate(entries):
        assert pts.dtype.__str__() == "torch.float64" and pts.is_contiguous() and pts.shape[1] == prob.dim
        it = arr[i]
        it.problem = prob.handle
        it.points = pts.data_ptr()
        it.n_points = pts.shape[0]
        it.problem_index = pidx
        it.sum = acc.sum.data_ptr()
        it.sum_sq = acc.sum_sq.data_ptr()
        it.n_walks = acc.n_walks.data_ptr()
        it.n_steps = acc.n_steps.data_ptr()
        it.counters = acc.counters.data_ptr()
        if acc.grad_sum is not None:
            assert acc.grad_sum.shape == (pts.shape[0], prob.dim)
            it.grad_sum = acc.grad_sum.data_ptr()
            it.grad_sum_sq = acc.grad_sum_sq.data_ptr()
    return arr


def solve(entries, opt, stream=None):
    """entries: list of (Problem, points[n, dim] float64 cuda tensor, Accumulators, problem_index)."""
    arr = _items(entries)
    _check(lib().wos_solve(arr, len(entries), C.byref(opt), _stream(stream)))


def solve_static(entries, opt, stream=None):
    """As solve, on the library's static scratch array (wos_solve_static): no allocation."""
    arr = _items(entries)
    _check(lib().wos_solve_static(arr, len(entries), C.byref(opt), _stream(stream)))


EVENT_NAMES = ["steps", "bvh_nodes", "prims", "trials", "trials_free", "volume", "exit", "terminal", "gamma_evals",
               "walks", "rr_draws", "ball_large_s", "grid_cells", "lane_iterations", "active_lane_iterations",
               "coefficient_lane_iterations"]


def count_events(entries, opt, stream=None):
    """Same walks as solve() with the event-counting walker; returns {event: count}."""
    import torch
    arr = _items(entries)
    ev = torch.zeros(len(EVENT_NAMES), dtype=torch.int64, device=entries[0][1].device)
    _check(lib().wos_count_events(arr, len(entries), C.byref(opt), _ptr(ev), _stream(stream)))
    torch.cuda.synchronize()
    return dict(zip(EVENT_NAMES, ev.cpu().tolist()))


def finalize(acc, stream=None):
    import torch
    n = acc.sum.shape[0]
    mean = torch.empty(n, dtype=torch.float64, device=acc.sum.device)
    se = torch.empty_like(mean)
    _check(lib().wos_finalize(_ptr(acc.sum), _ptr(acc.sum_sq), _ptr(acc.n_walks), n, _ptr(mean), _ptr(se),
                              _stream(stream)))
    return mean, se


def finalize_grad(acc, stream=None):
    """Mean and standard error of the gradient estimates, [n][dim] each."""
    import torch
    n, dim = acc.grad_sum.shape
    mean = torch.empty((n, dim), dtype=torch.float64, device=acc.grad_sum.device)
    se = torch.empty_like(mean)
    _check(lib().wos_finalize_grad(_ptr(acc.grad_sum), _ptr(acc.grad_sum_sq), _ptr(acc.n_walks), n, dim, _ptr(mean),
                                   _ptr(se), _stream(stream)))
    return mean, se


class Plan:
    """wos_plan: tables, scratch and a captured hipGraph of one batch."""

    def __init__(self, entries, opt, stream=None):
        self._entries = entries   # keep tensors alive
        arr = _items(entries)
        h = C.c_void_p()
        _check(lib().wos_plan_create(arr, len(entries), C.byref(opt), _stream(stream), C.byref(h)))
        self.handle = h

    def launch(self, seed, walk_offset_add=0, stream=None):
        _check(lib().wos_plan_launch(self.handle, seed, walk_offset_add, _stream(stream)))

    def time(self, seed, walk_offset_add=0, stream=None):
        """Runs the plan's work once as separate launches with HIP events around the
        walker; returns (walker_ms, total_ms). Accumulates like launch()."""
        w, t = C.c_double(), C.c_double()
        _check(lib().wos_plan_time(self.handle, seed, walk_offset_add, _stream(stream), C.byref(w), C.byref(t)))
        return w.value, t.value

    def info(self):
        b, t, g, n = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().wos_plan_info(self.handle, C.byref(b), C.byref(t), C.byref(g), C.byref(n)))
        return {"block_size": b.value, "tile_walks": t.value, "grid": g.value, "launches": n.value}

    def setup_times(self):
        b, t, h = C.c_double(), C.c_double(), C.c_int32()
        _check(lib().wos_plan_setup_times(self.handle, C.byref(b), C.byref(t), C.byref(h)))
        return {"build_ms": b.value, "tune_ms": t.value, "tuned_here": bool(h.value)}

    def close(self):
        if getattr(self, "handle", None):
            lib().wos_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_cache_save(path):
    """Writes the launch shapes tuned in this process to `path`; returns the lines written."""
    n = C.c_int32()
    _check(lib().wos_tune_cache_save(str(path).encode(), C.byref(n)))
    return n.value


def tune_cache_load(path):
    """Makes the shapes in `path` the tuned shapes of matching devices; returns how many were set."""
    n = C.c_int32()
    _check(lib().wos_tune_cache_load(str(path).encode(), C.byref(n)))
    return n.value


# ----------------------------------------------------------------------------- diagnostics

def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def eval_coefficients(prob, pts, precision="fp64", stream=None):
    import torch
    out = torch.empty((pts.shape[0], 6), dtype=torch.float64, device=pts.device)
    _check(lib().wos_eval_coefficients(prob.handle, _ptr(pts), pts.shape[0], _prec(precision), _ptr(out),
                                       _stream(stream)))
    return out


def eval_distance(prob, pts, precision="fp64", stream=None):
    import torch
    d = torch.empty(pts.shape[0], dtype=torch.float64, device=pts.device)
    xb = torch.empty_like(pts)
    _check(lib().wos_eval_distance(prob.handle, _ptr(pts), pts.shape[0], _prec(precision), _ptr(d), _ptr(xb),
                                   _stream(stream)))
    return d, xb


def eval_ball(dim, s, precision="fp64", stream=None):
    import torch
    out = torch.empty((s.shape[0], 2), dtype=torch.float64, device=s.device)
    _check(lib().wos_eval_ball(dim, _prec(precision), _ptr(s), s.shape[0], _ptr(out), _stream(stream)))
    return out


def sample_radius(dim, s, n, seed=0, precision="fp64", device="cuda", stream=None):
    import torch
    t = torch.empty(n, dtype=torch.float64, device=device)
    tr = torch.zeros(1, dtype=torch.int64, device=device)
    _check(lib().wos_sample_radius(dim, _prec(precision), float(s), n, seed, _ptr(t), _ptr(tr), _stream(stream)))
    return t, tr


def philox(ctr, key, stream=None):
    import torch
    out = torch.empty_like(ctr)
    _check(lib().wos_philox(_ptr(ctr), key, ctr.shape[0], _ptr(out), _stream(stream)))
    return out


def eval_bessel(which, x, precision="fp64", stream=None):
    import torch
    out = torch.empty_like(x)
    _check(lib().wos_eval_bessel({"i0e": 0, "k0e": 1, "i1e": 2, "k1e": 3}[which], _prec(precision), _ptr(x),
                                 x.shape[0], _ptr(out), _stream(stream)))
    return out


def eval_offcentred(which, dim, R, sigma_bar, u, v, precision="fp64", stream=None):
    """Next-flight kernels: which 'green' gives G(x, y)|B| (u = x - c, v = y - c), 'poisson'
    gives P(x, z)|dB| (v = z - c on the sphere). u, v: device float64 [n][dim]."""
    import torch
    assert u.shape == v.shape and u.shape[1] == dim and u.dtype == torch.float64 and v.dtype == torch.float64
    out = torch.empty(u.shape[0], dtype=torch.float64, device=u.device)
    _check(lib().wos_eval_offcentred({"green": 0, "poisson": 1}[which], dim, _prec(precision), float(R),
                                     float(sigma_bar), _ptr(u.contiguous()), _ptr(v.contiguous()), u.shape[0],
                                     _ptr(out), _stream(stream)))
    return out


def classify(prob, pts, stream=None):
    import torch
    out = torch.empty(pts.shape[0], dtype=torch.int8, device=pts.device)
    _check(lib().wos_classify(prob.handle, _ptr(pts), pts.shape[0], _ptr(out), _stream(stream)))
    return out
