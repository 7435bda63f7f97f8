"""Seeded synthetic problem generators.

This module only *describes* problems: domain geometry, the parameters of the
coefficient/source/boundary fields, and query points. It contains none of the
Monte Carlo method's arithmetic (no change of variables, no Green's functions,
no walks), so both the FP64 CPU oracle and the GPU library can consume its
output without sharing any computation.

A problem is a plain dict::

    {"dim": 2 | 3,
     "geometry": {...},               # see the geometry constructors below
     "alpha": field, "psi": field,    # diffusion alpha(x) > 0; drift omega = alpha * grad(psi)
     "sigma": field,                  # absorption sigma(x) >= 0
     "source": field, "boundary": field,
     "epsilon": float}                # epsilon-shell width

and a field is ``{"base": kind, "transform": "affine" | "exp", "c0", "c1", ...}``
whose value is ``c0 + c1*B(x)`` (affine) or ``exp(c0 + c1*B(x))`` (exp), with the
base B one of

* ``none``        B = 0
* ``fourier``     B = sum_j a_j cos(2*pi*k_j.x + phi_j)     (k integer vectors)
* ``bumps``       B = sum_j amp_j exp(-|x - c_j|^2 / (2 w_j^2))
* ``tanh``        B = (1 + tanh((x[axis] - x0) / width)) / 2
* ``tanh_drift``  B = psi(x) with alpha(x) psi'(x) = omega along ``axis``, for
                  alpha = low + (high - low) * (1 + tanh((x[axis]-x0)/width)) / 2
                  and psi(x0) = 0 (closed form; used for a constant drift)
* ``manufactured`` (source / boundary only) the data of a manufactured solution
                  u named by ``u``: the boundary field is u itself, the source
                  field is f = -div(alpha grad u) - omega.grad u + sigma u
                  evaluated with the problem's own alpha, psi and sigma.

Manufactured solutions: ``expcos`` u = exp(x0) cos(x1) (harmonic in 2D and 3D),
``quadratic`` u = 1 + x0^2 + x0*x1 / 2 (Laplacian 2).

The five workload families follow the paper's problem statement (Sec. 1, eq. 1:
Dirichlet problem for div(alpha grad u) + omega.grad u - sigma u = -f) with
synthetic data in place of the paper's scenes, which are not available.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "field_const", "field_fourier", "field_bumps", "field_tanh", "field_tanh_drift",
    "field_manufactured", "random_fourier", "random_bumps",
    "geom_ball", "geom_box", "geom_polygon", "geom_trimesh", "star_polygon", "icosphere",
    "grid_points", "inside_mask", "sample_inside", "make_problem",
    "config1", "config2", "config3", "config4", "config5", "CONFIG_BUILDERS",
]


# ----------------------------------------------------------------------------- fields

def _field(base, transform="affine", c0=0.0, c1=1.0, **params):
    f = {"base": base, "transform": transform, "c0": float(c0), "c1": float(c1)}
    f.update(params)
    return f


def field_const(value):
    """Constant field: affine transform of the zero base."""
    return _field("none", "affine", c0=value, c1=0.0)


def field_fourier(k, a, phi, transform="affine", c0=0.0, c1=1.0):
    k = np.asarray(k, dtype=np.float64)
    return _field("fourier", transform, c0, c1, k=k, a=np.asarray(a, np.float64).ravel(),
                  phi=np.asarray(phi, np.float64).ravel())


def field_bumps(centers, widths, amps, transform="affine", c0=0.0, c1=1.0):
    return _field("bumps", transform, c0, c1, centers=np.asarray(centers, np.float64),
                  widths=np.asarray(widths, np.float64).ravel(),
                  amps=np.asarray(amps, np.float64).ravel())


def field_tanh(axis, x0, width, low, high):
    """low + (high-low) * (1 + tanh((x[axis]-x0)/width)) / 2."""
    return _field("tanh", "affine", c0=low, c1=high - low, axis=int(axis), x0=float(x0),
                  width=float(width))


def field_tanh_drift(axis, x0, width, low, high, omega):
    """Drift potential psi for omega = alpha*grad(psi) = omega*e_axis with a tanh-step alpha."""
    return _field("tanh_drift", "affine", c0=0.0, c1=1.0, axis=int(axis), x0=float(x0),
                  width=float(width), low=float(low), high=float(high), omega=float(omega))


def field_manufactured(u_name):
    return _field("manufactured", "affine", c0=0.0, c1=1.0, u=str(u_name))


def random_fourier(rng, n_modes, dim, amp, kmax=3):
    """n_modes random modes, integer wave vectors in [-kmax, kmax]^dim \\ {0},
    coefficients c ~ U(-1,1) rescaled so that sum|a| = amp (hence |B| <= amp),
    phases ~ U[0, 2pi)."""
    k = np.zeros((n_modes, dim))
    for j in range(n_modes):
        while True:
            kk = rng.integers(-kmax, kmax + 1, size=dim)
            if np.any(kk != 0):
                break
        k[j] = kk
    c = rng.uniform(-1.0, 1.0, size=n_modes)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    a = amp * c / np.sum(np.abs(c))
    return k, a, phi


def random_bumps(rng, n, lo, hi, width_range, amp_range):
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    centers = rng.uniform(lo, hi, size=(n, lo.size))
    widths = np.exp(rng.uniform(math.log(width_range[0]), math.log(width_range[1]), size=n))
    amps = rng.uniform(amp_range[0], amp_range[1], size=n)
    return centers, widths, amps


# ----------------------------------------------------------------------------- geometry

def geom_ball(center, radius):
    return {"kind": "ball", "center": np.asarray(center, np.float64), "radius": float(radius)}


def geom_box(lo, hi):
    return {"kind": "box", "lo": np.asarray(lo, np.float64), "hi": np.asarray(hi, np.float64)}


def geom_polygon(vertices, star=False):
    """Closed counter-clockwise polygon; segment j joins vertex j and j+1 (mod n).
    ``star`` marks polygons whose vertex j lies at angle 2*pi*j/n around the origin."""
    v = np.ascontiguousarray(np.asarray(vertices, np.float64))
    return {"kind": "polygon", "vertices": v, "star": bool(star)}


def geom_trimesh(vertices, triangles, star=None):
    """Closed triangle mesh with outward (counter-clockwise seen from outside) faces.
    ``star`` optionally holds the unit vertex directions of a mesh that is star-shaped
    about the origin (used only for fast inside classification)."""
    g = {"kind": "trimesh",
         "vertices": np.ascontiguousarray(np.asarray(vertices, np.float64)),
         "triangles": np.ascontiguousarray(np.asarray(triangles, np.int32))}
    if star is not None:
        g["star_dirs"] = np.ascontiguousarray(np.asarray(star, np.float64))
    return g


SDF_UNION, SDF_INTERSECT, SDF_SUBTRACT = 0, 1, 2


def sdf_row(op, shape, center, params):
    """One CSG row (op, shape, c0, c1, c2, p0, p1, p2): shape "ball" (params = [radius]),
    "box" (half extents) or "halfspace" (center holds the normal n, params = [offset];
    the inside is x.n < offset)."""
    r = np.zeros(8)
    r[0] = op
    r[1] = {"ball": 0, "box": 1, "halfspace": 2}[shape]
    c = np.asarray(center, np.float64)
    r[2:2 + c.size] = c
    p = np.asarray(params, np.float64)
    r[5:5 + p.size] = p
    return r


def geom_sdf(rows, lo, hi):
    """Domain given by a list of CSG rows on signed distance fields (Sec. 7.2); lo/hi is
    a box holding the domain."""
    return {"kind": "sdf", "rows": np.ascontiguousarray(np.asarray(rows, np.float64).reshape(-1, 8)),
            "lo": np.asarray(lo, np.float64), "hi": np.asarray(hi, np.float64)}


def _sdf_member(rows, pts):
    """Set membership of the CSG list by boolean set operations on the primitives'
    interiors (harness helper for sampling query points)."""
    dim = pts.shape[1]
    inside = np.zeros(pts.shape[0], bool)
    for r in rows:
        op, shape = int(r[0]), int(r[1])
        c = r[2:2 + dim]
        if shape == 0:
            m = ((pts - c) ** 2).sum(1) < r[5] ** 2
        elif shape == 1:
            m = np.all(np.abs(pts - c) < r[5:5 + dim], axis=1)
        else:
            m = pts @ c < r[5]
        if op == SDF_UNION:
            inside |= m
        elif op == SDF_INTERSECT:
            inside &= m
        else:
            inside &= ~m
    return inside


def star_polygon(rng, n_edges=256, n_modes=8, amp=0.3):
    """Vertices at theta_j = 2*pi*j/n, radius 1 + amp*P(theta_j) with P a sum of
    n_modes Fourier modes (N(0,1) coefficients) scaled so max_j |P(theta_j)| = 1."""
    a = rng.standard_normal(n_modes)
    b = rng.standard_normal(n_modes)
    th = 2.0 * math.pi * np.arange(n_edges) / n_edges
    m = np.arange(1, n_modes + 1)
    P = (a[None, :] * np.cos(np.outer(th, m)) + b[None, :] * np.sin(np.outer(th, m))).sum(1)
    P /= np.max(np.abs(P))
    rho = 1.0 + amp * P
    return geom_polygon(np.stack([rho * np.cos(th), rho * np.sin(th)], 1), star=True)


def _icosphere_unit(subdiv):
    t = (1.0 + math.sqrt(5.0)) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
             (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(v, np.float64) / np.linalg.norm(v) for v in verts]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
             (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
             (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        cache = {}
        new_faces = []

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = verts[i] + verts[j]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        for (a, b, c) in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    V = np.array(verts)
    F = np.array(faces, np.int32)
    # orient outward
    n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    flip = (n * V[F].mean(1)).sum(1) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def icosphere(rng, subdiv=5, noise=0.1):
    """Icosphere with ``subdiv`` subdivisions, each vertex scaled radially by 1+U(-noise, noise).
    Radial scaling keeps the mesh star-shaped about the origin (no self-intersections)."""
    V, F = _icosphere_unit(subdiv)
    scale = 1.0 + rng.uniform(-noise, noise, size=V.shape[0])
    return geom_trimesh(V * scale[:, None], F, star=V)


# ----------------------------------------------------------------------------- points

def grid_points(n, lo, hi, dim=2, z=None):
    """Cell-centred n x n grid over [lo, hi]^2 (row-major, x fastest); in 3D the
    points lie on the plane x2 = z."""
    h = (hi - lo) / n
    c = lo + h * (np.arange(n) + 0.5)
    X, Y = np.meshgrid(c, c, indexing="xy")
    pts = np.stack([X.ravel(), Y.ravel()], 1)
    if dim == 3:
        pts = np.concatenate([pts, np.full((pts.shape[0], 1), 0.0 if z is None else z)], 1)
    return np.ascontiguousarray(pts)


def _polygon_inside_crossing(V, pts, chunk=4096):
    n = V.shape[0]
    a = V
    b = np.roll(V, -1, axis=0)
    inside = np.zeros(pts.shape[0], bool)
    for s in range(0, pts.shape[0], chunk):
        p = pts[s:s + chunk]
        px, py = p[:, :1], p[:, 1:2]
        ay, by = a[None, :, 1], b[None, :, 1]
        ax, bx = a[None, :, 0], b[None, :, 0]
        cond = (ay > py) != (by > py)
        with np.errstate(divide="ignore", invalid="ignore"):
            xint = ax + (py - ay) * (bx - ax) / (by - ay)
        cross = cond & (px < xint)
        inside[s:s + chunk] = (cross.sum(1) % 2) == 1
    del n
    return inside


def _star_polygon_inside(V, pts):
    n = V.shape[0]
    th = np.mod(np.arctan2(pts[:, 1], pts[:, 0]), 2.0 * math.pi)
    j = np.minimum((th / (2.0 * math.pi) * n).astype(np.int64), n - 1)
    a = V[j]
    b = V[(j + 1) % n]
    # side of the directed edge a->b (CCW polygon: inside is to the left)
    cr = (b[:, 0] - a[:, 0]) * (pts[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (pts[:, 0] - a[:, 0])
    return cr > 0.0


def _star_mesh_inside(g, pts):
    from scipy.spatial import cKDTree
    V = g["vertices"]
    F = g["triangles"]
    D = g["star_dirs"]
    cen = D[F].mean(1)
    cen /= np.linalg.norm(cen, axis=1, keepdims=True)
    tree = cKDTree(cen)
    r = np.linalg.norm(pts, axis=1)
    d = pts / np.maximum(r, 1e-300)[:, None]
    _, idx = tree.query(d, k=8)
    inside = np.zeros(pts.shape[0], bool)
    found = np.zeros(pts.shape[0], bool)
    for c in range(idx.shape[1]):
        f = F[idx[:, c]]
        d0, d1, d2 = D[f[:, 0]], D[f[:, 1]], D[f[:, 2]]
        s0 = (d * np.cross(d0, d1)).sum(1)
        s1 = (d * np.cross(d1, d2)).sum(1)
        s2 = (d * np.cross(d2, d0)).sum(1)
        ok = (s0 >= -1e-14) & (s1 >= -1e-14) & (s2 >= -1e-14) & ~found
        P0, P1, P2 = V[f[:, 0]], V[f[:, 1]], V[f[:, 2]]
        nrm = np.cross(P1 - P0, P2 - P0)
        t = (nrm * P0).sum(1) / (nrm * d).sum(1)
        inside = np.where(ok, r < t, inside)
        found |= ok
    if not np.all(found):
        raise RuntimeError("star mesh classification failed for some directions")
    return inside | (r == 0.0)


def inside_mask(geometry, pts):
    """Strict interior test of query points (harness helper, not part of the method)."""
    pts = np.asarray(pts, np.float64)
    k = geometry["kind"]
    if k == "ball":
        return np.linalg.norm(pts - geometry["center"][None, :], axis=1) < geometry["radius"]
    if k == "box":
        return np.all((pts > geometry["lo"][None, :]) & (pts < geometry["hi"][None, :]), axis=1)
    if k == "polygon":
        if geometry.get("star", False):
            return _star_polygon_inside(geometry["vertices"], pts)
        return _polygon_inside_crossing(geometry["vertices"], pts)
    if k == "sdf":
        return _sdf_member(geometry["rows"], pts)
    if k == "trimesh":
        if "star_dirs" not in geometry:
            raise ValueError("inside_mask: only star-shaped meshes are supported")
        return _star_mesh_inside(geometry, pts)
    raise ValueError(k)


def _bbox(geometry, dim):
    k = geometry["kind"]
    if k == "ball":
        c, r = geometry["center"], geometry["radius"]
        return c - r, c + r
    if k in ("box", "sdf"):
        return geometry["lo"], geometry["hi"]
    V = geometry["vertices"]
    return V.min(0), V.max(0)


def sample_inside(rng, geometry, dim, n):
    """n points uniform in the interior (rejection from the bounding box)."""
    lo, hi = _bbox(geometry, dim)
    out = []
    have = 0
    while have < n:
        p = rng.uniform(lo, hi, size=(max(2 * (n - have), 64), dim))
        p = p[inside_mask(geometry, p)]
        out.append(p)
        have += p.shape[0]
    return np.ascontiguousarray(np.concatenate(out)[:n])


def make_problem(dim, geometry, alpha, psi, sigma, source, boundary, epsilon=1e-3):
    return {"dim": int(dim), "geometry": geometry, "alpha": alpha, "psi": psi, "sigma": sigma,
            "source": source, "boundary": boundary, "epsilon": float(epsilon)}


# ----------------------------------------------------------------------------- workloads

def config1(n_grid=32):
    """Unit disk; alpha = 1 + 0.5 sin(2 pi x) sin(2 pi y), omega = 0, sigma = 1;
    manufactured u = exp(x) cos(y); cell-centred n_grid^2 grid on [-1,1]^2 inside the disk."""
    # 0.5 sin(2pi x) sin(2pi y) = 0.25 cos(2pi(x - y)) - 0.25 cos(2pi(x + y))
    alpha = field_fourier([[1.0, -1.0], [1.0, 1.0]], [0.25, -0.25], [0.0, 0.0],
                          transform="affine", c0=1.0, c1=1.0)
    prob = make_problem(2, geom_ball([0.0, 0.0], 1.0), alpha, field_const(0.0), field_const(1.0),
                        field_manufactured("expcos"), field_manufactured("expcos"), 1e-3)
    pts = grid_points(n_grid, -1.0, 1.0)
    pts = pts[inside_mask(prob["geometry"], pts)]
    return {"name": "disk-manufactured", "problems": [prob], "points": [pts], "walks": 128,
            "exact": "expcos"}


def _polygon_problem(rng, geometry, n_alpha=16, n_psi=16, n_sigma=16, drift=True):
    lo, hi = _bbox(geometry, 2)
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
    k, a, phi = random_fourier(rng, n_alpha, 2, 0.5)
    alpha = field_fourier(k, a, phi, transform="exp")
    if drift:
        k2, a2, phi2 = random_fourier(rng, n_psi, 2, 1.0)
        # rescale psi so that max over the interior of |omega| = |alpha grad psi| is 1
        g = grid_points(128, float(lo.min()), float(hi.max()))
        g = g[inside_mask(geometry, g)]
        arg = 2 * math.pi * g @ k2.T + phi2[None, :]
        grad = -(np.sin(arg) * a2[None, :]) @ (2 * math.pi * k2)
        Fa = np.cos(2 * math.pi * g @ k.T + phi[None, :]) @ a
        om = np.exp(Fa) * np.linalg.norm(grad, axis=1)
        psi = field_fourier(k2, a2 / om.max(), phi2)
    else:
        psi = field_const(0.0)
    k3, a3, phi3 = random_fourier(rng, n_sigma, 2, 1.0)
    sigma = field_fourier(k3, a3, phi3, transform="affine", c0=5.0, c1=5.0)
    c, w, am = random_bumps(rng, 8, lo, hi, (0.05, 0.3), (-10.0, 10.0))
    source = field_bumps(c, w, am)
    c, w, am = random_bumps(rng, 8, lo, hi, (0.1, 0.5), (-1.0, 1.0))
    boundary = field_bumps(c, w, am)
    return make_problem(2, geometry, alpha, psi, sigma, source, boundary, 1e-3)


def config2(n_grid=512):
    """Star polygon (256 edges, radius 1 +- 0.3 from 8 modes); alpha = exp(16 modes, amp 0.5);
    omega = alpha grad psi with |omega| <= 1; sigma = 5 (1 + 16 modes) in [0, 10];
    f, g = 8 Gaussian bumps; n_grid^2 grid on [-1.3, 1.3]^2 inside the polygon; 1024 walks."""
    rng = np.random.default_rng(2000)
    geometry = star_polygon(rng, 256, 8, 0.3)
    prob = _polygon_problem(rng, geometry)
    pts = grid_points(n_grid, -1.3, 1.3)
    pts = pts[inside_mask(geometry, pts)]
    return {"name": "star-polygon-256", "problems": [prob], "points": [pts], "walks": 1024}


def config3(n_grid=1024, subdiv=5):
    """Perturbed icosphere (20480 triangles at subdiv 5, radial noise 0.1); alpha = exp(32 modes,
    amp 0.5); sigma = 5 (1 + 32 modes); omega = 0; f, g = 8 bumps; n_grid^2 points on z = 0."""
    rng = np.random.default_rng(3000)
    geometry = icosphere(rng, subdiv, 0.1)
    lo, hi = geometry["vertices"].min(0), geometry["vertices"].max(0)
    k, a, phi = random_fourier(rng, 32, 3, 0.5)
    alpha = field_fourier(k, a, phi, transform="exp")
    k3, a3, phi3 = random_fourier(rng, 32, 3, 1.0)
    sigma = field_fourier(k3, a3, phi3, transform="affine", c0=5.0, c1=5.0)
    c, w, am = random_bumps(rng, 8, lo, hi, (0.05, 0.3), (-10.0, 10.0))
    source = field_bumps(c, w, am)
    c, w, am = random_bumps(rng, 8, lo, hi, (0.1, 0.5), (-1.0, 1.0))
    boundary = field_bumps(c, w, am)
    prob = make_problem(3, geometry, alpha, field_const(0.0), sigma, source, boundary, 1e-3)
    pts = grid_points(n_grid, -1.1, 1.1, dim=3, z=0.0)
    pts = pts[inside_mask(geometry, pts)]
    return {"name": "icosphere-20480", "problems": [prob], "points": [pts], "walks": 256}


def config4(n_problems=64, points_scale=1.0, min_edges=16, max_edges=4096,
            min_pts=1024, max_pts=262144):
    """Batch of star-polygon problems: log-uniform edge counts and query counts."""
    problems, points = [], []
    for i in range(n_problems):
        rng = np.random.default_rng(4000 + i)
        E = int(round(math.exp(rng.uniform(math.log(min_edges), math.log(max_edges)))))
        Q = int(round(math.exp(rng.uniform(math.log(min_pts), math.log(max_pts)))))
        Q = max(1, int(round(Q * points_scale)))
        geometry = star_polygon(rng, E, 8, 0.3)
        problems.append(_polygon_problem(rng, geometry))
        points.append(sample_inside(rng, geometry, 2, Q))
    return {"name": "batched-64-polygons", "problems": problems, "points": points, "walks": 512}


def csg_scatter(rng, n_disks=24, n_boxes=8):
    """CSG list of a square [-1, 1]^2 with n_disks round and n_boxes rectangular holes
    scattered at uniform positions (radii U(0.03, 0.1), half sides U(0.03, 0.08)), in
    the manner of Sec. 7.2's edited SDF scenes."""
    rows = [sdf_row(SDF_UNION, "box", [0.0, 0.0], [1.0, 1.0])]
    for _ in range(n_disks):
        rows.append(sdf_row(SDF_SUBTRACT, "ball", rng.uniform(-0.9, 0.9, 2), [rng.uniform(0.03, 0.1)]))
    for _ in range(n_boxes):
        rows.append(sdf_row(SDF_SUBTRACT, "box", rng.uniform(-0.9, 0.9, 2), rng.uniform(0.03, 0.08, 2)))
    return geom_sdf(rows, [-1.0, -1.0], [1.0, 1.0])


def config6(n_grid=256):
    """CSG scene (csg_scatter: square with 24 round and 8 rectangular holes) with the star
    polygon's kind of fields (alpha = exp(16 modes), drift |omega| <= 1, sigma in [0, 10],
    8-bump f and g); n_grid^2 grid on [-1, 1]^2 inside; 256 walks."""
    rng = np.random.default_rng(6000)
    geometry = csg_scatter(rng)
    prob = _polygon_problem(rng, geometry)
    pts = grid_points(n_grid, -1.0, 1.0)
    pts = pts[inside_mask(geometry, pts)]
    return {"name": "csg-scatter-32", "problems": [prob], "points": [pts], "walks": 256}


def config5(n_grid=256):
    """Unit square; alpha = 1 + 99 (1 + tanh((x - 0.5)/0.01))/2; sigma = 100 + 450 (1 + 16 modes)
    in [100, 1000]; omega = (50, 0); f, g = 8 bumps; n_grid^2 cell-centred points."""
    rng = np.random.default_rng(5000)
    geometry = geom_box([0.0, 0.0], [1.0, 1.0])
    alpha = field_tanh(0, 0.5, 0.01, 1.0, 100.0)
    psi = field_tanh_drift(0, 0.5, 0.01, 1.0, 100.0, 50.0)
    k3, a3, phi3 = random_fourier(rng, 16, 2, 1.0)
    sigma = field_fourier(k3, a3, phi3, transform="affine", c0=550.0, c1=450.0)
    c, w, am = random_bumps(rng, 8, [0, 0], [1, 1], (0.05, 0.3), (-10.0, 10.0))
    source = field_bumps(c, w, am)
    c, w, am = random_bumps(rng, 8, [0, 0], [1, 1], (0.1, 0.5), (-1.0, 1.0))
    boundary = field_bumps(c, w, am)
    prob = make_problem(2, geometry, alpha, psi, sigma, source, boundary, 1e-3)
    pts = grid_points(n_grid, 0.0, 1.0)
    return {"name": "high-contrast-square", "problems": [prob], "points": [pts], "walks": 64}


def config7(n_grid=256):
    """Unit disk; alpha = 1, omega = 0, sigma = 2 + 1.5 (16 random Fourier modes) in
    [0.5, 3.5], so that sigma' = sigma >= 0 and every ball has s = R sqrt(sigma_bar) < 2;
    f, g = 8 bumps; n_grid^2 cell-centred points on [-1, 1]^2 inside. The regime in which
    the next-flight walk (Sec. 5.2) has finite variance."""
    rng = np.random.default_rng(7000)
    geometry = geom_ball([0.0, 0.0], 1.0)
    k3, a3, phi3 = random_fourier(rng, 16, 2, 1.0)
    sigma = field_fourier(k3, a3, phi3, transform="affine", c0=2.0, c1=1.5)
    c, w, am = random_bumps(rng, 8, [-1, -1], [1, 1], (0.05, 0.3), (-10.0, 10.0))
    source = field_bumps(c, w, am)
    c, w, am = random_bumps(rng, 8, [-1, -1], [1, 1], (0.1, 0.5), (-1.0, 1.0))
    boundary = field_bumps(c, w, am)
    prob = make_problem(2, geometry, field_const(1.0), field_const(0.0), sigma, source, boundary, 1e-3)
    pts = grid_points(n_grid, -1.0, 1.0)
    pts = pts[inside_mask(geometry, pts)]
    return {"name": "screened-disk", "problems": [prob], "points": [pts], "walks": 256}


def manufactured(prob, u="expcos", epsilon=1e-4):
    """The same geometry and coefficient fields (alpha, drift potential, sigma) with the
    source and boundary data of a manufactured solution u (eq. 1 gives f from u and the
    problem's own alpha, psi and sigma; g = u), so that the solution is known exactly on a
    workload of any shape. The epsilon shell is narrowed (1e-4) so that its O(epsilon)
    bias stays far below the Monte Carlo error of long runs."""
    q = dict(prob)
    q["source"] = field_manufactured(u)
    q["boundary"] = field_manufactured(u)
    q["epsilon"] = epsilon
    return q


CONFIG_BUILDERS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}
