// C ABI of the walk-on-spheres library: problem compilation (fields, geometry, BVH,
// sigma_bar), solves, plans with hipGraph replay, and diagnostics.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/wos.h"
#include "bvh.h"
#include "wos_launch.h"
#include "wos_types.h"

using namespace wos;

namespace {

thread_local std::string g_error;

wos_status fail(wos_status s, const std::string& msg) {
  g_error = msg;
  return s;
}

// Runs f and turns a C++ exception (a failed host allocation, a thread that could not
// start) into a status, so that none crosses the C ABI.
template <typename F>
wos_status guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(WOS_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(WOS_ERR_INTERNAL, std::string("host error: ") + e.what());
  } catch (...) {
    return fail(WOS_ERR_INTERNAL, "unknown host error");
  }
}

#define WOS_HIP(call)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(e_ == hipErrorOutOfMemory ? WOS_ERR_OUT_OF_MEMORY : WOS_ERR_DEVICE,       \
                  std::string(#call) + ": " + hipGetErrorString(e_));                       \
  } while (0)

constexpr double kTwoPi = 6.283185307179586476925286766559;

// Bump allocator over one host staging buffer mirrored by one device allocation.
struct Blob {
  std::vector<unsigned char> host;
  size_t alloc(size_t bytes, size_t align = 256) {
    size_t off = (host.size() + align - 1) / align * align;
    host.resize(off + bytes);
    return off;
  }
};

}  // namespace

struct wos_problem {
  int device = 0;
  int dim = 2;
  int geom = 0;
  double epsilon = 0;
  double sigma_bar = 0;
  double sp_min = NAN, sp_max = NAN;
  void* dmem = nullptr;
  size_t off32 = 0, off64 = 0;
  int64_t n_nodes = 0, n_prims = 0;
  int32_t depth = 0;
  int32_t grid_nx = 0, grid_ny = 0, grid_nz = 0;
  int64_t grid_candidates = 0;
  std::vector<unsigned char> staging;  // host copy of the device blob
  double geometry_ms = 0, sigma_bar_ms = 0, upload_ms = 0;   // set-up time (host wall clock)
  const void* d32() const { return (const unsigned char*)dmem + off32; }
  const void* d64() const { return (const unsigned char*)dmem + off64; }
};

namespace {

// ------------------------------------------------------------------ fields

wos_status check_field(const wos_field_desc& f, int dim, const char* name, bool source_or_boundary) {
  if (f.transform != WOS_TRANSFORM_AFFINE && f.transform != WOS_TRANSFORM_EXP)
    return fail(WOS_ERR_INVALID_ARG, std::string(name) + ": unknown transform");
  switch (f.base) {
    case WOS_FIELD_NONE: break;
    case WOS_FIELD_FOURIER:
    case WOS_FIELD_BUMPS:
      if (f.n_terms < 0 || (f.n_terms > 0 && !f.terms))
        return fail(WOS_ERR_INVALID_ARG, std::string(name) + ": terms missing");
      for (int j = 0; j < f.n_terms; ++j)
        for (int k = 0; k < dim + 2; ++k)
          if (!std::isfinite(f.terms[j * (dim + 2) + k]))
            return fail(WOS_ERR_INVALID_ARG, std::string(name) + ": non-finite term");
      if (f.base == WOS_FIELD_BUMPS)
        for (int j = 0; j < f.n_terms; ++j)
          if (!(f.terms[j * (dim + 2) + dim] > 0)) return fail(WOS_ERR_INVALID_ARG, std::string(name) + ": bump width <= 0");
      break;
    case WOS_FIELD_TANH:
    case WOS_FIELD_TANH_DRIFT: {
      const int ax = (int)f.params[0];
      if (ax < 0 || ax >= dim || !(f.params[2] > 0))
        return fail(WOS_ERR_INVALID_ARG, std::string(name) + ": bad tanh axis or width");
      if (f.base == WOS_FIELD_TANH_DRIFT && (!(f.params[3] > 0) || !(f.params[4] > 0) || f.params[3] == f.params[4] ||
                                            f.transform != WOS_TRANSFORM_AFFINE || f.c0 != 0 || f.c1 != 1))
        return fail(WOS_ERR_INVALID_ARG, std::string(name) + ": tanh_drift needs 0 < low != high, affine (0, 1)");
      break;
    }
    case WOS_FIELD_MANUFACTURED:
      if (!source_or_boundary) return fail(WOS_ERR_INVALID_ARG, std::string(name) + ": manufactured only for f and g");
      if (f.solution_id != 1 && f.solution_id != 2) return fail(WOS_ERR_INVALID_ARG, std::string(name) + ": unknown solution");
      break;
    default: return fail(WOS_ERR_INVALID_ARG, std::string(name) + ": unknown base");
  }
  if (!std::isfinite(f.c0) || !std::isfinite(f.c1)) return fail(WOS_ERR_INVALID_ARG, std::string(name) + ": bad c0/c1");
  return WOS_OK;
}

template <typename T>
std::vector<T> field_terms(const wos_field_desc& f, int dim) {
  std::vector<T> out((size_t)std::max(f.n_terms, 0) * kTermStride, (T)0);
  for (int j = 0; j < f.n_terms; ++j) {
    const double* t = f.terms + j * (dim + 2);
    T* o = out.data() + (size_t)j * kTermStride;
    if (f.base == WOS_FIELD_FOURIER) {
      // wave vector in cycles per unit length: the device takes the sine and cosine of
      // k.x in revolutions
      double k2 = 0;
      for (int i = 0; i < dim; ++i) {
        o[i] = (T)t[i];
        k2 += (kTwoPi * t[i]) * (kTwoPi * t[i]);
      }
      const double a = t[dim], phi = t[dim + 1];
      o[3] = (T)(a * std::cos(phi));
      o[4] = (T)(a * std::sin(phi));
      o[5] = (T)k2;
      // the phase in revolutions, reduced to [-1/2, 1/2]
      const double rev = phi / kTwoPi;
      o[6] = (T)a;
      o[7] = (T)(rev - std::nearbyint(rev));
    } else {  // bumps
      for (int i = 0; i < dim; ++i) o[i] = (T)t[i];
      const double w = t[dim];
      o[3] = (T)(1.4426950408889634074 / (2 * w * w));   // log2(e) / (2 w^2): the device takes exp2
      o[4] = (T)t[dim + 1];
      o[5] = (T)(1.0 / (w * w));
    }
  }
  return out;
}

template <typename T>
DevField<T> field_header(const wos_field_desc& f) {
  DevField<T> d;
  std::memset(&d, 0, sizeof(d));
  d.base = f.base;
  d.transform = f.transform;
  d.n = (f.base == WOS_FIELD_FOURIER || f.base == WOS_FIELD_BUMPS) ? f.n_terms : 0;
  d.sol = f.solution_id;
  d.c0 = (T)f.c0;
  d.c1 = (T)f.c1;
  if (f.base == WOS_FIELD_TANH) {
    d.prm[0] = (T)f.params[0];
    d.prm[1] = (T)f.params[1];
    d.prm[2] = (T)(1.0 / f.params[2]);
  } else if (f.base == WOS_FIELD_TANH_DRIFT) {
    const double w = f.params[2], lo = f.params[3], hi = f.params[4], om = f.params[5];
    const double A = 0.5 * (lo + hi), B = 0.5 * (hi - lo);
    d.prm[0] = (T)f.params[0];
    d.prm[1] = (T)f.params[1];
    d.prm[2] = (T)(1.0 / w);
    d.prm[3] = (T)A;
    d.prm[4] = (T)B;
    d.prm[5] = (T)(om * w / (A * A - B * B));
    d.prm[6] = (T)std::log(A);
    d.prm[7] = (T)om;
  }
  return d;
}

// ------------------------------------------------------------------ geometry

struct HostGeometry {
  int kind = 0;
  int64_t n_prims = 0;
  std::vector<double> prims64;       // leaf order, device layout
  std::vector<float> prims32;
  BvhTopology topo;
  std::vector<double> bounds64;      // node child bounds
  std::vector<float> bounds32;
  SegmentGrid grid;                  // polygons and triangle meshes
  double grid_margin = 0;            // rounding margin of the candidate lists
};

wos_status build_geometry(const wos_problem_desc& d, HostGeometry& g) {
  const wos_geometry_desc& G = d.geometry;
  const int dim = d.dim;
  g.kind = G.kind;
  if (G.kind == WOS_GEOM_BALL) {
    if (!(G.radius > 0) || !std::isfinite(G.radius)) return fail(WOS_ERR_GEOMETRY, "ball radius must be > 0");
    return WOS_OK;
  }
  if (G.kind == WOS_GEOM_BOX) {
    for (int i = 0; i < dim; ++i)
      if (!(G.hi[i] > G.lo[i])) return fail(WOS_ERR_GEOMETRY, "box needs lo < hi");
    return WOS_OK;
  }
  if (G.kind == WOS_GEOM_SDF) {
    // CSG operation list (Sec. 7.2), stored as it is given, with half-space normals made
    // unit length so that every primitive field is a true signed distance
    if (!G.vertices || G.n_vertices < 1 || G.n_vertices > WOS_SDF_MAX_OPS)
      return fail(WOS_ERR_GEOMETRY, "SDF needs 1..WOS_SDF_MAX_OPS operation rows");
    for (int i = 0; i < dim; ++i)
      if (!(G.hi[i] > G.lo[i]) || !std::isfinite(G.lo[i]) || !std::isfinite(G.hi[i]))
        return fail(WOS_ERR_GEOMETRY, "SDF needs a bounding box lo < hi");
    const int64_t n = G.n_vertices;
    g.n_prims = n;
    g.prims64.assign((size_t)n * kSdfStride, 0.0);
    for (int64_t j = 0; j < n; ++j) {
      const double* r = G.vertices + kSdfStride * j;
      for (int k = 0; k < kSdfStride; ++k)
        if (!std::isfinite(r[k])) return fail(WOS_ERR_GEOMETRY, "non-finite SDF row");
      const double op = r[0], shape = r[1];
      if (!(op == 0 || op == 1 || op == 2)) return fail(WOS_ERR_GEOMETRY, "SDF op must be 0, 1 or 2");
      if (j == 0 && op != 0) return fail(WOS_ERR_GEOMETRY, "the first SDF row must be a union");
      double* o = g.prims64.data() + kSdfStride * j;
      o[0] = op;
      o[1] = shape;
      for (int i = 0; i < dim; ++i) o[2 + i] = r[2 + i];
      if (shape == 0) {
        if (!(r[5] > 0)) return fail(WOS_ERR_GEOMETRY, "SDF ball radius must be > 0");
        o[5] = r[5];
      } else if (shape == 1) {
        for (int i = 0; i < dim; ++i) {
          if (!(r[5 + i] > 0)) return fail(WOS_ERR_GEOMETRY, "SDF box half extents must be > 0");
          o[5 + i] = r[5 + i];
        }
      } else if (shape == 2) {
        double nn = 0;
        for (int i = 0; i < dim; ++i) nn += r[2 + i] * r[2 + i];
        nn = std::sqrt(nn);
        if (!(nn > 0)) return fail(WOS_ERR_GEOMETRY, "SDF half-space normal must be nonzero");
        for (int i = 0; i < dim; ++i) o[2 + i] = r[2 + i] / nn;
        o[5] = r[5] / nn;
      } else {
        return fail(WOS_ERR_GEOMETRY, "SDF shape must be 0, 1 or 2");
      }
    }
    g.prims32.resize(g.prims64.size());
    for (size_t k = 0; k < g.prims64.size(); ++k) g.prims32[k] = (float)g.prims64[k];
    return WOS_OK;
  }
  const int pdim = dim;
  int stride;
  std::vector<double> lo, hi, cen, raw;
  if (G.kind == WOS_GEOM_POLYGON) {
    if (dim != 2) return fail(WOS_ERR_GEOMETRY, "polygons are 2D");
    if (!G.vertices || G.n_vertices < 3) return fail(WOS_ERR_GEOMETRY, "polygon needs >= 3 vertices");
    const int64_t n = G.n_vertices;
    g.n_prims = n;
    stride = 4;
    raw.resize((size_t)n * 4);
    for (int64_t j = 0; j < n; ++j) {
      const double* a = G.vertices + 2 * j;
      const double* b = G.vertices + 2 * ((j + 1) % n);
      if (!std::isfinite(a[0]) || !std::isfinite(a[1])) return fail(WOS_ERR_GEOMETRY, "non-finite vertex");
      raw[4 * j] = a[0];
      raw[4 * j + 1] = a[1];
      raw[4 * j + 2] = b[0];
      raw[4 * j + 3] = b[1];
    }
  } else if (G.kind == WOS_GEOM_TRIMESH) {
    if (dim != 3) return fail(WOS_ERR_GEOMETRY, "triangle meshes are 3D");
    if (!G.vertices || !G.triangles || G.n_vertices < 4 || G.n_triangles < 4)
      return fail(WOS_ERR_GEOMETRY, "mesh needs >= 4 vertices and triangles");
    const int64_t n = G.n_triangles;
    g.n_prims = n;
    stride = 12;
    raw.assign((size_t)n * 12, 0.0);
    for (int64_t j = 0; j < n; ++j)
      for (int v = 0; v < 3; ++v) {
        const int32_t vi = G.triangles[3 * j + v];
        if (vi < 0 || vi >= G.n_vertices) return fail(WOS_ERR_GEOMETRY, "triangle index out of range");
        for (int k = 0; k < 3; ++k) {
          const double c = G.vertices[3 * (int64_t)vi + k];
          if (!std::isfinite(c)) return fail(WOS_ERR_GEOMETRY, "non-finite vertex");
          raw[12 * j + 3 * v + k] = c;
        }
      }
  } else {
    return fail(WOS_ERR_INVALID_ARG, "unknown geometry kind");
  }
  if (g.n_prims >= (1ll << 27)) return fail(WOS_ERR_GEOMETRY, "too many primitives");
  const int64_t n = g.n_prims;
  const int nv = G.kind == WOS_GEOM_POLYGON ? 2 : 3;
  lo.resize((size_t)n * pdim);
  hi.resize((size_t)n * pdim);
  cen.resize((size_t)n * pdim);
  for (int64_t j = 0; j < n; ++j)
    for (int k = 0; k < pdim; ++k) {
      double mn = 1e300, mx = -1e300, s = 0;
      for (int v = 0; v < nv; ++v) {
        const double c = raw[(size_t)stride * j + pdim * v + k];
        mn = std::min(mn, c);
        mx = std::max(mx, c);
        s += c;
      }
      lo[j * pdim + k] = mn;
      hi[j * pdim + k] = mx;
      cen[j * pdim + k] = s / nv;
    }
  g.topo = build_bvh(lo, hi, cen, pdim, n, 4);
  if (g.topo.depth >= 46) return fail(WOS_ERR_GEOMETRY, "BVH too deep");
  g.prims64.resize((size_t)n * stride);
  g.prims32.resize((size_t)n * stride);
  std::vector<double> plo64((size_t)n * pdim), phi64((size_t)n * pdim);
  std::vector<float> plo32((size_t)n * pdim), phi32((size_t)n * pdim);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t src = g.topo.order[i];
    for (int k = 0; k < stride; ++k) {
      g.prims64[(size_t)stride * i + k] = raw[(size_t)stride * src + k];
      g.prims32[(size_t)stride * i + k] = (float)raw[(size_t)stride * src + k];
    }
    for (int k = 0; k < pdim; ++k) {
      double mn = 1e300, mx = -1e300;
      float mnf = 3e38f, mxf = -3e38f;
      for (int v = 0; v < nv; ++v) {
        mn = std::min(mn, g.prims64[(size_t)stride * i + pdim * v + k]);
        mx = std::max(mx, g.prims64[(size_t)stride * i + pdim * v + k]);
        mnf = std::min(mnf, g.prims32[(size_t)stride * i + pdim * v + k]);
        mxf = std::max(mxf, g.prims32[(size_t)stride * i + pdim * v + k]);
      }
      plo64[i * pdim + k] = mn;
      phi64[i * pdim + k] = mx;
      plo32[i * pdim + k] = mnf;
      phi32[i * pdim + k] = mxf;
    }
  }
  bvh_child_bounds<double>(g.topo, plo64, phi64, pdim, g.bounds64);
  bvh_child_bounds<float>(g.topo, plo32, phi32, pdim, g.bounds32);
  if (G.kind == WOS_GEOM_POLYGON) {
    // about 64 cells per segment, between 64^2 and 2^20 cells, lists of up to 32
    // candidates (longer ones, deep inside large polygons, keep their 16 nearest); the
    // margin covers FP32 rounding of the query point and of the cell index
    double scale = 0;
    for (double c : g.prims64) scale = std::max(scale, std::fabs(c));
    const int64_t target = std::min<int64_t>(1 << 20, std::max<int64_t>(4096, 64 * n));
    g.grid_margin = 4e-6 * (scale + 1.0);
    g.grid = build_segment_grid(g.prims64, n, g.topo, g.bounds64, target, g.grid_margin, kPolygonCellMax,
                                kPolygonDeepList);
  } else {
    // meshes: about 128 cells per triangle, between 32^3 and 2^21 cells, lists of the 6
    // candidates nearest to the cell centre (on the perturbed icosphere these walks ran
    // 1.5x faster than with 64 cells per triangle and lists of 16: shorter scans, and few
    // queries left to the BVH)
    double scale = 0;
    for (double c : g.prims64) scale = std::max(scale, std::fabs(c));
    const int64_t target = std::min<int64_t>(1 << 21, std::max<int64_t>(32768, 128 * n));
    g.grid_margin = 4e-6 * (scale + 1.0);
    const int threads = (int)std::min<unsigned>(16, std::max<unsigned>(1, std::thread::hardware_concurrency()));
    g.grid = build_triangle_grid(g.prims64, n, g.topo, g.bounds64, target, g.grid_margin, kMeshCellList, threads);
  }
  return WOS_OK;
}

template <typename T>
const std::vector<T>& pick(const std::vector<float>& f, const std::vector<double>& d) {
  if constexpr (sizeof(T) == 4) {
    (void)d;
    return f;
  } else {
    (void)f;
    return d;
  }
}

template <typename T, int DIM>
void write_nodes(const HostGeometry& g, const std::vector<T>& bounds, BvhNode<T, DIM>* out) {
  const size_t nn = g.topo.child.size() / 2;
  for (size_t i = 0; i < nn; ++i) {
    const T* b = bounds.data() + i * 4 * DIM;
    for (int s = 0; s < 2; ++s)
      for (int k = 0; k < DIM; ++k) {
        out[i].lo[s][k] = b[s * DIM + k];
        out[i].hi[s][k] = b[2 * DIM + s * DIM + k];
      }
    out[i].child[0] = g.topo.child[2 * i];
    out[i].child[1] = g.topo.child[2 * i + 1];
  }
}

// Lays out DevProblem<T> and everything it points to inside the blob; pointers are
// device addresses (dbase + offset), patched once the device allocation exists.
template <typename T>
size_t layout_problem(Blob& blob, const wos_problem_desc& d, const HostGeometry& g, std::vector<std::pair<size_t, size_t>>& ptr_fixups) {
  const size_t off_struct = blob.alloc(sizeof(DevProblem<T>));
  DevProblem<T> P;
  std::memset(&P, 0, sizeof(P));
  P.dim = d.dim;
  P.epsilon = (T)d.epsilon;
  const wos_field_desc* fd[5] = {&d.alpha, &d.psi, &d.sigma, &d.source, &d.boundary};
  DevField<T>* fp[5] = {&P.alpha, &P.psi, &P.sigma, &P.source, &P.boundary};
  size_t term_off[5] = {0, 0, 0, 0, 0};
  for (int k = 0; k < 5; ++k) {
    *fp[k] = field_header<T>(*fd[k]);
    if (fp[k]->n > 0) {
      const std::vector<T> terms = field_terms<T>(*fd[k], d.dim);
      term_off[k] = blob.alloc(terms.size() * sizeof(T));
      std::memcpy(blob.host.data() + term_off[k], terms.data(), terms.size() * sizeof(T));
    }
  }
  // dense trigonometric table for 2D Fourier fields with integer wave vectors |k_i| <= 3,
  // used when it replaces enough per-mode sin/cos evaluations
  if (d.dim == 2) {
    const wos_field_desc* slots[3] = {&d.alpha, &d.psi, &d.sigma};
    int eligible = 0, modes = 0;
    for (int sidx = 0; sidx < 3; ++sidx) {
      const wos_field_desc& f = *slots[sidx];
      if (f.base != WOS_FIELD_FOURIER || f.n_terms <= 0) continue;
      bool ok = true;
      for (int j = 0; j < f.n_terms && ok; ++j)
        for (int i = 0; i < 2; ++i) {
          const double k = f.terms[j * 4 + i];
          if (k != std::floor(k) || std::fabs(k) > kSpecK) ok = false;
        }
      if (ok) {
        eligible |= 1 << sidx;
        modes += f.n_terms;
      }
    }
    if (eligible && modes >= 12) {
      // complex coefficients per slot, in double
      double re[3][kSpecK + 1][kSpecRow] = {}, im[3][kSpecK + 1][kSpecRow] = {}, c[3] = {0, 0, 0};
      for (int sidx = 0; sidx < 3; ++sidx) {
        if (!(eligible & (1 << sidx))) continue;
        const wos_field_desc& f = *slots[sidx];
        for (int j = 0; j < f.n_terms; ++j) {
          int kx = (int)f.terms[j * 4], ky = (int)f.terms[j * 4 + 1];
          const double a = f.terms[j * 4 + 2], phi = f.terms[j * 4 + 3];
          double cr = a * std::cos(phi), ci = a * std::sin(phi);
          if (kx == 0 && ky == 0) {
            c[sidx] += cr;
            continue;
          }
          if (kx < 0 || (kx == 0 && ky < 0)) {  // cos is even: use -k and the conjugate
            kx = -kx;
            ky = -ky;
            ci = -ci;
          }
          re[sidx][kx][ky + kSpecK] += cr;
          im[sidx][kx][ky + kSpecK] += ci;
        }
      }
      // With alpha = exp(c0 + c1 B_alpha) and an affine (or absent) psi, gamma =
      // (ln alpha + psi)/2 is itself a trigonometric sum: slot 0 then holds gamma (the
      // only slot whose derivatives are needed) and slot 1 the base of alpha.
      const bool psi_none = d.psi.base == WOS_FIELD_NONE && d.psi.transform == WOS_TRANSFORM_AFFINE;
      const bool merge = (eligible & 1) && d.alpha.transform == WOS_TRANSFORM_EXP &&
                         (psi_none || ((eligible & 2) && d.psi.transform == WOS_TRANSFORM_AFFINE));
      P.spectral = eligible;
      if (merge) {
        const double a0 = d.alpha.c0, a1 = d.alpha.c1;
        const double p0 = d.psi.c0, p1 = psi_none ? 0.0 : d.psi.c1;
        double gre[kSpecK + 1][kSpecRow], gim[kSpecK + 1][kSpecRow];
        for (int kx = 0; kx <= kSpecK; ++kx)
          for (int j = 0; j < kSpecRow; ++j) {
            gre[kx][j] = 0.5 * (a1 * re[0][kx][j] + p1 * re[1][kx][j]);
            gim[kx][j] = 0.5 * (a1 * im[0][kx][j] + p1 * im[1][kx][j]);
          }
        const double gc = 0.5 * (a0 + a1 * c[0] + p0 + p1 * c[1]);
        for (int kx = 0; kx <= kSpecK; ++kx)
          for (int j = 0; j < kSpecRow; ++j) {
            re[1][kx][j] = re[0][kx][j];
            im[1][kx][j] = im[0][kx][j];
            re[0][kx][j] = gre[kx][j];
            im[0][kx][j] = gim[kx][j];
          }
        c[1] = c[0];
        c[0] = gc;
        P.spectral = eligible | 1 | 2 | kSpecGammaMerged;
      }
      // product form: Re(C e^{i(A + B)}) = cr cA cB - cr sA sB - ci sA cB - ci cA sB with
      // A = 2 pi kx x, B = 2 pi ky y; cos(ky y) and sin(ky y) are the basis functions of
      // |ky| (the sine with the sign of ky). Basis index: 0 for the constant, 2n - 1 for
      // cos(2 pi n .), 2n for sin(2 pi n .).
      const double two_pi = 6.283185307179586476925286766559;
      for (int sidx = 0; sidx < 3; ++sidx) {
        if (!(P.spectral & (1 << sidx))) continue;
        double M[kSpecRow][kSpecRow] = {};
        M[0][0] = c[sidx];
        for (int kx = 0; kx <= kSpecK; ++kx)
          for (int j = 0; j < kSpecRow; ++j) {
            const double cr = re[sidx][kx][j], ci = im[sidx][kx][j];
            if (cr == 0.0 && ci == 0.0) continue;
            const int ky = j - kSpecK, ay = std::abs(ky);
            const double sg = ky < 0 ? -1.0 : 1.0;
            const int ac = kx ? 2 * kx - 1 : 0, as = 2 * kx, bc = ay ? 2 * ay - 1 : 0, bs = 2 * ay;
            M[ac][bc] += cr;
            if (kx && ay) M[as][bs] -= cr * sg;
            if (kx) M[as][bc] -= ci;
            if (ay) M[ac][bs] -= ci * sg;
          }
        for (int a = 0; a < kSpecRow; ++a) {
          double My[kSpecRow] = {}, Myy[kSpecRow] = {};
          for (int n = 1; n <= kSpecK; ++n) {
            const double w = two_pi * n;
            My[2 * n] = -w * M[a][2 * n - 1];      // d/dy cos = -w sin
            My[2 * n - 1] = w * M[a][2 * n];       // d/dy sin = w cos
            Myy[2 * n - 1] = -w * w * M[a][2 * n - 1];
            Myy[2 * n] = -w * w * M[a][2 * n];
          }
          for (int b = 0; b < kSpecRow; ++b) {
            P.spec.m[a][sidx][0][b] = (T)M[a][b];
            P.spec.m[a][sidx][1][b] = (T)My[b];
            P.spec.m[a][sidx][2][b] = (T)Myy[b];
          }
        }
      }
    }
  }
  DevGeometry<T>& G = P.geom;
  G.kind = d.geometry.kind;
  for (int i = 0; i < 3; ++i) {
    G.center[i] = (T)d.geometry.center[i];
    G.lo[i] = (T)d.geometry.lo[i];
    G.hi[i] = (T)d.geometry.hi[i];
  }
  G.radius = (T)d.geometry.radius;
  size_t node_off = 0, prim_off = 0, grid_start_off = 0, grid_prim_off = 0, grid_seg_off = 0, grid_dc_off = 0;
  if (g.n_prims > 0) {
    G.n_prims = (int32_t)g.n_prims;
    G.n_nodes = (int32_t)(g.topo.child.size() / 2);
    G.root = g.topo.root;
    G.depth = g.topo.depth;
    const std::vector<T>& prims = pick<T>(g.prims32, g.prims64);
    prim_off = blob.alloc(prims.size() * sizeof(T));
    std::memcpy(blob.host.data() + prim_off, prims.data(), prims.size() * sizeof(T));
    const std::vector<T>& bounds = pick<T>(g.bounds32, g.bounds64);
    if (d.dim == 2) {
      node_off = blob.alloc(std::max<size_t>(1, G.n_nodes) * sizeof(BvhNode<T, 2>));
      write_nodes<T, 2>(g, bounds, (BvhNode<T, 2>*)(blob.host.data() + node_off));
      if (g.grid.nx > 0) {
        G.grid_nx = g.grid.nx;
        G.grid_ny = g.grid.ny;
        G.grid_lo[0] = (T)g.grid.lo[0];
        G.grid_lo[1] = (T)g.grid.lo[1];
        G.grid_inv_h = (T)(1.0 / g.grid.h);
        G.grid_h = (T)g.grid.h;
        G.grid_lb_min = (T)std::max(0.25 * g.grid.h, 2.0 * d.epsilon);
        const size_t nc = g.grid.prim.size();
        const size_t ncell = g.grid.start.size() - 1;
        grid_start_off = blob.alloc(ncell * sizeof(CellRec<T>));
        CellRec<T>* cells = (CellRec<T>*)(blob.host.data() + grid_start_off);
        for (size_t c = 0; c < ncell; ++c) {
          CellRec<T> r;
          std::memset(&r, 0, sizeof(r));
          r.start = g.grid.start[c];
          r.count = g.grid.start[c + 1] - g.grid.start[c];
          r.tail = std::isfinite(g.grid.tail[c]) ? (T)(g.grid.tail[c] - g.grid_margin)
                                                 : std::numeric_limits<T>::infinity();
          // inline entries beyond the list repeat its last candidate: their distance equals
          // that candidate's, so they never replace it as the nearest (strict comparison)
          for (uint32_t k = 0; r.count > 0 && k < (uint32_t)kCellInline; ++k) {
            const uint32_t kk = std::min<uint32_t>(k, r.count - 1);
            const double* sg = g.prims64.data() + (size_t)g.grid.prim[r.start + kk] * 4;
            r.seg[k][0] = (T)sg[0];
            r.seg[k][1] = (T)sg[1];
            r.seg[k][2] = (T)(sg[2] - sg[0]);
            r.seg[k][3] = (T)(sg[3] - sg[1]);
            const double ex = (double)r.seg[k][2], ey = (double)r.seg[k][3], l2 = ex * ex + ey * ey;
            r.inv_len2[k] = l2 > 0 ? (T)(1.0 / l2) : (T)0;
          }
          cells[c] = r;
        }
        grid_prim_off = blob.alloc(std::max<size_t>(nc, 1) * sizeof(int32_t));
        std::memcpy(blob.host.data() + grid_prim_off, g.grid.prim.data(), nc * sizeof(int32_t));
        grid_seg_off = blob.alloc(std::max<size_t>(nc, 1) * 4 * sizeof(T));
        T* cs = (T*)(blob.host.data() + grid_seg_off);
        for (size_t k = 0; k < nc; ++k)
          for (int c = 0; c < 4; ++c) cs[4 * k + c] = prims[(size_t)g.grid.prim[k] * 4 + c];
        grid_dc_off = blob.alloc(std::max<size_t>(nc, 1) * sizeof(T));
        T* dc = (T*)(blob.host.data() + grid_dc_off);
        for (size_t k = 0; k < nc; ++k) dc[k] = (T)(g.grid.dc[k] - g.grid_margin);
      }
    } else {
      node_off = blob.alloc(std::max<size_t>(1, G.n_nodes) * sizeof(BvhNode<T, 3>));
      write_nodes<T, 3>(g, bounds, (BvhNode<T, 3>*)(blob.host.data() + node_off));
      if (g.grid.nx > 0) {
        G.grid_nx = g.grid.nx;
        G.grid_ny = g.grid.ny;
        G.grid_nz = g.grid.nz;
        for (int k = 0; k < 3; ++k) G.grid_lo[k] = (T)g.grid.lo[k];
        G.grid_inv_h = (T)(1.0 / g.grid.h);
        G.grid_h = (T)g.grid.h;
        // a quarter cell: lower, the walks make more steps; higher, more queries take the
        // BVH, which a whole wave then waits for (h: 11% slower on the perturbed icosphere)
        G.grid_lb_min = (T)std::max(0.25 * g.grid.h, 2.0 * d.epsilon);
        const size_t nc = g.grid.prim.size();
        const size_t ncell = g.grid.start.size() - 1;
        grid_start_off = blob.alloc(ncell * sizeof(MeshCell<T>));
        MeshCell<T>* cells = (MeshCell<T>*)(blob.host.data() + grid_start_off);
        for (size_t c = 0; c < ncell; ++c) {
          std::memset(&cells[c], 0, sizeof(MeshCell<T>));
          cells[c].start = g.grid.start[c];
          cells[c].count = g.grid.start[c + 1] - g.grid.start[c];
          cells[c].tail = std::isfinite(g.grid.tail[c]) ? (T)(g.grid.tail[c] - g.grid_margin)
                                                        : std::numeric_limits<T>::infinity();
        }
        grid_prim_off = blob.alloc(std::max<size_t>(nc, 1) * sizeof(int32_t));
        std::memcpy(blob.host.data() + grid_prim_off, g.grid.prim.data(), nc * sizeof(int32_t));
        grid_dc_off = blob.alloc(std::max<size_t>(nc, 1) * sizeof(T));
        T* dc = (T*)(blob.host.data() + grid_dc_off);
        for (size_t k = 0; k < nc; ++k) dc[k] = (T)(g.grid.dc[k] - g.grid_margin);
      }
    }
  }
  std::memcpy(blob.host.data() + off_struct, &P, sizeof(P));
  // record pointer fields (location in blob, target offset) to patch with the device base
  auto field_ptr_loc = [&](int k) {
    const size_t base = off_struct + ((const unsigned char*)fp[k] - (const unsigned char*)&P);
    return base + offsetof(DevField<T>, terms);
  };
  for (int k = 0; k < 5; ++k)
    if (fp[k]->n > 0) ptr_fixups.push_back({field_ptr_loc(k), term_off[k]});
  if (g.n_prims > 0) {
    const size_t gbase = off_struct + offsetof(DevProblem<T>, geom);
    ptr_fixups.push_back({gbase + offsetof(DevGeometry<T>, nodes), node_off});
    ptr_fixups.push_back({gbase + offsetof(DevGeometry<T>, prims), prim_off});
    if (g.grid.nx > 0) {
      ptr_fixups.push_back({gbase + offsetof(DevGeometry<T>, cells), grid_start_off});
      ptr_fixups.push_back({gbase + offsetof(DevGeometry<T>, cell_prim), grid_prim_off});
      if (grid_seg_off) ptr_fixups.push_back({gbase + offsetof(DevGeometry<T>, cell_segs), grid_seg_off});
      ptr_fixups.push_back({gbase + offsetof(DevGeometry<T>, cell_dc), grid_dc_off});
    }
  }
  return off_struct;
}

template <typename T>
void set_sigma_bar(unsigned char* host_struct, double sb) {
  DevProblem<T>* P = (DevProblem<T>*)host_struct;
  P->sigma_bar = (T)sb;
  P->inv_sigma_bar = sb > 0 ? (T)(1.0 / sb) : (T)0;
  P->sqrt_sigma_bar = (T)std::sqrt(std::max(sb, 0.0));
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

const char* wos_last_error(void) { return g_error.c_str(); }

int wos_version(void) { return 100; }

static wos_status problem_create_impl(const wos_problem_desc* desc, int device, wos_problem** out) {
  if (!desc || !out) return fail(WOS_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  const wos_problem_desc& d = *desc;
  if (d.dim != 2 && d.dim != 3) return fail(WOS_ERR_INVALID_ARG, "dim must be 2 or 3");
  if (!(d.epsilon > 0) || !std::isfinite(d.epsilon)) return fail(WOS_ERR_INVALID_ARG, "epsilon must be > 0");
  if (std::isnan(d.sigma_bar)) return fail(WOS_ERR_INVALID_ARG, "sigma_bar is NaN");
  if (d.geometry.kind < 0 || d.geometry.kind > 4) return fail(WOS_ERR_INVALID_ARG, "unknown geometry kind");
  const char* names[5] = {"alpha", "psi", "sigma", "source", "boundary"};
  const wos_field_desc* fds[5] = {&d.alpha, &d.psi, &d.sigma, &d.source, &d.boundary};
  for (int k = 0; k < 5; ++k) {
    const wos_status s = check_field(*fds[k], d.dim, names[k], k >= 3);
    if (s != WOS_OK) return s;
  }
  using clock = std::chrono::steady_clock;
  auto ms_since = [](clock::time_point t) { return std::chrono::duration<double, std::milli>(clock::now() - t).count(); };
  clock::time_point t0 = clock::now();
  HostGeometry g;
  {
    const wos_status s = build_geometry(d, g);
    if (s != WOS_OK) return s;
  }
  const double geometry_ms = ms_since(t0);
  t0 = clock::now();
  int n_dev = 0;
  WOS_HIP(hipGetDeviceCount(&n_dev));
  if (device < 0 || device >= n_dev) return fail(WOS_ERR_DEVICE, "no such device");
  WOS_HIP(hipSetDevice(device));

  wos_problem* p = new wos_problem();
  p->device = device;
  p->dim = d.dim;
  p->geom = d.geometry.kind;
  p->epsilon = d.epsilon;
  p->n_prims = g.n_prims;
  p->n_nodes = (int64_t)(g.topo.child.size() / 2);
  p->depth = g.topo.depth;
  p->grid_nx = g.grid.nx;
  p->grid_ny = g.grid.ny;
  p->grid_nz = g.grid.nx > 0 ? g.grid.nz : 0;
  p->grid_candidates = (int64_t)g.grid.prim.size();
  Blob blob;
  std::vector<std::pair<size_t, size_t>> fix;
  p->off32 = layout_problem<float>(blob, d, g, fix);
  p->off64 = layout_problem<double>(blob, d, g, fix);
  hipError_t e = hipMalloc(&p->dmem, blob.host.size());
  if (e != hipSuccess) {
    delete p;
    return fail(e == hipErrorOutOfMemory ? WOS_ERR_OUT_OF_MEMORY : WOS_ERR_DEVICE, "hipMalloc of problem data failed");
  }
  for (const auto& f : fix) {
    const uint64_t addr = (uint64_t)p->dmem + f.second;
    std::memcpy(blob.host.data() + f.first, &addr, sizeof(addr));
  }
  p->staging = blob.host;
  auto upload = [&]() { return hipMemcpy(p->dmem, p->staging.data(), p->staging.size(), hipMemcpyHostToDevice); };
  if ((e = upload()) != hipSuccess) {
    (void)hipFree(p->dmem);
    delete p;
    return fail(WOS_ERR_DEVICE, "upload of problem data failed");
  }
  const double upload_ms = ms_since(t0);
  t0 = clock::now();
  // sample alpha, sigma and sigma' in FP64 over a grid of the bounding box (interior points)
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  if (g.kind == WOS_GEOM_BALL) {
    for (int i = 0; i < d.dim; ++i) {
      lo[i] = d.geometry.center[i] - d.geometry.radius;
      hi[i] = d.geometry.center[i] + d.geometry.radius;
    }
  } else if (g.kind == WOS_GEOM_BOX || g.kind == WOS_GEOM_SDF) {
    for (int i = 0; i < d.dim; ++i) {
      lo[i] = d.geometry.lo[i];
      hi[i] = d.geometry.hi[i];
    }
  } else {
    for (int i = 0; i < d.dim; ++i) {
      lo[i] = 1e300;
      hi[i] = -1e300;
    }
    for (int64_t v = 0; v < d.geometry.n_vertices; ++v)
      for (int i = 0; i < d.dim; ++i) {
        lo[i] = std::min(lo[i], d.geometry.vertices[v * d.dim + i]);
        hi[i] = std::max(hi[i], d.geometry.vertices[v * d.dim + i]);
      }
  }
  const int grid = d.sigma_bar_grid > 0 ? d.sigma_bar_grid : (d.dim == 2 ? 1024 : 64);
  double h[3] = {0, 0, 0};
  for (int i = 0; i < d.dim; ++i) h[i] = (hi[i] - lo[i]) / grid;
  const int nblocks = 1024;
  double* dout = nullptr;
  std::vector<double> hout((size_t)nblocks * 6);
  auto cleanup = [&]() {
    if (dout) (void)hipFree(dout);
    (void)hipFree(p->dmem);
    delete p;
  };
  if ((e = hipMalloc(&dout, hout.size() * sizeof(double))) != hipSuccess ||
      (e = launch_sigma_sample(d.dim, g.kind, p->d64(), lo, h, grid, nblocks, dout, 0)) != hipSuccess ||
      (e = hipMemcpy(hout.data(), dout, hout.size() * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess) {
    cleanup();
    return fail(WOS_ERR_DEVICE, std::string("sigma' sampling failed: ") + hipGetErrorString(e));
  }
  (void)hipFree(dout);
  dout = nullptr;
  double mn = INFINITY, mx = -INFINITY, amin = INFINITY, smin = INFINITY, bad = 0, cnt = 0;
  for (int b = 0; b < nblocks; ++b) {
    mn = std::min(mn, hout[6 * b]);
    mx = std::max(mx, hout[6 * b + 1]);
    amin = std::min(amin, hout[6 * b + 2]);
    smin = std::min(smin, hout[6 * b + 3]);
    bad += hout[6 * b + 4];
    cnt += hout[6 * b + 5];
  }
  wos_status st = WOS_OK;
  std::string msg;
  if (cnt == 0) {
    st = WOS_ERR_GEOMETRY;
    msg = "no interior sample points (domain empty or inside-out)";
  } else if (bad > 0) {
    st = WOS_ERR_COEFFICIENT;
    msg = "non-finite alpha or sigma' at sample points";
  } else if (!(amin > 0)) {
    st = WOS_ERR_COEFFICIENT;
    msg = "alpha <= 0 at sample points";
  } else if (smin < 0 && !d.allow_negative_sigma) {
    st = WOS_ERR_COEFFICIENT;
    msg = "sigma < 0 at sample points";
  }
  double sb = d.sigma_bar;
  if (st == WOS_OK) {
    p->sp_min = mn;
    p->sp_max = mx;
    const double scale = std::max(1.0, std::max(std::fabs(mn), std::fabs(mx)));
    const bool sp_zero = std::fabs(mn) <= 1e-12 * scale && std::fabs(mx) <= 1e-12 * scale && mx - mn <= 1e-12;
    if (sb < 0) {
      sb = sp_zero ? 0.0 : std::max(mx, 0.0) - std::min(mn, 0.0);
    } else if (sb == 0 && !sp_zero) {
      st = WOS_ERR_COEFFICIENT;
      msg = "sigma_bar = 0 requires sigma' = 0 everywhere";
    }
  }
  if (st != WOS_OK) {
    cleanup();
    return fail(st, msg);
  }
  p->sigma_bar = sb;
  set_sigma_bar<float>(p->staging.data() + p->off32, sb);
  set_sigma_bar<double>(p->staging.data() + p->off64, sb);
  if ((e = upload()) != hipSuccess) {
    cleanup();
    return fail(WOS_ERR_DEVICE, "upload of sigma_bar failed");
  }
  p->geometry_ms = geometry_ms;
  p->upload_ms = upload_ms;
  p->sigma_bar_ms = ms_since(t0);
  *out = p;
  return WOS_OK;
}

wos_status wos_problem_create(const wos_problem_desc* desc, int device, wos_problem** out) {
  return guarded([&] { return problem_create_impl(desc, device, out); });
}

wos_status wos_problem_info(const wos_problem* p, double* sp_min, double* sp_max, double* sigma_bar) {
  if (!p) return fail(WOS_ERR_INVALID_ARG, "null problem");
  if (sp_min) *sp_min = p->sp_min;
  if (sp_max) *sp_max = p->sp_max;
  if (sigma_bar) *sigma_bar = p->sigma_bar;
  return WOS_OK;
}

wos_status wos_problem_setup_times(const wos_problem* p, double* geometry_ms, double* sigma_bar_ms, double* upload_ms) {
  if (!p) return fail(WOS_ERR_INVALID_ARG, "null problem");
  if (geometry_ms) *geometry_ms = p->geometry_ms;
  if (sigma_bar_ms) *sigma_bar_ms = p->sigma_bar_ms;
  if (upload_ms) *upload_ms = p->upload_ms;
  return WOS_OK;
}

wos_status wos_problem_bvh_info(const wos_problem* p, int64_t* n_nodes, int32_t* depth, int64_t* n_prims) {
  if (!p) return fail(WOS_ERR_INVALID_ARG, "null problem");
  if (n_nodes) *n_nodes = p->n_nodes;
  if (depth) *depth = p->depth;
  if (n_prims) *n_prims = p->n_prims;
  return WOS_OK;
}

wos_status wos_problem_grid_info(const wos_problem* p, int32_t* nx, int32_t* ny, int32_t* nz,
                                 int64_t* n_candidates) {
  if (!p) return fail(WOS_ERR_INVALID_ARG, "null problem");
  if (nx) *nx = p->grid_nx;
  if (ny) *ny = p->grid_ny;
  if (nz) *nz = p->grid_nz;
  if (n_candidates) *n_candidates = p->grid_candidates;
  return WOS_OK;
}

wos_status wos_problem_destroy(wos_problem* p) {
  if (!p) return WOS_OK;
  (void)hipSetDevice(p->device);
  if (p->dmem) (void)hipFree(p->dmem);
  delete p;
  return WOS_OK;
}

}  // extern "C"

// ====================================================================== solving

namespace {

struct Schedule {
  int fp64 = 0, compensated = 0, dim = 2, geom = 0, device = 0;
  int fp32_draws = 0;         // FP64 walker drawing the FP32 walker's uniforms
  int variant = 0;            // 2 selects the next-flight walker
  int grad = 0;               // some item asks for gradient sums
  int mode = 0;               // walker instantiation (walker_mode)
  int batch = 0;              // more than one item: tuned apart from single problems, whose
                              // tile length does not pay for problem switches
  unsigned block = 256, grid = 0;
  uint32_t tile_walks = 256;
  uint64_t chunk_walks = 0;   // walks per point per launch
  uint64_t total_points = 0;
  int n_launches = 0;
  int slot_words = 16;        // words per accumulation slot
  int grad_dim = 0;           // dim when gradient sums are asked for, else 0
};

wos_status check_items(const wos_batch_item* items, int n_items, const wos_options* opt, Schedule& s) {
  if (!items || n_items <= 0 || !opt) return fail(WOS_ERR_INVALID_ARG, "null or empty batch");
  if (opt->precision < 0 || opt->precision > 3) return fail(WOS_ERR_INVALID_ARG, "unknown precision");
  if (opt->precision == WOS_FP64_FP32_DRAWS && opt->variant == 2)
    return fail(WOS_ERR_INVALID_ARG, "FP32 draws in the FP64 walker apply to delta tracking (variant 0 or 1)");
  if (opt->variant < 0 || opt->variant > 2) return fail(WOS_ERR_INVALID_ARG, "unknown variant");
  if (opt->variant == 2 && opt->russian_roulette)
    return fail(WOS_ERR_INVALID_ARG, "the next-flight walk has its own roulette; russian_roulette must be 0");
  if (opt->walks_per_point == 0) return fail(WOS_ERR_INVALID_ARG, "walks_per_point must be > 0");
  if (opt->walk_offset + opt->walks_per_point > (1ull << 32)) return fail(WOS_ERR_INVALID_ARG, "walk indices exceed 32 bits");
  if (opt->russian_roulette && !(opt->ww_lo > 0)) return fail(WOS_ERR_INVALID_ARG, "ww_lo must be > 0");
  if (opt->ww_hi < 0 || opt->ww_hi != opt->ww_hi) return fail(WOS_ERR_INVALID_ARG, "ww_hi must be >= 0");
  if (opt->ww_hi > 0 && opt->variant == 2)
    return fail(WOS_ERR_INVALID_ARG, "weight-window splitting applies to delta tracking (variant 0 or 1)");
  if (opt->ww_hi > 0 && opt->russian_roulette && !(opt->ww_hi > opt->ww_lo))
    return fail(WOS_ERR_INVALID_ARG, "ww_hi must exceed ww_lo");
  if (opt->block_size != 0 && (opt->block_size < 64 || opt->block_size > 256 || opt->block_size % 64))
    return fail(WOS_ERR_INVALID_ARG, "block_size must be 64, 128, 192 or 256");
  if (opt->tile_walks < 0 || (uint32_t)opt->tile_walks > kMaxTileLen)
    return fail(WOS_ERR_INVALID_ARG, "tile_walks must be in 0..65536");
  const wos_problem* p0 = items[0].problem;
  if (!p0) return fail(WOS_ERR_INVALID_ARG, "null problem in item 0");
  s.dim = p0->dim;
  s.geom = p0->geom;
  s.device = p0->device;
  s.fp64 = opt->precision == WOS_FP64 || opt->precision == WOS_FP64_FP32_DRAWS;
  s.fp32_draws = opt->precision == WOS_FP64_FP32_DRAWS;
  s.variant = opt->variant;
  s.compensated = opt->precision == WOS_FP32_COMPENSATED;
  s.total_points = 0;
  s.batch = n_items > 1 ? 1 : 0;
  for (int k = 0; k < n_items; ++k) {
    const wos_batch_item& it = items[k];
    if (!it.problem) return fail(WOS_ERR_INVALID_ARG, "null problem in batch");
    if (it.problem->dim != s.dim || it.problem->geom != s.geom || it.problem->device != s.device)
      return fail(WOS_ERR_UNSUPPORTED, "batch items must share dim, geometry kind and device");
    if (it.n_points < 0) return fail(WOS_ERR_INVALID_ARG, "n_points < 0");
    if (it.n_points >= (1ll << 32)) return fail(WOS_ERR_INVALID_ARG, "n_points must be < 2^32");
    if (opt->ww_hi > 0 && it.problem_index >= (1u << 16))
      return fail(WOS_ERR_INVALID_ARG, "problem_index must be < 2^16 with weight-window splitting");
    if (it.n_points > 0 && (!it.points || !it.sum || !it.sum_sq || !it.n_walks || !it.n_steps))
      return fail(WOS_ERR_INVALID_ARG, "null device pointer in batch item");
    if ((it.grad_sum == nullptr) != (it.grad_sum_sq == nullptr))
      return fail(WOS_ERR_INVALID_ARG, "grad_sum and grad_sum_sq must both be set or both be null");
    if (it.grad_sum) s.grad = 1;
    s.total_points += (uint64_t)it.n_points;
  }
  if (s.grad && s.variant == 2) return fail(WOS_ERR_INVALID_ARG, "gradient estimates need delta tracking (variant 0 or 1)");
  s.mode = walker_mode(s.variant, s.grad != 0, opt->ww_hi > 0);
  s.grad_dim = s.grad ? s.dim : 0;
  s.slot_words = slot_words(s.grad_dim);
  return WOS_OK;
}

// Bytes of one lane's gradient record, and the lanes of any persistent grid on the device
// (resident threads per CU at most 2048).
size_t grad_record_bytes(const Schedule& s) {
  return (size_t)(1 + 3 * s.dim) * (s.fp64 ? sizeof(double) : sizeof(float));
}

std::mutex g_occ_mutex;
std::map<std::tuple<int, int, int, int, int, unsigned>, unsigned> g_occ;
std::map<int, int> g_cus;

// Launch shapes found by the plan autotuner, per (device, fp64, compensated, dim, geometry).
std::map<std::tuple<int, int, int, int, int, int, int>, std::pair<unsigned, uint32_t>> g_tuned;

std::tuple<int, int, int, int, int, int, int> tune_key(const Schedule& s) {
  return std::make_tuple(s.device, s.fp64, s.compensated, s.dim, s.geom, s.mode, s.batch);
}

wos_status device_cus(int device, int* cus) {
  std::lock_guard<std::mutex> lk(g_occ_mutex);
  auto it = g_cus.find(device);
  if (it == g_cus.end()) {
    int n = 0;
    WOS_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device));
    it = g_cus.emplace(device, std::max(1, n)).first;
  }
  *cus = it->second;
  return WOS_OK;
}

uint64_t max_grid_lanes(int cus) { return (uint64_t)cus * 2048u; }

// Persistent grid for a block size: resident blocks per CU times CUs.
wos_status grid_for_block(Schedule& s, unsigned block) {
  int cus = 0;
  wos_status r = device_cus(s.device, &cus);
  if (r != WOS_OK) return r;
  const auto key = std::make_tuple(s.device, s.fp64, s.dim, s.geom, s.mode, block);
  std::lock_guard<std::mutex> lk(g_occ_mutex);
  auto it = g_occ.find(key);
  if (it == g_occ.end()) {
    int per_cu = 0;
    WOS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, walker_symbol(s.fp64, s.dim, s.geom, s.mode), (int)block, 0));
    unsigned grid = (unsigned)std::max(1, per_cu) * (unsigned)cus;
    it = g_occ.emplace(key, grid).first;
  }
  s.block = block;
  s.grid = it->second;
  return WOS_OK;
}

// Slots of one launch of `chunk` walks per point: every point takes max(1, ceil(chunk /
// tile)) of them.
uint64_t slots_for(uint64_t total_points, uint64_t chunk, uint32_t tile) {
  return total_points * std::max<uint64_t>(1, (chunk + tile - 1) / tile);
}

// Block size and tile length: the caller's, else the tuned shape of this walker, else
// 256 / 256. Walks per point are split into launches only when the slots of one launch
// would exceed the workspace cap.
wos_status pick_shape(const wos_options* opt, Schedule& s) {
  unsigned block = 256u;
  uint32_t tile = 256u;
  {
    std::lock_guard<std::mutex> lk(g_occ_mutex);
    auto t = g_tuned.find(tune_key(s));
    if (t != g_tuned.end()) {
      block = t->second.first;
      tile = t->second.second;
    }
  }
  if (opt->block_size) block = (unsigned)opt->block_size;
  if (opt->tile_walks > 0) tile = (uint32_t)opt->tile_walks;
  s.tile_walks = tile;
  wos_status r = grid_for_block(s, block);
  if (r != WOS_OK) return r;
  const uint64_t cap = opt->workspace_bytes ? opt->workspace_bytes : (4ull << 30);
  const uint64_t slot_bytes = (uint64_t)s.slot_words * 8u;
  const uint64_t N = opt->walks_per_point;
  uint64_t nc = N;
  if (s.total_points > 0 && slots_for(s.total_points, N, tile) * slot_bytes > cap) {
    const uint64_t tiles_per_point = std::max<uint64_t>(1, cap / slot_bytes / s.total_points);
    nc = std::min<uint64_t>(N, tiles_per_point * tile);
  }
  s.chunk_walks = nc;
  s.n_launches = (int)((N + nc - 1) / nc);
  return WOS_OK;
}

// Cuts each item's walks of one launch into point-major tiles of `tile` walks and numbers
// their slots (DevItem); returns the launch's tiles and slots.
void layout_items(std::vector<DevItem>& dit, uint32_t tile, uint64_t* n_tiles, uint64_t* n_slots) {
  uint64_t tb = 0, sb = 0;
  for (DevItem& d : dit) {
    const uint64_t n = (uint64_t)d.n_points;
    d.tile_len = tile;
    d.tile_base = tb;
    d.slot_base = sb;
    if (d.walks >= tile) {
      d.tiles_per_point = (uint32_t)((d.walks + tile - 1) / tile);
      d.points_per_tile = 0;
      d.n_tiles = n * d.tiles_per_point;
      sb += d.n_tiles;
    } else {
      d.tiles_per_point = 0;
      d.points_per_tile = (uint32_t)(tile / d.walks);
      d.n_tiles = (n + d.points_per_tile - 1) / d.points_per_tile;
      sb += n;
    }
    tb += d.n_tiles;
  }
  *n_tiles = tb;
  *n_slots = sb;
}

// Per-launch item tables (walks and walk offset of the launch's chunk, tile cut, slots).
void build_items(const wos_batch_item* items, int n_items, const wos_options* opt, const Schedule& s, uint64_t w0,
                 uint64_t nw, const std::vector<int8_t*>& inside, const std::vector<void*>& gamma0,
                 std::vector<DevItem>& dit, uint64_t* n_tiles, uint64_t* n_slots) {
  dit.resize(n_items);
  uint64_t pbase = 0;
  for (int k = 0; k < n_items; ++k) {
    const wos_batch_item& it = items[k];
    DevItem& d = dit[k];
    std::memset(&d, 0, sizeof(d));
    d.problem = s.fp64 ? it.problem->d64() : it.problem->d32();
    d.points = it.points;
    d.inside = inside[k];
    d.gamma0 = gamma0[k];
    d.sum = it.sum;
    d.sum_sq = it.sum_sq;
    d.n_walks = it.n_walks;
    d.n_steps = it.n_steps;
    d.counters = it.counters;
    d.grad_sum = it.grad_sum;
    d.grad_sum_sq = it.grad_sum_sq;
    d.n_points = it.n_points;
    d.walks = nw;
    d.walk_offset = opt->walk_offset + w0;
    d.point_base = pbase;
    d.problem_index = it.problem_index;
    pbase += (uint64_t)it.n_points;
  }
  layout_items(dit, s.tile_walks, n_tiles, n_slots);
}

struct Workspace {
  int8_t* inside = nullptr;
  unsigned char* gamma0 = nullptr;  // [total points] gamma(x0), walker precision
  DevItem* items = nullptr;       // [n_launches][n_items]
  uint32_t* counter = nullptr;
  LaunchParams* lp = nullptr;
  uint64_t* slots = nullptr;      // [slots of the largest launch][slot_words]
  void* grad = nullptr;           // per-lane gradient records, when any item asks for gradients
};

}  // namespace

struct wos_plan {
  Schedule s;
  std::vector<wos_batch_item> items;
  wos_options opt;
  Workspace ws;
  void* dmem = nullptr;
  std::vector<uint64_t> n_tiles;      // per launch
  std::vector<uint64_t> n_slots;      // per launch
  std::vector<std::vector<DevItem>> dit;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double tune_ms = 0, build_ms = 0;   // set-up time (host wall clock)
  int tuned_here = 0;                 // 1 if this plan ran the autotuner
};

namespace {

size_t align_up(size_t v) { return (v + 255) / 256 * 256; }

// Byte layout of a job's workspace.
struct WsLayout {
  size_t inside, gamma0, items, counter, lp, slots, grad, total;
};

WsLayout ws_layout(const Schedule& s, int n_items, uint64_t max_slots, int cus) {
  WsLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.inside = take(std::max<uint64_t>(s.total_points, 1));
  L.gamma0 = take(std::max<uint64_t>(s.total_points, 1) * (s.fp64 ? 8 : 4));
  L.items = take(sizeof(DevItem) * (size_t)n_items * s.n_launches);
  L.counter = take(sizeof(uint32_t) * 64);
  L.lp = take(sizeof(LaunchParams));
  L.slots = take((size_t)std::max<uint64_t>(max_slots, 1) * s.slot_words * sizeof(uint64_t));
  L.grad = take(s.grad ? grad_record_bytes(s) * max_grid_lanes(cus) : 0);
  L.total = off;
  return L;
}

void ws_bind(Workspace& w, void* base, const WsLayout& L) {
  unsigned char* b = (unsigned char*)base;
  w.inside = (int8_t*)(b + L.inside);
  w.gamma0 = b + L.gamma0;
  w.items = (DevItem*)(b + L.items);
  w.counter = (uint32_t*)(b + L.counter);
  w.lp = (LaunchParams*)(b + L.lp);
  w.slots = (uint64_t*)(b + L.slots);
  w.grad = (void*)(b + L.grad);
}

// Item tables of every launch of a job, on the host; tiles and slots per launch.
wos_status prepare(const wos_batch_item* items, int n_items, const wos_options* opt, const Schedule& s,
                   const Workspace& w, std::vector<std::vector<DevItem>>& dit, std::vector<uint64_t>& n_tiles,
                   std::vector<uint64_t>& n_slots) {
  std::vector<int8_t*> inside(n_items);
  std::vector<void*> gamma0(n_items);
  uint64_t pb = 0;
  for (int k = 0; k < n_items; ++k) {
    inside[k] = w.inside + pb;
    gamma0[k] = w.gamma0 + pb * (s.fp64 ? 8 : 4);
    pb += (uint64_t)items[k].n_points;
  }
  dit.resize(s.n_launches);
  n_tiles.assign(s.n_launches, 0);
  n_slots.assign(s.n_launches, 0);
  for (int c = 0; c < s.n_launches; ++c) {
    const uint64_t w0 = (uint64_t)c * s.chunk_walks;
    const uint64_t nw = std::min(s.chunk_walks, opt->walks_per_point - w0);
    build_items(items, n_items, opt, s, w0, nw, inside, gamma0, dit[c], &n_tiles[c], &n_slots[c]);
    if (n_tiles[c] >= (1ull << 32) || n_slots[c] >= (1ull << 31))
      return fail(WOS_ERR_INVALID_ARG, "job too large: a launch would hold 2^32 tiles or 2^31 slots or more");
  }
  return WOS_OK;
}

// Slots of the largest launch of a schedule (no tables are built).
uint64_t max_launch_slots(const wos_batch_item* items, int n_items, const wos_options* opt, const Schedule& s) {
  (void)items;
  (void)n_items;
  uint64_t m = 0;
  for (int c = 0; c < s.n_launches; ++c) {
    const uint64_t w0 = (uint64_t)c * s.chunk_walks;
    const uint64_t nw = std::min(s.chunk_walks, opt->walks_per_point - w0);
    m = std::max(m, slots_for(s.total_points, nw, s.tile_walks));
  }
  return m;
}

// Launch record of the walker for launch c of a schedule over the given item table.
WalkerLaunch walker_launch(const wos_options* opt, const Schedule& s, const Workspace& w, const DevItem* items,
                           int n_items, uint64_t n_tiles) {
  WalkerLaunch L;
  L.fp64 = s.fp64;
  L.dim = s.dim;
  L.geom = s.geom;
  L.grid = s.grid;
  L.block = s.block;
  L.items = items;
  L.n_items = n_items;
  L.n_tiles = (uint32_t)n_tiles;
  L.tile_counter = w.counter;
  L.slots = w.slots;
  L.slot_words = s.slot_words;
  L.lp = w.lp;
  L.max_steps = opt->max_steps ? opt->max_steps : 1000000ull;
  L.variant = opt->variant;
  L.compensated = s.compensated;
  L.fp32_draws = s.fp32_draws;
  L.rr = opt->russian_roulette;
  L.ww_lo = opt->ww_lo > 0 ? opt->ww_lo : 0.5;
  L.ww_hi = opt->ww_hi > 0 ? opt->ww_hi : 0.0;
  L.grad = s.grad ? w.grad : nullptr;
  L.events = nullptr;
  return L;
}

// Classifies every query point (FP64) and evaluates gamma at the interior ones in the
// walker's precision.
hipError_t classify_items(const wos_batch_item* items, int n_items, const Schedule& s, const Workspace& w,
                          hipStream_t st) {
  uint64_t pb = 0;
  for (int k = 0; k < n_items; ++k) {
    const wos_batch_item& it = items[k];
    hipError_t e = launch_classify(s.dim, s.geom, it.problem->d64(), it.points, it.n_points, w.inside + pb,
                                   it.counters, st);
    if (e == hipSuccess)
      e = launch_gamma0(s.fp64, s.dim, s.fp64 ? it.problem->d64() : it.problem->d32(), it.points, it.n_points,
                        w.inside + pb, w.gamma0 + pb * (s.fp64 ? 8 : 4), st);
    if (e != hipSuccess) return e;
    pb += (uint64_t)it.n_points;
  }
  return hipSuccess;
}

// Enqueues [clear, walker, reduce per item] for every launch of the schedule. With
// `marks`, an event pair is recorded around each walker launch (eager timing only: a
// captured job takes none).
wos_status enqueue_job(const wos_batch_item* items, int n_items, const wos_options* opt, const Schedule& s,
                       const Workspace& w, const std::vector<std::vector<DevItem>>& dit,
                       const std::vector<uint64_t>& n_tiles, const std::vector<uint64_t>& n_slots, bool classify,
                       uint64_t* events, hipStream_t st, const std::vector<hipEvent_t>* marks = nullptr) {
  if (classify) WOS_HIP(classify_items(items, n_items, s, w, st));
  for (int c = 0; c < s.n_launches; ++c) {
    if (n_tiles[c] == 0) continue;
    WOS_HIP(launch_clear(w.slots, n_slots[c] * (uint64_t)s.slot_words, w.counter, st));
    WalkerLaunch L = walker_launch(opt, s, w, w.items + (size_t)c * n_items, n_items, n_tiles[c]);
    L.events = events;
    if (marks) WOS_HIP(hipEventRecord((*marks)[2 * c], st));
    WOS_HIP(launch_walker(L, st));
    if (marks) WOS_HIP(hipEventRecord((*marks)[2 * c + 1], st));
    for (int k = 0; k < n_items; ++k) WOS_HIP(launch_reduce(s.grad_dim, dit[c][k], w.slots, s.slot_words, st));
  }
  return WOS_OK;
}

wos_status upload_items(const Schedule& s, int n_items, const Workspace& w, const std::vector<std::vector<DevItem>>& dit,
                        hipStream_t st) {
  // Pageable host source: the runtime stages the copy before returning.
  std::vector<DevItem> all_items((size_t)n_items * s.n_launches);
  for (int c = 0; c < s.n_launches; ++c) std::copy(dit[c].begin(), dit[c].end(), all_items.begin() + (size_t)c * n_items);
  WOS_HIP(hipMemcpyAsync(w.items, all_items.data(), all_items.size() * sizeof(DevItem), hipMemcpyHostToDevice, st));
  WOS_HIP(hipStreamSynchronize(st));
  return WOS_OK;
}

}  // namespace

extern "C" {

static wos_status solve_impl(const wos_batch_item* items, int32_t n_items, const wos_options* opt, uint64_t* events,
                             void* stream) {
  Schedule s;
  wos_status r = check_items(items, n_items, opt, s);
  if (r != WOS_OK) return r;
  WOS_HIP(hipSetDevice(s.device));
  if ((r = pick_shape(opt, s)) != WOS_OK) return r;
  if (s.total_points == 0) return WOS_OK;
  int cus = 0;
  if ((r = device_cus(s.device, &cus)) != WOS_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  Workspace w;
  std::vector<std::vector<DevItem>> dit;
  std::vector<uint64_t> n_tiles, n_slots;
  // tables reference workspace addresses, so allocate first
  const WsLayout L = ws_layout(s, n_items, max_launch_slots(items, n_items, opt, s), cus);
  void* base = nullptr;
  WOS_HIP(hipMallocAsync(&base, L.total, st));
  ws_bind(w, base, L);
  r = prepare(items, n_items, opt, s, w, dit, n_tiles, n_slots);
  if (r == WOS_OK) r = upload_items(s, n_items, w, dit, st);
  if (r == WOS_OK) {
    const hipError_t e = launch_set_params(w.lp, opt->seed, 0, st);
    r = e != hipSuccess ? fail(WOS_ERR_DEVICE, "launch failed")
                        : enqueue_job(items, n_items, opt, s, w, dit, n_tiles, n_slots, true, events, st);
  }
  (void)hipFreeAsync(base, st);
  return r;
}

wos_status wos_solve(const wos_batch_item* items, int32_t n_items, const wos_options* opt, void* stream) {
  return guarded([&] { return solve_impl(items, n_items, opt, nullptr, stream); });
}

// wos_solve on the library's static scratch array instead of allocated memory: the same
// schedule, tables and kernels; the accumulation slots get what the array leaves after the
// per-point tables, and walks per point are split into launches when they do not fit.
static wos_status solve_static_impl(const wos_batch_item* items, int32_t n_items, const wos_options* opt,
                                    void* stream) {
  Schedule s;
  wos_status r = check_items(items, n_items, opt, s);
  if (r != WOS_OK) return r;
  WOS_HIP(hipSetDevice(s.device));
  void* base = nullptr;
  WOS_HIP(static_scratch(s.device, &base));
  int cus = 0;
  if ((r = device_cus(s.device, &cus)) != WOS_OK) return r;
  // everything but the slots, with room for the item tables of up to 64 launches
  Schedule probe = s;
  probe.n_launches = 64;
  const size_t fixed = ws_layout(probe, n_items, 0, cus).total;
  const size_t cap = kStaticScratchBytes;
  if (fixed + (size_t)s.slot_words * 8 * std::max<uint64_t>(s.total_points, 1) > cap)
    return fail(WOS_ERR_INVALID_ARG, "wos_solve_static: " + std::to_string(s.total_points) + " query points need " +
                                         std::to_string(fixed) + " bytes of tables and one " +
                                         std::to_string(s.slot_words * 8) + "-byte slot each, more than the " +
                                         std::to_string(cap) + "-byte static scratch");
  wos_options o = *opt;
  const uint64_t room = cap - fixed;
  o.workspace_bytes = opt->workspace_bytes ? std::min<uint64_t>(opt->workspace_bytes, room) : room;
  if ((r = pick_shape(&o, s)) != WOS_OK) return r;
  if (s.total_points == 0) return WOS_OK;
  const WsLayout L = ws_layout(s, n_items, max_launch_slots(items, n_items, &o, s), cus);
  if (L.total > cap)
    return fail(WOS_ERR_INVALID_ARG, "wos_solve_static: the job needs " + std::to_string(L.total) +
                                         " bytes of scratch, more than the " + std::to_string(cap) + " available");
  hipStream_t st = (hipStream_t)stream;
  Workspace w;
  ws_bind(w, base, L);
  std::vector<std::vector<DevItem>> dit;
  std::vector<uint64_t> n_tiles, n_slots;
  if ((r = prepare(items, n_items, &o, s, w, dit, n_tiles, n_slots)) != WOS_OK) return r;
  if ((r = upload_items(s, n_items, w, dit, st)) != WOS_OK) return r;
  WOS_HIP(launch_set_params(w.lp, o.seed, 0, st));
  return enqueue_job(items, n_items, &o, s, w, dit, n_tiles, n_slots, true, nullptr, st);
}

wos_status wos_solve_static(const wos_batch_item* items, int32_t n_items, const wos_options* opt, void* stream) {
  return guarded([&] { return solve_static_impl(items, n_items, opt, stream); });
}

wos_status wos_count_events(const wos_batch_item* items, int32_t n_items, const wos_options* opt, uint64_t* events,
                            void* stream) {
  if (!events) return fail(WOS_ERR_INVALID_ARG, "null events");
  return guarded([&] { return solve_impl(items, n_items, opt, events, stream); });
}

wos_status wos_finalize(const double* sum, const double* sum_sq, const uint64_t* n_walks, int64_t n, double* mean,
                        double* std_err, void* stream) {
  if (n < 0 || (n > 0 && (!sum || !sum_sq || !n_walks || !mean || !std_err)))
    return fail(WOS_ERR_INVALID_ARG, "bad finalize arguments");
  WOS_HIP(launch_finalize(sum, sum_sq, n_walks, n, mean, std_err, (hipStream_t)stream));
  return WOS_OK;
}

}  // extern "C"

namespace {

wos_status plan_build(const wos_batch_item* items, int32_t n_items, const wos_options* opt, void* stream,
                      wos_plan** out) {
  if (!out) return fail(WOS_ERR_INVALID_ARG, "null out");
  *out = nullptr;
  wos_plan* P = new wos_plan();
  wos_status r = check_items(items, n_items, opt, P->s);
  if (r != WOS_OK) {
    delete P;
    return r;
  }
  (void)hipSetDevice(P->s.device);
  if ((r = pick_shape(opt, P->s)) != WOS_OK) {
    delete P;
    return r;
  }
  int cus = 0;
  if ((r = device_cus(P->s.device, &cus)) != WOS_OK) {
    delete P;
    return r;
  }
  P->items.assign(items, items + n_items);
  P->opt = *opt;
  hipStream_t st = (hipStream_t)stream;
  const Schedule& s = P->s;
  const WsLayout L = ws_layout(s, n_items, max_launch_slots(items, n_items, opt, s), cus);
  hipError_t e = hipMalloc(&P->dmem, L.total);
  if (e != hipSuccess) {
    delete P;
    return fail(e == hipErrorOutOfMemory ? WOS_ERR_OUT_OF_MEMORY : WOS_ERR_DEVICE, "plan workspace allocation failed");
  }
  ws_bind(P->ws, P->dmem, L);
  auto bail = [&](wos_status code, const std::string& m) {
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    (void)hipFree(P->dmem);
    delete P;
    return fail(code, m);
  };
  if ((r = prepare(items, n_items, opt, s, P->ws, P->dit, P->n_tiles, P->n_slots)) != WOS_OK) return bail(r, g_error);
  if ((r = upload_items(s, n_items, P->ws, P->dit, st)) != WOS_OK) return bail(r, g_error);
  // classification and gamma(x0) once, outside the graph
  if ((e = classify_items(items, n_items, s, P->ws, st)) != hipSuccess)
    return bail(WOS_ERR_DEVICE, "classification launch failed");
  // capture clear + walker + reduce of every launch on a private stream
  hipStream_t cap;
  if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess) return bail(WOS_ERR_DEVICE, "stream creation failed");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) {
    (void)hipStreamDestroy(cap);
    return bail(WOS_ERR_DEVICE, "classification failed");
  }
  if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
    (void)hipStreamDestroy(cap);
    return bail(WOS_ERR_DEVICE, "graph capture failed to start");
  }
  r = enqueue_job(items, n_items, opt, s, P->ws, P->dit, P->n_tiles, P->n_slots, false, nullptr, cap);
  const hipError_t ec = hipStreamEndCapture(cap, &P->graph);
  (void)hipStreamDestroy(cap);
  if (r != WOS_OK || ec != hipSuccess) return bail(WOS_ERR_DEVICE, "graph capture failed");
  if ((e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0)) != hipSuccess)
    return bail(WOS_ERR_DEVICE, "graph instantiation failed");
  *out = P;
  return WOS_OK;
}

// Item table of an autotuning sample: every item of the plan's first launch contributes
// the first tiles of its share, in item order as in the real job, so that the sample
// switches problems as the job does; `walks` walks in all, each item in proportion to its
// walks. Slots are numbered for the sample alone.
void sample_items(const wos_plan* P, uint32_t tile, uint64_t walks, std::vector<DevItem>& d, uint64_t* n_tiles,
                  uint64_t* n_slots) {
  d = P->dit[0];
  double all = 0;
  for (const DevItem& x : d) all += (double)x.n_points * x.walks;
  uint64_t dummy_t = 0, dummy_s = 0;
  layout_items(d, tile, &dummy_t, &dummy_s);
  uint64_t tb = 0, sb = 0;
  for (DevItem& x : d) {
    const uint64_t item_walks = (uint64_t)x.n_points * x.walks;
    const uint64_t share = std::min<uint64_t>(item_walks, (uint64_t)((double)walks * (double)item_walks / all));
    const uint64_t per_tile = x.tiles_per_point > 0 ? tile : (uint64_t)x.points_per_tile * x.walks;
    const uint64_t m = std::min<uint64_t>(x.n_tiles, (share + per_tile - 1) / per_tile);
    x.tile_base = tb;
    x.slot_base = sb;
    x.n_tiles = m;
    tb += m;
    sb += x.tiles_per_point > 0 ? m : m * x.points_per_tile;
  }
  *n_tiles = tb;
  *n_slots = sb;
}

// Times the walker of a plan's first launch over an autotuning sample with the given
// shape, on the plan's counter and launch parameters and the sample's own item table and
// slots (the reduction, and with it the caller's outputs, is not run). Returns the best of
// `reps` runs in ms.
wos_status time_shape(wos_plan* P, unsigned block, uint32_t tile, uint64_t walks, DevItem* ditems, uint64_t* dslots,
                      int reps, hipStream_t st, float* best_ms) {
  Schedule s = P->s;
  wos_status r = grid_for_block(s, block);
  if (r != WOS_OK) return r;
  s.tile_walks = tile;
  std::vector<DevItem> d;
  uint64_t nt = 0, ns = 0;
  sample_items(P, tile, walks, d, &nt, &ns);
  const int n_items = (int)P->items.size();
  WOS_HIP(hipMemcpyAsync(ditems, d.data(), d.size() * sizeof(DevItem), hipMemcpyHostToDevice, st));
  WOS_HIP(hipStreamSynchronize(st));
  Workspace w = P->ws;
  w.slots = dslots;
  const WalkerLaunch L = walker_launch(&P->opt, s, w, ditems, n_items, nt);
  hipEvent_t a, b;
  WOS_HIP(hipEventCreate(&a));
  WOS_HIP(hipEventCreate(&b));
  *best_ms = 1e30f;
  hipError_t e = hipSuccess;
  for (int i = 0; i < reps && e == hipSuccess; ++i) {
    if ((e = launch_clear(dslots, ns * (uint64_t)s.slot_words, P->ws.counter, st)) != hipSuccess) break;
    if ((e = hipEventRecord(a, st)) != hipSuccess) break;
    if ((e = launch_walker(L, st)) != hipSuccess) break;
    if ((e = hipEventRecord(b, st)) != hipSuccess) break;
    if ((e = hipEventSynchronize(b)) != hipSuccess) break;
    float ms = 0;
    if ((e = hipEventElapsedTime(&ms, a, b)) != hipSuccess) break;
    *best_ms = std::min(*best_ms, ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return fail(WOS_ERR_DEVICE, std::string("autotune run failed: ") + hipGetErrorString(e));
  return WOS_OK;
}

// Chooses block size and tile length for this walker by timing candidates on samples of
// the plan's own walks (about eight and 40 walks per resident lane, so that every wave
// takes several tiles; each item contributes in proportion to its walks), and caches the
// winner per process. Jobs too small to time leave the defaults.
wos_status autotune(wos_plan* P, hipStream_t st, unsigned* block, uint32_t* tile, bool* ran) {
  static const unsigned kBlocks[] = {64, 128, 256};
  static const uint32_t kTiles[] = {64, 128, 256, 512, 1024};
  *block = P->s.block;
  *tile = P->s.tile_walks;
  *ran = false;
  uint64_t launch0 = 0;
  for (const DevItem& d : P->dit[0]) launch0 += (uint64_t)d.n_points * d.walks;
  uint64_t lanes = 0;
  for (unsigned b : kBlocks) {
    Schedule s = P->s;
    wos_status r = grid_for_block(s, b);
    if (r != WOS_OK) return r;
    lanes = std::max<uint64_t>(lanes, (uint64_t)s.grid * b);
  }
  const uint64_t walks = 8 * lanes;
  if (launch0 < walks) return WOS_OK;
  // A shape is scored by the marginal time of 4W more walks, T(5W) - T(W): in samples
  // this small the launch's drain (lanes idle while the last walks finish) is a large part
  // of T(W) and favours short tiles, which lose at full size (the FP64 walker ran 25%
  // slower with the shape chosen by T(W)). Jobs below 5W are scored by T(W). Shapes within
  // 3% of the best score count as ties, won by the longer tile (fewer slots): the sample's
  // scores scatter by a few per cent between runs, and on the star polygon tiles of 64
  // walks, picked by that scatter, ran 2% slower at full size than tiles of 256.
  const bool marginal = launch0 >= 5 * walks;
  const uint64_t sample_max = marginal ? 5 * walks : walks;
  WOS_HIP(launch_set_params(P->ws.lp, 0, 0, st));
  uint64_t max_slots = 0;
  for (uint32_t t : kTiles) {
    std::vector<DevItem> d;
    uint64_t nt = 0, ns = 0;
    sample_items(P, t, sample_max, d, &nt, &ns);
    max_slots = std::max(max_slots, ns);
  }
  DevItem* ditems = nullptr;
  uint64_t* dslots = nullptr;
  WOS_HIP(hipMalloc(&ditems, P->items.size() * sizeof(DevItem)));
  hipError_t e = hipMalloc(&dslots, std::max<uint64_t>(max_slots, 1) * P->s.slot_words * sizeof(uint64_t));
  if (e != hipSuccess) {
    (void)hipFree(ditems);
    return fail(WOS_ERR_OUT_OF_MEMORY, "autotune slot allocation failed");
  }
  struct Scored {
    unsigned block;
    uint32_t tile;
    float ms;
  };
  // Tiles longer than a point's walks hold several points, whose walks add into global
  // slots instead of the wave's LDS slot cache; the samples underrate that (on the
  // 64-polygon batch, 512 walks per point, tiles of 1024 ran 24% slower than 256 at full
  // size), so such tiles are tried only when no candidate fits one point.
  uint64_t min_walks = ~0ull;
  for (const DevItem& d : P->dit[0]) min_walks = std::min<uint64_t>(min_walks, (uint64_t)d.walks);
  const bool fits = min_walks >= kTiles[0];
  std::vector<Scored> scores;
  wos_status r = WOS_OK;
  for (unsigned b : kBlocks) {
    for (uint32_t t : kTiles) {
      if (fits && t > min_walks) continue;
      float ms = 0;
      if ((r = time_shape(P, b, t, walks, ditems, dslots, 3, st, &ms)) != WOS_OK) break;
      if (marginal) {
        float ms5 = 0;
        if ((r = time_shape(P, b, t, 5 * walks, ditems, dslots, 3, st, &ms5)) != WOS_OK) break;
        ms = ms5 - ms;
      }
      scores.push_back({b, t, ms});
    }
    if (r != WOS_OK) break;
  }
  if (r == WOS_OK && !scores.empty()) {
    float best = scores[0].ms;
    for (const Scored& c : scores) best = std::min(best, c.ms);
    const Scored* pick = nullptr;
    for (const Scored& c : scores) {
      if (c.ms > best + 0.03f * std::fabs(best)) continue;
      if (!pick || c.tile > pick->tile || (c.tile == pick->tile && c.ms < pick->ms)) pick = &c;
    }
    *block = pick->block;
    *tile = pick->tile;
  }
  (void)hipFree(ditems);
  (void)hipFree(dslots);
  if (r != WOS_OK) return r;
  std::lock_guard<std::mutex> lk(g_occ_mutex);
  g_tuned[tune_key(P->s)] = std::make_pair(*block, *tile);
  *ran = true;
  return WOS_OK;
}

}  // namespace

extern "C" {

wos_status wos_finalize_grad(const double* grad_sum, const double* grad_sum_sq, const uint64_t* n_walks, int64_t n,
                             int32_t dim, double* mean, double* std_err, void* stream) {
  if (n < 0 || (dim != 2 && dim != 3) || (n > 0 && (!grad_sum || !grad_sum_sq || !n_walks || !mean || !std_err)))
    return fail(WOS_ERR_INVALID_ARG, "bad finalize arguments");
  WOS_HIP(launch_finalize_components(grad_sum, grad_sum_sq, n_walks, n, dim, mean, std_err, (hipStream_t)stream));
  return WOS_OK;
}

static wos_status plan_create_impl(const wos_batch_item* items, int32_t n_items, const wos_options* opt,
                                   void* stream, wos_plan** out) {
  using clock = std::chrono::steady_clock;
  auto ms_since = [](clock::time_point t) { return std::chrono::duration<double, std::milli>(clock::now() - t).count(); };
  clock::time_point t0 = clock::now();
  wos_status r = plan_build(items, n_items, opt, stream, out);
  if (r != WOS_OK) return r;
  (*out)->build_ms = ms_since(t0);
  if (opt->block_size != 0 || opt->tile_walks != 0) return r;
  wos_plan* P = *out;
  bool tuned;
  {
    std::lock_guard<std::mutex> lk(g_occ_mutex);
    tuned = g_tuned.count(tune_key(P->s)) != 0;
  }
  if (tuned) return WOS_OK;
  unsigned block = 0;
  uint32_t tile = 0;
  bool ran = false;
  t0 = clock::now();
  if ((r = autotune(P, (hipStream_t)stream, &block, &tile, &ran)) != WOS_OK) {
    wos_plan_destroy(P);
    *out = nullptr;
    return r;
  }
  const double tune_ms = ms_since(t0);
  if (block == P->s.block && tile == P->s.tile_walks) {
    P->tune_ms = ran ? tune_ms : 0.0;
    P->tuned_here = ran ? 1 : 0;
    return WOS_OK;
  }
  // rebuild with the tuned shape (tile tables and workspace depend on it)
  wos_plan_destroy(P);
  *out = nullptr;
  wos_options o = *opt;
  o.block_size = (int32_t)block;
  o.tile_walks = (int32_t)tile;
  t0 = clock::now();
  r = plan_build(items, n_items, &o, stream, out);
  if (r == WOS_OK) {
    (*out)->build_ms = ms_since(t0);
    (*out)->tune_ms = tune_ms;
    (*out)->tuned_here = ran ? 1 : 0;
  }
  return r;
}

// ---------------------------------------------------------------- tuned-shape cache
// One line per tuned walker variant: arch CUs fp64 compensated dim geom mode batch block tile.
// The device is named by its architecture string and compute-unit count, so that a file
// written on one GPU applies to every GPU of the same kind.

static wos_status device_signature(int device, std::string* arch, int* cus) {
  hipDeviceProp_t prop;
  WOS_HIP(hipGetDeviceProperties(&prop, device));
  *arch = prop.gcnArchName;
  *cus = prop.multiProcessorCount;
  return WOS_OK;
}

static wos_status tune_cache_save_impl(const char* path, int32_t* n_saved) {
  if (!path) return fail(WOS_ERR_INVALID_ARG, "null path");
  std::map<std::tuple<int, int, int, int, int, int, int>, std::pair<unsigned, uint32_t>> tuned;
  {
    std::lock_guard<std::mutex> lk(g_occ_mutex);
    tuned = g_tuned;
  }
  std::string text = "# walk-on-spheres tuned launch shapes: arch cus fp64 compensated dim geom mode batch block tile\n";
  int n = 0;
  for (const auto& kv : tuned) {
    std::string arch;
    int cus = 0;
    const wos_status r = device_signature(std::get<0>(kv.first), &arch, &cus);
    if (r != WOS_OK) return r;
    char line[512];
    std::snprintf(line, sizeof(line), "%s %d %d %d %d %d %d %d %u %u\n", arch.c_str(), cus, std::get<1>(kv.first),
                  std::get<2>(kv.first), std::get<3>(kv.first), std::get<4>(kv.first), std::get<5>(kv.first),
                  std::get<6>(kv.first), kv.second.first, kv.second.second);
    text += line;
    ++n;
  }
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(WOS_ERR_INVALID_ARG, std::string("cannot write ") + path);
  const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
  if (std::fclose(f) != 0 || !ok) return fail(WOS_ERR_INVALID_ARG, std::string("write to ") + path + " failed");
  if (n_saved) *n_saved = n;
  return WOS_OK;
}

static wos_status tune_cache_load_impl(const char* path, int32_t* n_loaded) {
  if (!path) return fail(WOS_ERR_INVALID_ARG, "null path");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(WOS_ERR_INVALID_ARG, std::string("cannot read ") + path);
  struct Entry {
    std::string arch;
    int cus, key[6];
    unsigned block, tile;
  };
  std::vector<Entry> entries;
  char line[512];
  int lineno = 0;
  while (std::fgets(line, sizeof(line), f)) {
    ++lineno;
    if (line[0] == '#' || line[0] == '\n') continue;
    char arch[256];
    Entry e;
    if (std::sscanf(line, "%255s %d %d %d %d %d %d %d %u %u", arch, &e.cus, &e.key[0], &e.key[1], &e.key[2],
                    &e.key[3], &e.key[4], &e.key[5], &e.block, &e.tile) != 10 ||
        e.block < 64 || e.block > 256 || e.block % 64 || e.tile < 1 || e.tile > kMaxTileLen || e.key[0] < 0 ||
        e.key[0] > 1 || e.key[1] < 0 || e.key[1] > 1 || (e.key[2] != 2 && e.key[2] != 3) || e.key[3] < 0 ||
        e.key[3] > 4 || e.key[4] < 0 || e.key[4] > 2 || e.key[5] < 0 || e.key[5] > 1) {
      std::fclose(f);
      return fail(WOS_ERR_INVALID_ARG, std::string(path) + ": malformed line " + std::to_string(lineno));
    }
    e.arch = arch;
    entries.push_back(e);
  }
  std::fclose(f);
  int n_dev = 0;
  WOS_HIP(hipGetDeviceCount(&n_dev));
  int n = 0;
  for (int d = 0; d < n_dev; ++d) {
    std::string arch;
    int cus = 0;
    const wos_status r = device_signature(d, &arch, &cus);
    if (r != WOS_OK) return r;
    std::lock_guard<std::mutex> lk(g_occ_mutex);
    for (const Entry& e : entries) {
      if (e.arch != arch || e.cus != cus) continue;
      g_tuned[std::make_tuple(d, e.key[0], e.key[1], e.key[2], e.key[3], e.key[4], e.key[5])] =
          std::make_pair(e.block, (uint32_t)e.tile);
      ++n;
    }
  }
  if (n_loaded) *n_loaded = n;
  return WOS_OK;
}

wos_status wos_tune_cache_save(const char* path, int32_t* n_saved) {
  return guarded([&] { return tune_cache_save_impl(path, n_saved); });
}

wos_status wos_tune_cache_load(const char* path, int32_t* n_loaded) {
  return guarded([&] { return tune_cache_load_impl(path, n_loaded); });
}

wos_status wos_plan_create(const wos_batch_item* items, int32_t n_items, const wos_options* opt, void* stream,
                           wos_plan** out) {
  return guarded([&] { return plan_create_impl(items, n_items, opt, stream, out); });
}

wos_status wos_plan_time(wos_plan* P, uint64_t seed, uint64_t walk_offset_add, void* stream, double* walker_ms,
                         double* total_ms) {
  if (!P || !walker_ms) return fail(WOS_ERR_INVALID_ARG, "null plan or output");
  if (P->opt.walk_offset + walk_offset_add + P->opt.walks_per_point > (1ull << 32))
    return fail(WOS_ERR_INVALID_ARG, "walk indices exceed 32 bits");
  WOS_HIP(hipSetDevice(P->s.device));
  hipStream_t st = (hipStream_t)stream;
  std::vector<hipEvent_t> marks(2 * (size_t)P->s.n_launches + 2, nullptr);
  wos_status r = WOS_OK;
  for (auto& m : marks)
    if (hipEventCreate(&m) != hipSuccess) {
      r = fail(WOS_ERR_DEVICE, "event creation failed");
      break;
    }
  hipEvent_t& t0 = marks[marks.size() - 2];
  hipEvent_t& t1 = marks[marks.size() - 1];
  if (r == WOS_OK) {
    hipError_t e = launch_set_params(P->ws.lp, seed, walk_offset_add, st);
    if (e == hipSuccess) e = hipEventRecord(t0, st);
    if (e != hipSuccess) r = fail(WOS_ERR_DEVICE, "launch failed");
  }
  if (r == WOS_OK)
    r = enqueue_job(P->items.data(), (int)P->items.size(), &P->opt, P->s, P->ws, P->dit, P->n_tiles, P->n_slots,
                    false, nullptr, st, &marks);
  if (r == WOS_OK) {
    hipError_t e = hipEventRecord(t1, st);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    double w = 0;
    for (int c = 0; c < P->s.n_launches && e == hipSuccess; ++c) {
      if (P->n_tiles[c] == 0) continue;
      float ms = 0;
      e = hipEventElapsedTime(&ms, marks[2 * c], marks[2 * c + 1]);
      w += ms;
    }
    float tot = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&tot, t0, t1);
    if (e != hipSuccess) r = fail(WOS_ERR_DEVICE, std::string("timed run failed: ") + hipGetErrorString(e));
    *walker_ms = w;
    if (total_ms) *total_ms = tot;
  }
  for (auto& m : marks)
    if (m) (void)hipEventDestroy(m);
  return r;
}

wos_status wos_plan_launch(wos_plan* P, uint64_t seed, uint64_t walk_offset_add, void* stream) {
  if (!P) return fail(WOS_ERR_INVALID_ARG, "null plan");
  if (P->opt.walk_offset + walk_offset_add + P->opt.walks_per_point > (1ull << 32))
    return fail(WOS_ERR_INVALID_ARG, "walk indices exceed 32 bits");
  WOS_HIP(hipSetDevice(P->s.device));
  hipStream_t st = (hipStream_t)stream;
  WOS_HIP(launch_set_params(P->ws.lp, seed, walk_offset_add, st));
  WOS_HIP(hipGraphLaunch(P->exec, st));
  return WOS_OK;
}

wos_status wos_plan_info(const wos_plan* P, int32_t* block_size, int32_t* tile_walks, int32_t* grid_size,
                         int32_t* n_launches) {
  if (!P) return fail(WOS_ERR_INVALID_ARG, "null plan");
  if (block_size) *block_size = (int32_t)P->s.block;
  if (tile_walks) *tile_walks = (int32_t)P->s.tile_walks;
  if (grid_size) *grid_size = (int32_t)P->s.grid;
  if (n_launches) *n_launches = P->s.n_launches;
  return WOS_OK;
}

wos_status wos_plan_setup_times(const wos_plan* P, double* build_ms, double* tune_ms, int32_t* tuned_here) {
  if (!P) return fail(WOS_ERR_INVALID_ARG, "null plan");
  if (build_ms) *build_ms = P->build_ms;
  if (tune_ms) *tune_ms = P->tune_ms;
  if (tuned_here) *tuned_here = P->tuned_here;
  return WOS_OK;
}

wos_status wos_plan_destroy(wos_plan* P) {
  if (!P) return WOS_OK;
  (void)hipSetDevice(P->s.device);
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  if (P->dmem) (void)hipFree(P->dmem);
  delete P;
  return WOS_OK;
}

// ====================================================================== diagnostics

wos_status wos_eval_coefficients(const wos_problem* p, const double* points, int64_t n, int32_t precision, double* out,
                                 void* stream) {
  if (!p || n < 0 || (n > 0 && (!points || !out))) return fail(WOS_ERR_INVALID_ARG, "bad arguments");
  if (precision != WOS_FP32 && precision != WOS_FP64) return fail(WOS_ERR_INVALID_ARG, "precision must be FP32 or FP64");
  WOS_HIP(hipSetDevice(p->device));
  const int fp64 = precision == WOS_FP64;
  WOS_HIP(launch_coefficients(fp64, p->dim, fp64 ? p->d64() : p->d32(), points, n, out, (hipStream_t)stream));
  return WOS_OK;
}

wos_status wos_eval_distance(const wos_problem* p, const double* points, int64_t n, int32_t precision, double* d,
                             double* closest, void* stream) {
  if (!p || n < 0 || (n > 0 && (!points || !d || !closest))) return fail(WOS_ERR_INVALID_ARG, "bad arguments");
  if (precision != WOS_FP32 && precision != WOS_FP64) return fail(WOS_ERR_INVALID_ARG, "precision must be FP32 or FP64");
  WOS_HIP(hipSetDevice(p->device));
  const int fp64 = precision == WOS_FP64;
  WOS_HIP(launch_distance(fp64, p->dim, p->geom, fp64 ? p->d64() : p->d32(), points, n, d, closest, (hipStream_t)stream));
  return WOS_OK;
}

wos_status wos_eval_ball(int32_t dim, int32_t precision, const double* s, int64_t n, double* out, void* stream) {
  if ((dim != 2 && dim != 3) || n < 0 || (n > 0 && (!s || !out))) return fail(WOS_ERR_INVALID_ARG, "bad arguments");
  if (precision != WOS_FP32 && precision != WOS_FP64) return fail(WOS_ERR_INVALID_ARG, "precision must be FP32 or FP64");
  WOS_HIP(launch_ball(precision == WOS_FP64, dim, s, n, out, (hipStream_t)stream));
  return WOS_OK;
}

wos_status wos_sample_radius(int32_t dim, int32_t precision, double s, int64_t n, uint64_t seed, double* t,
                             uint64_t* trials, void* stream) {
  if ((dim != 2 && dim != 3) || n < 0 || (n > 0 && !t) || !(s >= 0) || !std::isfinite(s))
    return fail(WOS_ERR_INVALID_ARG, "bad arguments");
  if (n >= (1ll << 32)) return fail(WOS_ERR_INVALID_ARG, "n must be < 2^32");
  if (precision != WOS_FP32 && precision != WOS_FP64) return fail(WOS_ERR_INVALID_ARG, "precision must be FP32 or FP64");
  WOS_HIP(launch_sample(precision == WOS_FP64, dim, s, n, seed, t, trials, (hipStream_t)stream));
  return WOS_OK;
}

wos_status wos_philox(const uint32_t* ctr, uint64_t key, int64_t n, uint32_t* out, void* stream) {
  if (n < 0 || (n > 0 && (!ctr || !out))) return fail(WOS_ERR_INVALID_ARG, "bad arguments");
  WOS_HIP(launch_philox(ctr, key, n, out, (hipStream_t)stream));
  return WOS_OK;
}

wos_status wos_eval_bessel(int32_t which, int32_t precision, const double* x, int64_t n, double* out, void* stream) {
  if (which < 0 || which > 3 || n < 0 || (n > 0 && (!x || !out))) return fail(WOS_ERR_INVALID_ARG, "bad arguments");
  if (precision != WOS_FP32 && precision != WOS_FP64) return fail(WOS_ERR_INVALID_ARG, "precision must be FP32 or FP64");
  WOS_HIP(launch_bessel(precision == WOS_FP64, which, x, n, out, (hipStream_t)stream));
  return WOS_OK;
}

wos_status wos_eval_offcentred(int32_t which, int32_t dim, int32_t precision, double R, double sigma_bar,
                               const double* u, const double* v, int64_t n, double* out, void* stream) {
  if ((which != 0 && which != 1) || (dim != 2 && dim != 3) || n < 0 || (n > 0 && (!u || !v || !out)))
    return fail(WOS_ERR_INVALID_ARG, "bad arguments");
  if (!(R > 0) || !(sigma_bar >= 0)) return fail(WOS_ERR_INVALID_ARG, "R must be > 0 and sigma_bar >= 0");
  if (precision != WOS_FP32 && precision != WOS_FP64) return fail(WOS_ERR_INVALID_ARG, "precision must be FP32 or FP64");
  WOS_HIP(launch_offcentred(precision == WOS_FP64, dim, which, R, sigma_bar, u, v, n, out, (hipStream_t)stream));
  return WOS_OK;
}

wos_status wos_classify(const wos_problem* p, const double* points, int64_t n, int8_t* inside, void* stream) {
  if (!p || n < 0 || (n > 0 && (!points || !inside))) return fail(WOS_ERR_INVALID_ARG, "bad arguments");
  WOS_HIP(hipSetDevice(p->device));
  WOS_HIP(launch_classify(p->dim, p->geom, p->d64(), points, n, inside, nullptr, (hipStream_t)stream));
  return WOS_OK;
}

}  // extern "C"
