// Host check of the candidate grids (csrc/bvh.cpp) on CPU: for sampled points of each
// grid cell, the scan the walker performs (nearest to the cell centre first, stop once a
// candidate's centre distance minus the offset exceeds the best distance, then the tail
// bound) either returns the brute-force nearest distance or a lower bound of it, and the
// grid does not depend on the number of build threads.
//
// Usage: grid_check <tri|seg> <file of doubles: [n][12] triangles or [n][4] segments>
// Prints one line: "points P exact E bounded B bad_exact X bad_bound Y threads_equal T
// cells C" (the grid is built for 16 cells per primitive).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "bvh.h"

using namespace wos;

static double dot(const double* a, const double* b, int n) {
  double s = 0;
  for (int k = 0; k < n; ++k) s += a[k] * b[k];
  return s;
}

static double seg_d2(const double* a, const double* b, const double* p, int n) {
  double e[3], q[3];
  for (int k = 0; k < n; ++k) {
    e[k] = b[k] - a[k];
    q[k] = p[k] - a[k];
  }
  const double l2 = dot(e, e, n);
  double t = l2 > 0 ? dot(q, e, n) / l2 : 0.0;
  t = std::min(1.0, std::max(0.0, t));
  for (int k = 0; k < n; ++k) q[k] -= t * e[k];
  return dot(q, q, n);
}

// brute force by the plane projection and the edges, written independently of bvh.cpp's
static double tri_d2(const double* t, const double* p) {
  const double *a = t, *b = t + 3, *c = t + 6;
  double u[3], v[3], nrm[3];
  for (int k = 0; k < 3; ++k) {
    u[k] = b[k] - a[k];
    v[k] = c[k] - a[k];
  }
  nrm[0] = u[1] * v[2] - u[2] * v[1];
  nrm[1] = u[2] * v[0] - u[0] * v[2];
  nrm[2] = u[0] * v[1] - u[1] * v[0];
  const double nn = std::sqrt(dot(nrm, nrm, 3));
  double best = std::min(seg_d2(a, b, p, 3), std::min(seg_d2(b, c, p, 3), seg_d2(c, a, p, 3)));
  if (nn > 0) {
    for (int k = 0; k < 3; ++k) nrm[k] /= nn;
    double s = 0, q[3];
    for (int k = 0; k < 3; ++k) s += (p[k] - a[k]) * nrm[k];
    for (int k = 0; k < 3; ++k) q[k] = p[k] - s * nrm[k];
    auto side = [&](const double* x, const double* y) {
      double e[3], w[3];
      for (int k = 0; k < 3; ++k) {
        e[k] = y[k] - x[k];
        w[k] = q[k] - x[k];
      }
      const double cx = e[1] * w[2] - e[2] * w[1], cy = e[2] * w[0] - e[0] * w[2], cz = e[0] * w[1] - e[1] * w[0];
      return cx * nrm[0] + cy * nrm[1] + cz * nrm[2];
    };
    if (side(a, b) >= 0 && side(b, c) >= 0 && side(c, a) >= 0) best = std::min(best, s * s);
  }
  return best;
}

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  const bool tri = argv[1][0] == 't';
  const int dim = tri ? 3 : 2, stride = tri ? 12 : 4, nv = tri ? 3 : 2;
  FILE* f = std::fopen(argv[2], "rb");
  if (!f) return 2;
  std::vector<double> raw;
  double buf[12];
  while (std::fread(buf, sizeof(double), stride, f) == (size_t)stride) raw.insert(raw.end(), buf, buf + stride);
  std::fclose(f);
  const int64_t n = (int64_t)raw.size() / stride;
  std::vector<double> lo(n * dim), hi(n * dim), cen(n * dim);
  for (int64_t j = 0; j < n; ++j)
    for (int k = 0; k < dim; ++k) {
      double mn = 1e300, mx = -1e300, s = 0;
      for (int v = 0; v < nv; ++v) {
        const double c = raw[stride * j + dim * v + k];
        mn = std::min(mn, c);
        mx = std::max(mx, c);
        s += c;
      }
      lo[j * dim + k] = mn;
      hi[j * dim + k] = mx;
      cen[j * dim + k] = s / nv;
    }
  const BvhTopology t = build_bvh(lo, hi, cen, dim, n, 4);
  std::vector<double> prims(n * stride), plo(n * dim), phi(n * dim), bounds;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t s = t.order[i];
    for (int k = 0; k < stride; ++k) prims[stride * i + k] = raw[stride * s + k];
    for (int k = 0; k < dim; ++k) {
      plo[dim * i + k] = lo[dim * s + k];
      phi[dim * i + k] = hi[dim * s + k];
    }
  }
  bvh_child_bounds<double>(t, plo, phi, dim, bounds);
  const double margin = 1e-9;
  SegmentGrid g, g1;
  if (tri) {
    g = build_triangle_grid(prims, n, t, bounds, 16 * n, margin, 6, 4);
    g1 = build_triangle_grid(prims, n, t, bounds, 16 * n, margin, 6, 1);
  } else {
    // a small cap, so that long lists are truncated
    g = build_segment_grid(prims, n, t, bounds, 16 * n, margin, 8, 4);
    g1 = g;
  }
  const bool same = g.start == g1.start && g.prim == g1.prim && g.dc == g1.dc && g.tail == g1.tail;
  const int nn[3] = {g.nx, g.ny, g.nz};
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  int64_t points = 0, exact = 0, bounded = 0, bad_exact = 0, bad_bound = 0;
  const int64_t ncell = (int64_t)g.nx * g.ny * (tri ? g.nz : 1);
  for (int64_t c = 0; c < ncell; c += tri ? 7 : 1) {
    const int64_t idx[3] = {c % g.nx, (c / g.nx) % g.ny, tri ? c / ((int64_t)g.nx * g.ny) : 0};
    const uint32_t st = g.start[c], cnt = g.start[c + 1] - st;
    if (cnt == 0) continue;
    double p[3], o[3];
    for (int k = 0; k < dim; ++k) {
      p[k] = g.lo[k] + (idx[k] + U(rng)) * g.h;
      o[k] = p[k] - (g.lo[k] + (idx[k] + 0.5) * g.h);
    }
    const double r_pc = std::sqrt(dot(o, o, dim));
    double best = 1e300;
    uint32_t k = 0;
    for (; k < cnt; ++k) {
      const double lim = g.dc[st + k] - margin - r_pc;
      if (lim > 0 && lim * lim >= best) break;
      const double* q = &prims[(size_t)stride * g.prim[st + k]];
      best = std::min(best, tri ? tri_d2(q, p) : seg_d2(q, q + 2, p, 2));
    }
    double truth = 1e300;
    for (int64_t j = 0; j < n; ++j) {
      const double* q = &prims[(size_t)stride * j];
      truth = std::min(truth, tri ? tri_d2(q, p) : seg_d2(q, q + 2, p, 2));
    }
    const double d = std::sqrt(best), dt = std::sqrt(truth);
    const double lb = std::isfinite(g.tail[c]) ? g.tail[c] - margin - r_pc : HUGE_VAL;
    ++points;
    if (k < cnt || d <= lb) {
      ++exact;
      if (std::fabs(d - dt) > 1e-12) ++bad_exact;
    } else {
      ++bounded;
      if (lb > dt + 1e-12) ++bad_bound;
    }
  }
  std::printf("points %lld exact %lld bounded %lld bad_exact %lld bad_bound %lld threads_equal %d cells %lld\n",
              (long long)points, (long long)exact, (long long)bounded, (long long)bad_exact, (long long)bad_bound,
              same ? 1 : 0, (long long)ncell);
  return 0;
}
