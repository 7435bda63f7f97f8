#include "bvh.h"

#include <algorithm>
#include <cmath>
#include <functional>
#include <limits>

namespace wos {

BvhTopology build_bvh(const std::vector<double>& lo, const std::vector<double>& hi,
                      const std::vector<double>& centroid, int dim, int64_t n, int leaf_size) {
  (void)lo;
  (void)hi;
  BvhTopology t;
  t.order.resize(n);
  for (int64_t i = 0; i < n; ++i) t.order[i] = (int32_t)i;
  std::function<int32_t(int64_t, int64_t, int)> rec = [&](int64_t b, int64_t e, int d) -> int32_t {
    t.depth = std::max(t.depth, d);
    const int64_t cnt = e - b;
    if (cnt <= leaf_size) return -1 - (int32_t)((b << 3) | cnt);
    double cmin[3] = {1e300, 1e300, 1e300}, cmax[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = b; i < e; ++i)
      for (int k = 0; k < dim; ++k) {
        const double c = centroid[(size_t)t.order[i] * dim + k];
        cmin[k] = std::min(cmin[k], c);
        cmax[k] = std::max(cmax[k], c);
      }
    int axis = 0;
    for (int k = 1; k < dim; ++k)
      if (cmax[k] - cmin[k] > cmax[axis] - cmin[axis]) axis = k;
    const int64_t mid = b + cnt / 2;
    std::nth_element(t.order.begin() + b, t.order.begin() + mid, t.order.begin() + e, [&](int32_t a, int32_t c) {
      const double ca = centroid[(size_t)a * dim + axis], cc = centroid[(size_t)c * dim + axis];
      return ca < cc || (ca == cc && a < c);
    });
    const int32_t idx = (int32_t)(t.child.size() / 2);
    t.child.push_back(0);
    t.child.push_back(0);
    const int32_t l = rec(b, mid, d + 1);
    const int32_t r = rec(mid, e, d + 1);
    t.child[2 * idx] = l;
    t.child[2 * idx + 1] = r;
    return idx;
  };
  t.root = rec(0, n, 0);
  return t;
}

template <typename T>
void bvh_child_bounds(const BvhTopology& t, const std::vector<T>& plo, const std::vector<T>& phi, int dim,
                      std::vector<T>& out) {
  const size_t n_nodes = t.child.size() / 2;
  out.assign(n_nodes * 4 * dim, (T)0);
  // bounds of a child reference (recursive, post-order)
  std::function<void(int32_t, T*, T*)> bounds = [&](int32_t c, T* blo, T* bhi) {
    for (int k = 0; k < dim; ++k) {
      blo[k] = std::numeric_limits<T>::infinity();
      bhi[k] = -std::numeric_limits<T>::infinity();
    }
    if (c < 0) {
      const int32_t code = -1 - c;
      const int32_t first = code >> 3, cnt = code & 7;
      for (int32_t i = first; i < first + cnt; ++i)
        for (int k = 0; k < dim; ++k) {
          blo[k] = std::min(blo[k], plo[(size_t)i * dim + k]);
          bhi[k] = std::max(bhi[k], phi[(size_t)i * dim + k]);
        }
      return;
    }
    T* node = out.data() + (size_t)c * 4 * dim;  // lo[0][dim], lo[1][dim], hi[0][dim], hi[1][dim]
    for (int s = 0; s < 2; ++s) {
      T clo[3], chi[3];
      bounds(t.child[2 * c + s], clo, chi);
      for (int k = 0; k < dim; ++k) {
        node[s * dim + k] = clo[k];
        node[2 * dim + s * dim + k] = chi[k];
        blo[k] = std::min(blo[k], clo[k]);
        bhi[k] = std::max(bhi[k], chi[k]);
      }
    }
  };
  T rlo[3], rhi[3];
  bounds(t.root, rlo, rhi);
}

template void bvh_child_bounds<float>(const BvhTopology&, const std::vector<float>&, const std::vector<float>&, int,
                                      std::vector<float>&);
template void bvh_child_bounds<double>(const BvhTopology&, const std::vector<double>&, const std::vector<double>&,
                                       int, std::vector<double>&);

}  // namespace wos

namespace wos {

namespace {

double seg_dist2(const double* s, double px, double py) {
  const double ex = s[2] - s[0], ey = s[3] - s[1];
  const double qx = px - s[0], qy = py - s[1];
  const double l2 = ex * ex + ey * ey;
  double t = l2 > 0 ? (qx * ex + qy * ey) / l2 : 0.0;
  t = std::min(1.0, std::max(0.0, t));
  const double dx = qx - t * ex, dy = qy - t * ey;
  return dx * dx + dy * dy;
}

double box_d2(const double* lo, const double* hi, double px, double py) {
  const double ex = std::max(std::max(lo[0] - px, px - hi[0]), 0.0);
  const double ey = std::max(std::max(lo[1] - py, py - hi[1]), 0.0);
  return ex * ex + ey * ey;
}

struct SegQuery {
  const std::vector<double>& segs;
  const BvhTopology& topo;
  const std::vector<double>& bounds;

  // visits every leaf segment whose subtree box lies within sqrt(r2) of (px, py)
  template <typename F>
  void within(int32_t c, double px, double py, const double* r2, F&& f) const {
    if (c < 0) {
      const int32_t code = -1 - c;
      const int32_t first = code >> 3, cnt = code & 7;
      for (int32_t i = first; i < first + cnt; ++i) f(i, seg_dist2(&segs[4 * (size_t)i], px, py));
      return;
    }
    const double* b = &bounds[(size_t)c * 8];  // lo[2][2], hi[2][2]
    const double da = box_d2(b + 0, b + 4, px, py), db = box_d2(b + 2, b + 6, px, py);
    const int32_t ca = topo.child[2 * c], cb = topo.child[2 * c + 1];
    if (da <= db) {
      if (da <= *r2) within(ca, px, py, r2, f);
      if (db <= *r2) within(cb, px, py, r2, f);
    } else {
      if (db <= *r2) within(cb, px, py, r2, f);
      if (da <= *r2) within(ca, px, py, r2, f);
    }
  }
};

}  // namespace

SegmentGrid build_segment_grid(const std::vector<double>& segs, int64_t n, const BvhTopology& topo,
                               const std::vector<double>& bounds, int64_t target_cells, double margin,
                               int max_candidates) {
  SegmentGrid g;
  double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
  for (int64_t i = 0; i < n; ++i)
    for (int v = 0; v < 2; ++v)
      for (int k = 0; k < 2; ++k) {
        lo[k] = std::min(lo[k], segs[4 * i + 2 * v + k]);
        hi[k] = std::max(hi[k], segs[4 * i + 2 * v + k]);
      }
  const double ex = hi[0] - lo[0], ey = hi[1] - lo[1];
  const double pad = 1e-6 * std::max(ex, ey) + 1e-12;
  lo[0] -= pad;
  lo[1] -= pad;
  const double h = std::sqrt((ex + 2 * pad) * (ey + 2 * pad) / (double)target_cells);
  g.nx = std::max(1, (int32_t)std::ceil((ex + 2 * pad) / h));
  g.ny = std::max(1, (int32_t)std::ceil((ey + 2 * pad) / h));
  g.lo[0] = lo[0];
  g.lo[1] = lo[1];
  g.h = h;
  const double halfdiag = 0.5 * h * std::sqrt(2.0);
  SegQuery q{segs, topo, bounds};
  const int64_t ncell = (int64_t)g.nx * g.ny;
  g.start.resize(ncell + 1);
  g.start[0] = 0;
  for (int32_t j = 0; j < g.ny; ++j)
    for (int32_t i = 0; i < g.nx; ++i) {
      const double cx = lo[0] + (i + 0.5) * h, cy = lo[1] + (j + 0.5) * h;
      double best = 1e300;
      q.within(topo.root, cx, cy, &best, [&](int32_t, double d2) { best = std::min(best, d2); });
      const double r = std::sqrt(best) + 2 * halfdiag + margin;
      const double r2 = r * r;
      std::vector<std::pair<double, int32_t>> cand;
      q.within(topo.root, cx, cy, &r2, [&](int32_t s, double d2) {
        if (d2 <= r2) cand.emplace_back(d2, s);
      });
      if (cand.size() <= (size_t)max_candidates) {   // else an empty list: use the BVH
        std::sort(cand.begin(), cand.end());
        for (const auto& c : cand) {
          g.prim.push_back(c.second);
          g.dc.push_back(std::sqrt(c.first));
        }
      }
      g.start[(int64_t)j * g.nx + i + 1] = (uint32_t)g.prim.size();
    }
  return g;
}

}  // namespace wos
