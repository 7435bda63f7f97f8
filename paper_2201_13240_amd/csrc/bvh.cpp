#include "bvh.h"

#include <algorithm>
#include <cmath>
#include <exception>
#include <functional>
#include <limits>
#include <thread>

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

double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

double seg3_dist2(const double* a, const double* b, const double* p) {
  double e[3], q[3];
  for (int k = 0; k < 3; ++k) {
    e[k] = b[k] - a[k];
    q[k] = p[k] - a[k];
  }
  const double l2 = dot3(e, e);
  double t = l2 > 0 ? dot3(q, e) / l2 : 0.0;
  t = std::min(1.0, std::max(0.0, t));
  for (int k = 0; k < 3; ++k) q[k] -= t * e[k];
  return dot3(q, q);
}

// Squared distance from p to triangle (a, b, c): the plane distance when the projection
// of p falls inside the triangle (barycentric coordinates from the Gram system of the
// two edges at a), else the nearest of the three edges.
double tri_dist2(const double* t, const double* p) {
  const double *a = t, *b = t + 3, *c = t + 6;
  double e0[3], e1[3], ap[3];
  for (int k = 0; k < 3; ++k) {
    e0[k] = b[k] - a[k];
    e1[k] = c[k] - a[k];
    ap[k] = p[k] - a[k];
  }
  const double d00 = dot3(e0, e0), d01 = dot3(e0, e1), d11 = dot3(e1, e1);
  const double den = d00 * d11 - d01 * d01;
  if (den > 0) {
    const double d20 = dot3(ap, e0), d21 = dot3(ap, e1);
    const double v = (d11 * d20 - d01 * d21) / den, w = (d00 * d21 - d01 * d20) / den;
    if (v >= 0 && w >= 0 && v + w <= 1) {
      double q[3];
      for (int k = 0; k < 3; ++k) q[k] = ap[k] - v * e0[k] - w * e1[k];
      return dot3(q, q);
    }
  }
  return std::min(seg3_dist2(a, b, p), std::min(seg3_dist2(b, c, p), seg3_dist2(c, a, p)));
}

double box3_d2(const double* lo, const double* hi, const double* p) {
  double s = 0;
  for (int k = 0; k < 3; ++k) {
    const double e = std::max(std::max(lo[k] - p[k], p[k] - hi[k]), 0.0);
    s += e * e;
  }
  return s;
}

struct TriQuery {
  const std::vector<double>& tris;
  const BvhTopology& topo;
  const std::vector<double>& bounds;

  // visits leaf triangles whose subtree box lies within sqrt(*r2) of p, nearer boxes
  // first; f returns false to stop the whole traversal (then within returns false)
  template <typename F>
  bool within(int32_t c, const double* p, const double* r2, F&& f) const {
    if (c < 0) {
      const int32_t code = -1 - c;
      const int32_t first = code >> 3, cnt = code & 7;
      for (int32_t i = first; i < first + cnt; ++i)
        if (!f(i, tri_dist2(&tris[12 * (size_t)i], p))) return false;
      return true;
    }
    const double* b = &bounds[(size_t)c * 12];  // lo[2][3], hi[2][3]
    const double da = box3_d2(b + 0, b + 6, p), db = box3_d2(b + 3, b + 9, p);
    const int32_t ca = topo.child[2 * c], cb = topo.child[2 * c + 1];
    const bool a_first = da <= db;
    const int32_t c0 = a_first ? ca : cb, c1 = a_first ? cb : ca;
    const double d0 = a_first ? da : db, d1 = a_first ? db : da;
    if (d0 <= *r2 && !within(c0, p, r2, f)) return false;
    if (d1 <= *r2 && !within(c1, p, r2, f)) return false;
    return true;
  }
};

}  // namespace

SegmentGrid build_segment_grid(const std::vector<double>& segs, int64_t n, const BvhTopology& topo,
                               const std::vector<double>& bounds, int64_t target_cells, double margin,
                               int max_candidates, int deep_list) {
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
  double h = std::sqrt((ex + 2 * pad) * (ey + 2 * pad) / (double)target_cells);
  // a nearly flat set (degenerate input) would make the cells tiny: coarsen until the
  // grid holds at most twice the target
  while (std::max(1.0, std::ceil((ex + 2 * pad) / h)) * std::max(1.0, std::ceil((ey + 2 * pad) / h)) >
         2.0 * (double)target_cells)
    h *= 1.25;
  g.nx = std::max(1, (int32_t)std::ceil((ex + 2 * pad) / h));
  g.ny = std::max(1, (int32_t)std::ceil((ey + 2 * pad) / h));
  g.lo[0] = lo[0];
  g.lo[1] = lo[1];
  g.h = h;
  const double halfdiag = 0.5 * h * std::sqrt(2.0);
  SegQuery q{segs, topo, bounds};
  const int64_t ncell = (int64_t)g.nx * g.ny;
  g.start.resize(ncell + 1);
  g.tail.assign(ncell, HUGE_VAL);
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
      std::sort(cand.begin(), cand.end());
      // a list too long keeps its deep_list nearest candidates and the tail distance
      const size_t n_keep = cand.size() <= (size_t)max_candidates ? cand.size() : (size_t)deep_list;
      for (size_t e = 0; e < n_keep; ++e) {
        g.prim.push_back(cand[e].second);
        g.dc.push_back(std::sqrt(cand[e].first));
      }
      g.tail[(int64_t)j * g.nx + i] = n_keep < cand.size() ? std::sqrt(cand[n_keep].first) : HUGE_VAL;
      g.start[(int64_t)j * g.nx + i + 1] = (uint32_t)g.prim.size();
    }
  return g;
}

SegmentGrid build_triangle_grid(const std::vector<double>& tris, int64_t n, const BvhTopology& topo,
                                const std::vector<double>& bounds, int64_t target_cells, double margin,
                                int max_candidates, int threads) {
  SegmentGrid g;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = 0; i < n; ++i)
    for (int v = 0; v < 3; ++v)
      for (int k = 0; k < 3; ++k) {
        lo[k] = std::min(lo[k], tris[12 * i + 3 * v + k]);
        hi[k] = std::max(hi[k], tris[12 * i + 3 * v + k]);
      }
  double ext = 0, vol = 1;
  for (int k = 0; k < 3; ++k) ext = std::max(ext, hi[k] - lo[k]);
  const double pad = 1e-6 * ext + 1e-12;
  for (int k = 0; k < 3; ++k) {
    lo[k] -= pad;
    vol *= hi[k] - lo[k] + pad;
  }
  // a nearly flat set (degenerate input) would make the cells tiny: coarsen until the
  // grid holds at most twice the target
  double h = std::cbrt(vol / (double)target_cells);
  auto n_cells = [&](double hh) {
    double c = 1;
    for (int k = 0; k < 3; ++k) c *= std::max(1.0, std::ceil((hi[k] - lo[k] + pad) / hh));
    return c;
  };
  while (n_cells(h) > 2.0 * (double)target_cells) h *= 1.25;
  int32_t nn[3];
  for (int k = 0; k < 3; ++k) {
    nn[k] = std::max(1, (int32_t)std::ceil((hi[k] - lo[k] + pad) / h));
    g.lo[k] = lo[k];
  }
  g.nx = nn[0];
  g.ny = nn[1];
  g.nz = nn[2];
  g.h = h;
  const double halfdiag = 0.5 * h * std::sqrt(3.0);
  const double deep = 8 * h;
  const TriQuery q{tris, topo, bounds};
  const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
  threads = (int)std::max<int64_t>(1, std::min<int64_t>(threads, (ncell + 4095) / 4096));
  struct Part {
    std::vector<uint32_t> count;
    std::vector<int32_t> prim;
    std::vector<double> dc, tail;
  };
  std::vector<Part> parts(threads);
  auto work = [&](int t) {
    Part& P = parts[t];
    const int64_t c0 = ncell * t / threads, c1 = ncell * (t + 1) / threads;
    P.count.resize(c1 - c0);
    P.tail.resize(c1 - c0);
    std::vector<std::pair<double, int32_t>> heap;   // max-heap of the kept candidates
    const size_t keep = (size_t)max_candidates + 1;
    int32_t prev = -1;   // nearest triangle of the previous cell: seeds the search bound
    for (int64_t c = c0; c < c1; ++c) {
      const int64_t i = c % g.nx, j = (c / g.nx) % g.ny, k = c / ((int64_t)g.nx * g.ny);
      const double p[3] = {lo[0] + (i + 0.5) * h, lo[1] + (j + 0.5) * h, lo[2] + (k + 0.5) * h};
      double best = prev >= 0 ? tri_dist2(&tris[12 * (size_t)prev], p) : 1e300;
      q.within(topo.root, p, &best, [&](int32_t s, double d2) {
        if (d2 < best) {
          best = d2;
          prev = s;
        }
        return true;
      });
      if (std::sqrt(best) >= deep) {
        // deep inside many triangles are nearly equidistant and a list could not decide
        // anyway: keep the nearest one alone, with its distance as the tail (no
        // triangle is nearer to the centre)
        P.prim.push_back(prev);
        P.dc.push_back(std::sqrt(best));
        P.count[c - c0] = 1;
        P.tail[c - c0] = std::sqrt(best);
        continue;
      }
      const double r = std::sqrt(best) + 2 * halfdiag + margin;
      // the max_candidates + 1 nearest triangles within r of the centre; the bound
      // shrinks to the farthest kept one once the heap is full
      double r2 = r * r;
      heap.clear();
      q.within(topo.root, p, &r2, [&](int32_t s, double d2) {
        if (d2 > r2) return true;
        if (heap.size() == keep) {
          std::pop_heap(heap.begin(), heap.end());
          heap.pop_back();
        }
        heap.emplace_back(d2, s);
        std::push_heap(heap.begin(), heap.end());
        if (heap.size() == keep) r2 = heap.front().first;
        return true;
      });
      std::sort(heap.begin(), heap.end());
      const size_t n_keep = std::min(heap.size(), (size_t)max_candidates);
      for (size_t e = 0; e < n_keep; ++e) {
        P.prim.push_back(heap[e].second);
        P.dc.push_back(std::sqrt(heap[e].first));
      }
      P.count[c - c0] = (uint32_t)n_keep;
      P.tail[c - c0] = heap.size() > n_keep ? std::sqrt(heap[n_keep].first) : HUGE_VAL;
    }
  };
  // an exception inside a worker (a failed allocation) is carried to this thread and
  // rethrown after every worker has been joined; parts whose thread could not be started
  // run here
  std::vector<std::exception_ptr> errors(threads);
  auto run = [&](int t) {
    try {
      work(t);
    } catch (...) {
      errors[t] = std::current_exception();
    }
  };
  std::vector<std::thread> pool;
  int started = 1;
  try {
    pool.reserve(threads);
    for (; started < threads; ++started) pool.emplace_back(run, started);
  } catch (...) {
  }
  run(0);
  for (int t = started; t < threads; ++t) run(t);
  for (auto& th : pool) th.join();
  for (const std::exception_ptr& e : errors)
    if (e) std::rethrow_exception(e);
  g.start.resize(ncell + 1);
  g.tail.resize(ncell);
  g.start[0] = 0;
  int64_t c = 0;
  for (const Part& P : parts) {
    for (size_t e = 0; e < P.count.size(); ++e) {
      g.start[c + 1] = g.start[c] + P.count[e];
      g.tail[c] = P.tail[e];
      ++c;
    }
    g.prim.insert(g.prim.end(), P.prim.begin(), P.prim.end());
    g.dc.insert(g.dc.end(), P.dc.begin(), P.dc.end());
  }
  return g;
}

}  // namespace wos
