#include "bvh.h"

#include <algorithm>
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
