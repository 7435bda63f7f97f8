// Host construction of the axis-aligned BVH used for closest-point queries (Sec. 7.1).
#pragma once
#include <cstdint>
#include <vector>

namespace wos {

struct BvhTopology {
  std::vector<int32_t> order;                 // primitive permutation (leaf order)
  std::vector<int32_t> child;                 // [n_nodes][2], device child encoding
  int32_t root = 0;
  int32_t depth = 0;
};

// Median split on the longest axis of the primitive centroids, leaves of at most
// `leaf_size` (<= 7) primitives. lo/hi/centroid: [n][dim].
BvhTopology build_bvh(const std::vector<double>& lo, const std::vector<double>& hi,
                      const std::vector<double>& centroid, int dim, int64_t n, int leaf_size);

// Child bounds of every inner node from per-primitive bounds (given in leaf order) in
// the precision of the walker. out: [n_nodes][2][2][dim] as lo[2][dim], hi[2][dim].
template <typename T>
void bvh_child_bounds(const BvhTopology& t, const std::vector<T>& plo, const std::vector<T>& phi, int dim,
                      std::vector<T>& out);

}  // namespace wos
