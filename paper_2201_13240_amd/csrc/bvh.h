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

namespace wos {

// Uniform grid over the bounding box of a 2D segment set or a 3D triangle set. Cell c
// lists every primitive within d(center_c) + 2 * halfdiag + margin of its centre, a
// superset of the primitives that can be nearest to any point of the cell (or within
// `margin` of it): for p in the cell and s* nearest to p,
// |c - s*| <= |p - s*| + halfdiag <= d(c) + 2 halfdiag.
struct SegmentGrid {
  int32_t nx = 0, ny = 0, nz = 1;
  double lo[3] = {0, 0, 0};
  double h = 0;
  std::vector<uint32_t> start;   // [nx * ny * nz + 1], cell (i, j, k) at (k * ny + j) * nx + i
  std::vector<int32_t> prim;     // candidate indices (leaf order), nearest to the cell centre first
  std::vector<double> dc;        // distance from the cell centre to each candidate (ascending per cell)
  std::vector<double> tail;      // per cell, the centre distance of the nearest candidate left
                                 // off its list (+inf: the list is complete)
};

// segs: [n][4] in leaf order; topo/bounds: the BVH over them (child bounds as produced
// by bvh_child_bounds<double>). target_cells bounds the grid size. Each list is sorted by
// distance from the cell centre, so a query at p can stop once dc - |p - centre| exceeds
// its best distance (triangle inequality). A cell with more than max_candidates
// candidates keeps only the deep_list nearest ones and records in `tail` the centre
// distance of the first one left off (+inf for complete lists): every omitted segment
// lies at least tail - |p - centre| from p.
SegmentGrid build_segment_grid(const std::vector<double>& segs, int64_t n, const BvhTopology& topo,
                               const std::vector<double>& bounds, int64_t target_cells, double margin,
                               int max_candidates, int deep_list);

// The same for triangles: tris [n][12] (a, b, c, padding) in leaf order, a 3D grid of
// cubic cells. A cell keeps at most max_candidates of its candidates, the nearest to its
// centre, and records in `tail` the centre distance of the first one left off: for p in
// the cell every omitted triangle lies at least tail - |p - centre| from p, so a scan of
// the kept list either finds the nearest triangle or a lower bound of the distance. A
// cell whose centre lies 8 cell widths or more from the surface keeps only its nearest
// triangle, with tail = its distance.
// Cells are filled by up to `threads` host threads; the result does not depend on their
// number.
SegmentGrid build_triangle_grid(const std::vector<double>& tris, int64_t n, const BvhTopology& topo,
                                const std::vector<double>& bounds, int64_t target_cells, double margin,
                                int max_candidates, int threads);

}  // namespace wos
