// Device-side data layout of a compiled problem (shared by host set-up and kernels).
#pragma once
#include <cstdint>

namespace wos {

enum FieldBase : int32_t { FB_NONE = 0, FB_FOURIER = 1, FB_BUMPS = 2, FB_TANH = 3, FB_TANH_DRIFT = 4, FB_MANUFACTURED = 5 };
enum FieldTransform : int32_t { FT_AFFINE = 0, FT_EXP = 1 };
enum GeomKind : int32_t { GK_BALL = 0, GK_BOX = 1, GK_POLYGON = 2, GK_TRIMESH = 3, GK_SDF = 4 };
// CSG row of an SDF domain: op (0 union, 1 intersection, 2 subtraction), shape (0 ball,
// 1 box, 2 half-space), c[3], p[3]; half-space normals are stored unit length.
constexpr int kSdfStride = 8;
enum SolutionId : int32_t { SOL_EXPCOS = 1, SOL_QUADRATIC = 2 };

// Eight numbers per term, in the precision of the walker:
//   fourier: k0, k1, k2 (cycles per unit length), a cos(phi), a sin(phi), |2 pi k|^2, a,
//            phi / (2 pi): a cos(2 pi k.x + phi) = ac cos(th) - as sin(th) with
//            th = 2 pi k.x where derivatives are needed, a cos(2 pi (k.x + phi / 2 pi))
//            (one cosine) for the value alone
//   bumps:   c0, c1, c2, log2(e)/(2 w^2) (for exp2), amp, 1/w^2 (the last two unused)
constexpr int kTermStride = 8;

template <typename T>
struct DevField {
  int32_t base;
  int32_t transform;
  int32_t n;         // number of terms
  int32_t sol;       // manufactured solution id
  T c0, c1;          // value = c0 + c1 B  or  exp(c0 + c1 B)
  const T* terms;    // [n][kTermStride]
  T prm[8];          // tanh: axis, x0, 1/width ; tanh_drift: axis, x0, 1/width, A, B, omega*width/(A^2-B^2), ln A, omega
};

constexpr int kCellInline = 7;
// Length of the candidate lists of the triangle-mesh grid, and of the truncated lists
// of polygon grid cells with more than kPolygonCellMax candidates.
constexpr int kMeshCellList = 6;
constexpr int kPolygonCellMax = 32;
constexpr int kPolygonDeepList = 16;

// One cell of the polygon candidate grid: `count` candidates at cell_prim / cell_segs /
// cell_dc [start, start + count), the first kCellInline also held here as start point,
// edge vector and reciprocal squared length (x0, y0, ex, ey), 1/|e|^2, so that their
// distance needs no division (a shorter list is padded with copies of its last
// candidate). `tail` bounds from below the centre distance of every segment left off a
// truncated list (+inf: the list is complete).
template <typename T>
struct __attribute__((aligned(16))) CellRec {
  uint32_t count;
  uint32_t start;
  union {
    T tail;
    uint32_t pad[2];
  };
  T seg[kCellInline][4];
  T inv_len2[kCellInline];
};

// One cell of the triangle-mesh candidate grid: `count` candidates at cell_prim /
// cell_dc [start, start + count), and `tail`, a lower bound of the centre distance of
// every triangle left off the list (+inf: none was).
template <typename T>
struct __attribute__((aligned(16))) MeshCell {
  uint32_t count;
  uint32_t start;
  T tail;
};

// Binary BVH node that stores the bounds of both children, so a visit tests both
// boxes with one load. A child reference c >= 0 is an inner node index; c < 0 encodes
// a leaf: -1 - c = (first primitive << 3) | count, count in 1..7.
template <typename T, int DIM>
struct BvhNode {
  T lo[2][DIM];
  T hi[2][DIM];
  int32_t child[2];
};

template <typename T>
struct DevGeometry {
  int32_t kind;
  int32_t n_prims;
  int32_t n_nodes;
  int32_t root;          // root child reference (same encoding as BvhNode::child)
  int32_t depth;         // deepest inner node level (root = 0) plus one
  int32_t pad;
  T center[3];
  T radius;
  T lo[3];
  T hi[3];
  const void* nodes;     // BvhNode<T, DIM>[n_nodes]
  const T* prims;        // polygon: [n][4] (x0, y0, x1, y1); trimesh: [n][12] (a, b, c, padding);
                         // SDF: [n][kSdfStride] CSG rows
  // Uniform candidate grid of polygons and triangle meshes (grid_nx = 0: none). Cell
  // (i, j[, k]) covers [grid_lo + (i, j, k) h, grid_lo + (i + 1, j + 1, k + 1) h]; its
  // candidates are cell_prim[start .. start + count), nearest to the cell centre first;
  // cell_dc holds a lower bound of each one's distance from the centre (the distance
  // minus the rounding margin).
  // Polygons: cells[c] is a CellRec with the list's length and start and a copy of its
  // first kCellInline segments, so most queries read one record; cell_segs holds the
  // segments of the whole list. Meshes: cells[c] is a MeshCell, cell (i, j, k) at
  // (k ny + j) nx + i, and cell_prim holds triangle indices.
  int32_t grid_nx, grid_ny, grid_nz;
  int32_t grid_pad;
  T grid_lo[3];
  T grid_inv_h;
  T grid_h;
  T grid_lb_min;         // smallest lower bound a walk step may take (> 2 epsilon)
  const void* cells;     // CellRec<T>[nx * ny] or MeshCell<T>[nx * ny * nz]
  const int32_t* cell_prim;
  const T* cell_segs;
  const T* cell_dc;
};

// Dense trigonometric table of the 2D Fourier fields (alpha, psi and sigma: slots 0, 1,
// 2) with integer wave vectors |k_i| <= 3, in product form. With the bases
//   psi_a(x) = 1, cos 2 pi x, sin 2 pi x, cos 4 pi x, sin 4 pi x, cos 6 pi x, sin 6 pi x
// (a = 0 .. 6) and phi_b(y) the same in y, the base of a slot is
//   B(x, y) = sum_{a, b} M[a][b] psi_a(x) phi_b(y),
// which holds every mode a cos(2 pi k.x + phi) with |k_i| <= 3 and the constant. m[a][slot]
// holds row a of M (kind 0) and the same row of the matrices of dB/dy (kind 1) and
// d2B/dy2 (kind 2), so that each is one dot product with phi per row.
constexpr int kSpecK = 3;
constexpr int kSpecGammaMerged = 8;
constexpr int kSpecRow = 2 * kSpecK + 1;   // basis functions per variable

template <typename T>
struct Spectral2D {
  T m[kSpecRow][3][3][kSpecRow];
};

template <typename T>
struct DevProblem {
  int32_t dim;
  int32_t spectral;        // bit s set: field slot s (alpha, psi, sigma) is in `spec`; with
                           // kSpecGammaMerged, slot 0 holds gamma and slot 1 the base of alpha
  DevGeometry<T> geom;
  DevField<T> alpha, psi, sigma, source, boundary;
  T epsilon;
  T sigma_bar;
  T inv_sigma_bar;
  T sqrt_sigma_bar;
  Spectral2D<T> spec;
};

// One query batch of a launch (device copy). Walk j of point p is walk (p, j); the
// item's walks are cut into tiles in point-major order: with tiles_per_point > 0 every
// point takes that many tiles of tile_len walks (the last one may be shorter), otherwise
// a tile takes points_per_tile whole points. A wavefront runs every walk of a tile it
// takes. Each (tile, point) pair owns one accumulation slot; the slots of point p are
// slot_base + p * max(1, tiles_per_point) + k for its k-th tile.
struct DevItem {
  const void* problem;       // DevProblem<T>* in the walker's precision
  const double* points;      // [n_points][dim]
  const int8_t* inside;      // [n_points] classification (1 = interior)
  double* sum;
  double* sum_sq;
  uint64_t* n_walks;
  uint64_t* n_steps;
  uint64_t* counters;        // [4] or null
  int64_t n_points;
  uint64_t walks;            // walks per point in this launch
  uint64_t walk_offset;      // first global walk index of this launch
  uint64_t point_base;       // offset of this item in the launch's point space
  uint32_t problem_index;
  uint32_t tile_len;         // walks per tile when tiles_per_point > 0
  double* grad_sum;          // [n_points][dim] or null
  double* grad_sum_sq;
  const void* gamma0;        // [n_points] gamma at each interior query point, walker precision
  uint64_t tile_base;        // index of the item's first tile in the launch
  uint64_t n_tiles;          // tiles of this item
  uint64_t slot_base;        // first accumulation slot of this item
  uint32_t tiles_per_point;
  uint32_t points_per_tile;  // used when tiles_per_point == 0
};

// Per-(tile, point) accumulation slot, in 64-bit words. Sums of per-walk estimates are
// kept exactly, as fixed-point numbers: v 2^96 is cut into 32-bit chunks of weight
// 2^(32k - 96), k = 0..5, and chunk k is added to limb k with an integer atomic. Integer
// addition is associative, so a slot's content does not depend on the order in which
// the walks of its tile finish, and results are reproducible bit for bit whatever the
// launch shape. A double has 53 significant bits, so a walk touches at most three limbs
// per sum. Per-walk estimates are limited to |v| < 2^47 (then v^2 < 2^94 fits the top
// limb); a larger or non-finite one is counted in the `bad` field and makes the
// point's sums NaN.
constexpr int kFxLimbs = 6;
constexpr int kFxFracBits = 96;
constexpr double kFxMaxValue = 140737488355328.0;   // 2^47
constexpr int kSlotSum = 0;       // [kFxLimbs] limbs of the sum of estimates
constexpr int kSlotSumSq = 6;     // [kFxLimbs] limbs of the sum of their squares
constexpr int kSlotSteps = 12;    // distance queries
constexpr int kSlotFlags = 13;    // walks cut at max_steps | roulette kills << 21 | bad << 42
constexpr int kSlotGrad = 16;     // per gradient component c: [kFxLimbs] sum, [kFxLimbs] sum of squares
constexpr int kFlagShiftKilled = 21;
constexpr int kFlagShiftBad = 42;
constexpr uint32_t kMaxTileLen = 65536;   // keeps a slot's limbs below 2^49 before carries
// Words per slot (a multiple of 16: 128 bytes, one cache line).
inline constexpr int slot_words(int grad_dim) { return grad_dim ? (kSlotGrad + 2 * kFxLimbs * grad_dim + 15) / 16 * 16 : 16; }

// Per-walk record of the gradient estimate (supplemental Sec. 2), in the walker's
// precision: [A0, a (dim), b (dim), grad gamma(x0) (dim)]. One record per lane of the
// persistent grid (a lane runs one walk at a time); it is read back when the walk ends.
template <int DIM>
struct GradRecord {
  static constexpr int kStride = 1 + 3 * DIM;
};

struct LaunchParams {
  uint64_t seed;
  uint64_t walk_offset_add;  // added to every item's walk_offset (plan relaunches)
};

}  // namespace wos
