/* wos.h -- C ABI of the MI355X (gfx950) delta-tracking walk-on-spheres library.
 *
 * Solves the Dirichlet problem of Sawhney, Seyb, Jarosz, Crane, "Grid-Free Monte Carlo
 * for PDEs with Spatially Varying Coefficients" (SIGGRAPH 2022), Sec. 1, eq. 1:
 *
 *     div(alpha grad u) + omega . grad u - sigma u = -f   in Omega,   u = g on dOmega,
 *
 * with alpha > 0 and sigma >= 0 (Sec. 2.2), by the delta-tracking walk on spheres of
 * Sec. 5.1 (eq. 28; supplemental Alg. 1) applied after the change of variables of
 * Sec. 4.1 (eqs. 20-23) and App. A. The drift must be a gradient field (App. A); it is
 * given through a potential psi with omega = alpha grad(psi).
 *
 * Conventions for every entry point:
 *  - Every call returns a wos_status; WOS_OK is 0. On failure wos_last_error() returns a
 *    thread-local message. No C++ exception crosses this interface.
 *  - "host" pointers are read during the call and may be freed afterwards; the library
 *    copies what it keeps. "device" pointers are caller-owned device memory of the
 *    device the problem was created on; the library never frees or reallocates them.
 *  - Calls that take a stream are asynchronous on that hipStream_t (NULL = default
 *    stream); results are valid after the caller synchronises the stream. Argument
 *    errors are detected before any work is queued and leave outputs untouched.
 *  - A handle must not be used concurrently from two host threads.
 */
#ifndef WOS_H_
#define WOS_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WOS_OK = 0,
  WOS_ERR_INVALID_ARG = 1,
  WOS_ERR_GEOMETRY = 2,
  WOS_ERR_COEFFICIENT = 3,
  WOS_ERR_UNSUPPORTED = 4,
  WOS_ERR_DEVICE = 5,
  WOS_ERR_OUT_OF_MEMORY = 6,
  WOS_ERR_INTERNAL = 7
} wos_status;

/* Message describing the last non-OK status returned on this host thread. */
const char* wos_last_error(void);

/* Library version as an integer (major * 10000 + minor * 100 + patch). */
int wos_version(void);

/* ---------------------------------------------------------------- problem description */

/* Domain geometry (Sec. 7.1: any boundary representation with a closest-point query).
 *  BALL:    center[dim], radius.                       (disk in 2D, ball in 3D)
 *  BOX:     lo[dim], hi[dim].
 *  POLYGON: dim = 2; vertices: host double [n_vertices][2], one closed counter-clockwise
 *           loop; segment j joins vertex j and j+1 (mod n).
 *  TRIMESH: dim = 3; vertices: host double [n_vertices][3]; triangles: host int32
 *           [n_triangles][3], a closed surface.
 *  SDF:     a list of constructive-solid-geometry operations on signed distance fields
 *           (Sec. 7.2). vertices: host double [n_vertices][8], one operation per row:
 *           (op, shape, c0, c1, c2, p0, p1, p2); n_vertices in 1..WOS_SDF_MAX_OPS.
 *           shape 0 ball      |x - c| - p0                 (p0 > 0)
 *           shape 1 box       exact distance to the box c +- (p0, p1, p2) (> 0 each)
 *           shape 2 halfspace (x.c - p0) / |c|             (c != 0; inside: x.c < p0)
 *           Starting from the empty set (f = +inf), row k combines its field f_k into f:
 *           op 0 union min(f, f_k), op 1 intersection max(f, f_k), op 2 subtraction
 *           max(f, -f_k); row 0 must be a union. The domain is {f < 0}; -f is the
 *           distance used for the ball radius (a lower bound of the true distance, so
 *           every ball stays inside), and the epsilon-shell exit point is
 *           x - f(x) grad f(x) with the gradient of the row that decides f. Components
 *           beyond dim are ignored. lo[dim], hi[dim]: a box that holds the (bounded)
 *           domain, used to sample sigma'.
 * Polygons and meshes get an axis-aligned BVH (Sec. 7.1) and a candidate grid in front
 * of it, built on the host (for meshes with up to 16 threads). Where a grid cell's
 * truncated list cannot decide the nearest primitive (mostly deep inside a mesh or a
 * large polygon), the walk's ball radius may be a certified lower bound of the distance,
 * at least 2 epsilon and a quarter of the cell size: every ball stays inside the
 * domain, as the walk needs (Sec. 3), and no walk ends on such a value. Distance
 * queries are exact. */
typedef enum {
  WOS_GEOM_BALL = 0,
  WOS_GEOM_BOX = 1,
  WOS_GEOM_POLYGON = 2,
  WOS_GEOM_TRIMESH = 3,
  WOS_GEOM_SDF = 4
} wos_geom_kind;
#define WOS_SDF_MAX_OPS 256

typedef struct {
  int32_t kind;               /* wos_geom_kind */
  int32_t pad;
  const double* vertices;     /* host */
  int64_t n_vertices;
  const int32_t* triangles;   /* host, TRIMESH only */
  int64_t n_triangles;
  double center[3];
  double radius;
  double lo[3];
  double hi[3];
} wos_geometry_desc;

/* A scalar field F(x) = c0 + c1 B(x)  (AFFINE)  or  exp(c0 + c1 B(x))  (EXP), with base B:
 *  NONE:         B = 0 (constant field c0, or exp(c0)).
 *  FOURIER:      B = sum_j a_j cos(2 pi k_j . x + phi_j); terms: host double
 *                [n_terms][dim + 2] = (k_j[dim], a_j, phi_j).
 *  BUMPS:        B = sum_j amp_j exp(-|x - c_j|^2 / (2 w_j^2)); terms: host double
 *                [n_terms][dim + 2] = (c_j[dim], w_j, amp_j).
 *  TANH:         B = (1 + tanh((x[axis] - x0)/width))/2; params = (axis, x0, width).
 *  TANH_DRIFT:   drift potential psi with alpha psi' = omega along `axis` for
 *                alpha = low + (high - low)(1 + tanh((x[axis] - x0)/width))/2, psi(x0) = 0;
 *                params = (axis, x0, width, low, high, omega). Affine c0 = 0, c1 = 1 only.
 *  MANUFACTURED: source or boundary field of the manufactured solution `solution_id`
 *                (1: u = exp(x0) cos(x1); 2: u = 1 + x0^2 + x0 x1 / 2): the boundary
 *                field is u, the source is f = -div(alpha grad u) - omega.grad u + sigma u
 *                evaluated with the problem's own alpha, psi and sigma.
 * alpha and psi need first and second derivatives (Sec. 7.1); they are analytic here. */
typedef enum {
  WOS_FIELD_NONE = 0, WOS_FIELD_FOURIER = 1, WOS_FIELD_BUMPS = 2, WOS_FIELD_TANH = 3,
  WOS_FIELD_TANH_DRIFT = 4, WOS_FIELD_MANUFACTURED = 5
} wos_field_base;
typedef enum { WOS_TRANSFORM_AFFINE = 0, WOS_TRANSFORM_EXP = 1 } wos_field_transform;

typedef struct {
  int32_t base;               /* wos_field_base */
  int32_t transform;          /* wos_field_transform */
  double c0, c1;
  int32_t n_terms;
  int32_t solution_id;
  const double* terms;        /* host */
  double params[8];
} wos_field_desc;

/* The PDE of eq. 1 on one domain.
 *  epsilon:   width of the epsilon shell that ends a walk (Sec. 3.2; Alg. 1), > 0.
 *  sigma_bar: the constant majorant of the delta-tracking shift (eq. 23). A value < 0
 *             selects the default max(sigma'_max, 0) - min(sigma'_min, 0) over the
 *             domain, which is the paper's max - min (Sec. 5.1, Sec. 7.1) whenever
 *             sigma' changes sign; sigma' is sampled in FP64 on a grid of
 *             `sigma_bar_grid` points per axis over the bounding box (0: 1024 in 2D,
 *             64 in 3D), keeping interior points only. 0 is allowed only when
 *             sigma' = 0 everywhere (classic walk on spheres).
 *  allow_negative_sigma: 0 rejects sigma < 0 found while sampling (Sec. 2.2). */
typedef struct {
  int32_t dim;                /* 2 or 3 */
  int32_t allow_negative_sigma;
  wos_geometry_desc geometry;
  wos_field_desc alpha;       /* diffusion, > 0 */
  wos_field_desc psi;         /* drift potential: omega = alpha grad(psi) */
  wos_field_desc sigma;       /* absorption, >= 0 */
  wos_field_desc source;      /* f */
  wos_field_desc boundary;    /* g */
  double epsilon;
  double sigma_bar;
  int32_t sigma_bar_grid;
  int32_t pad;
} wos_problem_desc;

typedef struct wos_problem wos_problem;

/* Validates the description, builds the BVH and candidate grid, copies fields and
 * geometry to `device` in FP32 and FP64, and fixes sigma_bar. Synchronous. Errors: WOS_ERR_INVALID_ARG (bad
 * enums, dim, epsilon <= 0, empty terms), WOS_ERR_GEOMETRY (too few vertices, bad
 * indices, degenerate bounds), WOS_ERR_COEFFICIENT (alpha <= 0, sigma < 0 or
 * non-finite sigma' among the samples, or sigma_bar = 0 with sigma' != 0),
 * WOS_ERR_DEVICE / WOS_ERR_OUT_OF_MEMORY. */
wos_status wos_problem_create(const wos_problem_desc* desc, int device, wos_problem** out);

/* sigma' range seen while sampling the grid and the sigma_bar in use. */
wos_status wos_problem_info(const wos_problem* p, double* sigma_prime_min, double* sigma_prime_max,
                            double* sigma_bar);

/* Set-up time of wos_problem_create in milliseconds of host wall clock (any output may be
 * null): geometry_ms building the BVH and the candidate grid (Sec. 7.1), sigma_bar_ms
 * sampling sigma' and fixing sigma_bar (Sec. 5.1), upload_ms laying out and copying the
 * problem tables to the device. */
wos_status wos_problem_setup_times(const wos_problem* p, double* geometry_ms, double* sigma_bar_ms, double* upload_ms);

/* BVH statistics: nodes, depth, primitives (0 for analytic shapes). */
wos_status wos_problem_bvh_info(const wos_problem* p, int64_t* n_nodes, int32_t* depth, int64_t* n_prims);

/* Candidate grid of a polygon or a triangle mesh (all zero for analytic and SDF
 * domains): a uniform grid (nx x ny cells in 2D, nz = 1; nx x ny x nz in 3D) whose cells
 * list every segment or triangle that can be nearest to a point of the cell; closest-point
 * queries then scan one short list instead of traversing the BVH (Sec. 7.1 answers them
 * with a BVH). A polygon cell with more than 32 candidates keeps the 16 nearest to its
 * centre, a mesh cell at most the 6 nearest.
 * n_candidates: total list length. Any output pointer may be null. */
wos_status wos_problem_grid_info(const wos_problem* p, int32_t* nx, int32_t* ny, int32_t* nz,
                                 int64_t* n_candidates);

wos_status wos_problem_destroy(wos_problem* p);

/* ---------------------------------------------------------------- solving */

/* Arithmetic of the walk:
 *  FP32:             geometry, sampling, coefficients and the per-walk sum in FP32;
 *                    exact per-point sums, rounded once to FP64.
 *  FP32_COMPENSATED: as FP32 with a compensated (two-sum) per-walk sum.
 *  FP64:             everything in FP64 (the plain FP64 walker).
 *  FP64_FP32_DRAWS:  the FP64 walker drawing exactly the FP32 walker's uniforms (21-bit
 *                    fields of the Philox blocks, the FP32 layout), so that FP32 and FP64
 *                    walks of one seed follow the same path up to rounding (common random
 *                    numbers: for measuring the error of the FP32 walker, Sec. 3.1).
 *                    Delta tracking only (variant 0 or 1). */
typedef enum { WOS_FP32 = 0, WOS_FP32_COMPENSATED = 1, WOS_FP64 = 2, WOS_FP64_FP32_DRAWS = 3 } wos_precision;

typedef struct {
  int32_t precision;          /* wos_precision */
  int32_t variant;            /* 0: Alg. 1 (source estimated at every ball);
                                 1: eq. 28 (source only on volume events, weight 1/sigma_bar);
                                 2: next flight (Sec. 5.2, supplemental Alg. 2): every ball
                                    exits on its sphere, the recursion inside the ball is
                                    unrolled over uniform inner points with roulette on the
                                    throughput, using the closed-form off-centred kernels of
                                    supplemental Sec. 1.2 (biased off the centre, as the
                                    supplement states). russian_roulette must be 0. */
  uint64_t seed;              /* Philox4x32-10 key */
  uint64_t walks_per_point;   /* > 0 */
  uint64_t walk_offset;       /* global index of the first walk: running N walks and then
                                 M more with walk_offset = N equals one run of N + M walks */
  int32_t russian_roulette;   /* low side of the static weight window (Sec. 6) */
  int32_t pad;
  double ww_lo;               /* w-, default 0.5 (Sec. 6) */
  double ww_hi;               /* w+ > 0: expected-value splitting of walks whose weight
                                 exceeds it (Sec. 6): N branches of weight W/m, m = |W|/w+,
                                 E[N] = m; 0: no splitting. Delta tracking only; needs
                                 problem_index < 2^16 (branch streams use the top half
                                 of that counter word) and ww_hi > ww_lo with roulette. */
  uint64_t max_steps;         /* distance queries per walk before it is cut (0: 10^6) */
  int32_t block_size;         /* 0: autotuned/default; else 64..1024, multiple of 64 */
  int32_t tile_walks;         /* 0: default; walks of one point per work tile taken by a
                                 wavefront (a tile holds whole points when a point has
                                 fewer walks), at most 65536 */
  uint64_t workspace_bytes;   /* 0: default cap (4 GiB) on the accumulation slots of one
                                 launch (128 bytes per tile and point, 384 or 512 with
                                 gradients); a job whose slots exceed it runs its walks per
                                 point in several launches */
} wos_options;

/* One batch of query points of one problem.
 *  points:   device double [n_points][dim] (caller-owned).
 *  sum, sum_sq, n_walks, n_steps: device [n_points] accumulators; every call ADDS the new
 *            walks' sum of estimates, sum of squares, walk count and distance-query count.
 *  counters: device uint64 [4] or NULL, also accumulated: [0] query points outside the
 *            domain or non-finite (their sum becomes NaN), [1] walks cut at max_steps,
 *            [2] walks ended by Russian roulette, [3] radius proposals drawn by the
 *            Green's-function sampler (next flight: points sampled inside balls).
 *  problem_index: fourth word of the Philox counter (distinguishes problems of a batch). */
typedef struct {
  const wos_problem* problem;
  const double* points;
  int64_t n_points;
  uint32_t problem_index;
  uint32_t pad;
  double* sum;
  double* sum_sq;
  uint64_t* n_walks;
  uint64_t* n_steps;
  uint64_t* counters;
  double* grad_sum;       /* device [n_points][dim] or NULL: sums of the per-walk estimates of
                             grad u (supplemental Sec. 2), accumulated like sum; delta
                             tracking only (variant 0 or 1). Points within epsilon of the
                             boundary get no gradient term from their (empty) first ball. */
  double* grad_sum_sq;    /* device [n_points][dim]: sums of their squares (NULL iff grad_sum is) */
} wos_batch_item;

/* Runs walks_per_point walks from every query point of every item (Sec. 3.1: the estimate
 * of u(x) is the mean of independent single-walk estimates) in one persistent kernel
 * launch (several only when workspace_bytes is too small for the job's accumulation
 * slots). All items must share dim, geometry kind and device. Walk j of point i of item k
 * uses the Philox stream key = seed, counter = (draw, walk_offset + j, i, problem_index),
 * so the walks do not depend on scheduling; their estimates are summed exactly (as
 * fixed-point integers, then rounded once to double per point and launch), so results
 * are bit-reproducible whatever the launch shape. A walk estimate must stay below 2^47 in
 * magnitude: a larger or non-finite one makes its point's sum and sum_sq NaN. Scratch
 * memory is allocated and freed in stream order. */
wos_status wos_solve(const wos_batch_item* items, int32_t n_items, const wos_options* opt, void* stream);

/* wos_solve for callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid it): the same walks,
 * outputs and accumulation as wos_solve, with every scratch buffer (point classification,
 * gamma at the query points, item tables, tile counter, accumulation slots, gradient
 * records) in a static array of 128 MiB that the library holds on each GPU it runs on
 * until the process ends. No hipMalloc, hipFree or other allocating routine is called.
 * The caller still passes the inputs and outputs. Limit: the per-point tables and one
 * 128-byte slot per query point (384-512 with gradients) must fit in the array (about
 * 480,000 FP64 points without gradients); larger jobs fail with WOS_ERR_INVALID_ARG before
 * any work is queued. Walks per point that do not fit at once run in several launches.
 * Calls on one GPU share its array: two calls that overlap on one GPU (other streams or
 * host threads) race and corrupt each other's results; calls in one stream are safe.
 * Synchronous like wos_solve up to the item-table upload; then asynchronous on stream. */
wos_status wos_solve_static(const wos_batch_item* items, int32_t n_items, const wos_options* opt, void* stream);

/* Runs the same walks as wos_solve (same outputs, accumulated the same way) with the
 * event-counting build of the walker, and adds per-launch totals into `events` (device
 * uint64 [16]): [0] distance queries, [1] BVH inner nodes visited, [2] primitives whose
 * distance was computed, [3] radius proposals, [4] of which from the free-space law,
 * [5] volume (null-collision) events, [6] exit events, [7] epsilon-shell terminations,
 * [8] gamma-only evaluations, [9] walks started, [10] Russian-roulette draws,
 * [11] balls with large s (2D s >= 2, 3D s >= 1), [12] candidate-grid lookups, and the
 * walker's lane occupancy: [13] lane iterations (64 per wavefront iteration), [14] those
 * of lanes holding a walk, [15] those that evaluated the coefficients. For measuring
 * the algorithmic work of a workload; slower than wos_solve. events: device uint64 [16]. */
wos_status wos_count_events(const wos_batch_item* items, int32_t n_items, const wos_options* opt, uint64_t* events,
                            void* stream);

/* mean = sum / n, std_err = sqrt((sum_sq/n - mean^2) / (n - 1)) per point (eqs. 17-18);
 * all device arrays of length n. std_err is NaN where fewer than two walks were added. */
wos_status wos_finalize(const double* sum, const double* sum_sq, const uint64_t* n_walks, int64_t n,
                        double* mean, double* std_err, void* stream);

/* The same for gradient sums (supplemental Sec. 2): grad_sum, grad_sum_sq, mean, std_err are
 * device double [n][dim] (row-major), n_walks device uint64 [n]. */
wos_status wos_finalize_grad(const double* grad_sum, const double* grad_sum_sq, const uint64_t* n_walks, int64_t n,
                             int32_t dim, double* mean, double* std_err, void* stream);

/* A plan fixes items and options once: it copies the item and tile tables to the device,
 * allocates the scratch memory, classifies the points, picks the launch shape and captures
 * the launches in a hipGraph. wos_plan_launch replays it with a new seed and an extra walk
 * offset (added to opt->walk_offset), accumulating into the same outputs.
 *
 * Launch shape (the batched schedule is the method's embarrassingly parallel structure,
 * Sec. 3.1): with opt->block_size and opt->tile_walks both 0, the first plan of a walker
 * variant (device, precision, dimension, geometry kind) in the process times every block
 * size in {64, 128, 256} with every tile length in {64, ..., 1024} on a prefix of its own
 * walks (eight per resident lane; the per-walk buffers of the plan's workspace only, the
 * caller's outputs are not touched), keeps the fastest for that variant, and builds with
 * it. Later plans and wos_solve of the same variant reuse it. Jobs with fewer walks than
 * the prefix keep 256 / 256. Explicit values are used as given. Synchronous; the caller's
 * stream is used for the timing runs. */
typedef struct wos_plan wos_plan;
wos_status wos_plan_create(const wos_batch_item* items, int32_t n_items, const wos_options* opt,
                           void* stream, wos_plan** out);
wos_status wos_plan_launch(wos_plan* plan, uint64_t seed, uint64_t walk_offset_add, void* stream);
/* The same work as wos_plan_launch (same kernels, tables and outputs, accumulated the
 * same way) issued as separate launches on `stream` with HIP events around each walker
 * launch; waits for it. walker_ms: the walker's time summed over the plan's launches;
 * total_ms (may be null): the whole job. For measurement: the graph replay of
 * wos_plan_launch is the production path. */
wos_status wos_plan_time(wos_plan* plan, uint64_t seed, uint64_t walk_offset_add, void* stream,
                         double* walker_ms, double* total_ms);
/* Launch shape chosen by the plan. */
wos_status wos_plan_info(const wos_plan* plan, int32_t* block_size, int32_t* tile_walks,
                         int32_t* grid_size, int32_t* n_launches);
/* Set-up time of wos_plan_create in milliseconds of host wall clock: build_ms for the
 * tables, scratch, classification, gamma(x0) and graph capture of the final plan, tune_ms
 * for the autotuning runs (0 when the shape was given, already tuned, or the job has too
 * few walks to time); tuned_here = 1 when this plan ran the autotuner. Any output may be
 * null. */
wos_status wos_plan_setup_times(const wos_plan* plan, double* build_ms, double* tune_ms, int32_t* tuned_here);
wos_status wos_plan_destroy(wos_plan* plan);

/* Persistence of the autotuner's choices (the launch shapes of the batched schedule).
 * wos_tune_cache_save writes every shape tuned in this process to the text file `path`,
 * one line per walker variant: device architecture and compute-unit count, precision,
 * dimension, geometry kind, walker mode, batch flag, block size and tile length.
 * wos_tune_cache_load reads such a file and makes its shapes the tuned shapes of every
 * device of this process with the same architecture and compute-unit count (replacing
 * shapes tuned before), so that later plans of those variants skip the autotuning runs.
 * Errors: WOS_ERR_INVALID_ARG for a null path, a file that cannot be opened or written,
 * or a malformed line (nothing is loaded then). n_saved / n_loaded (may be null): lines
 * written, shapes set. */
wos_status wos_tune_cache_save(const char* path, int32_t* n_saved);
wos_status wos_tune_cache_load(const char* path, int32_t* n_loaded);

/* ---------------------------------------------------------------- diagnostics
 * These run the walker's own device functions on explicit inputs so each step of the
 * walk can be checked on its own. precision: WOS_FP32 or WOS_FP64. */

/* Per point [alpha, gamma, sigma', f, f', g] with gamma = (ln alpha + psi)/2,
 * sigma' = sigma/alpha + Lap(gamma) + |grad gamma|^2, f' = e^gamma f / alpha (Sec. 4.1,
 * eq. 21; App. A) and g the boundary field at the point. out: device double [n][6]. */
wos_status wos_eval_coefficients(const wos_problem* p, const double* points, int64_t n, int32_t precision,
                                 double* out, void* stream);

/* Exact distance to the boundary and closest point (Alg. 1, first step). d: device
 * double [n]; closest: device double [n][dim]. */
wos_status wos_eval_distance(const wos_problem* p, const double* points, int64_t n, int32_t precision,
                             double* d, double* closest, void* stream);

/* For each s_i = R sqrt(sigma_bar): [P_B = sigma_bar |G|, |G|/R^2] of the centred ball
 * (supp. Sec. 1.1). s: device double [n]; out: device double [n][2]. */
wos_status wos_eval_ball(int32_t dim, int32_t precision, const double* s, int64_t n, double* out, void* stream);

/* n radius fractions t = |y - x|/R of y ~ G(x,.)/|G| for the given s (supp. Sec. 1.4),
 * sample i drawn from the Philox stream (seed, counter (draw, i, 0, 0)); s = 0 samples
 * the harmonic law. t: device double [n]; trials (optional): device uint64 [1], added. */
wos_status wos_sample_radius(int32_t dim, int32_t precision, double s, int64_t n, uint64_t seed,
                             double* t, uint64_t* trials, void* stream);

/* Philox4x32-10 blocks: out[i] = philox(ctr[i], key). ctr, out: device uint32 [n][4]. */
wos_status wos_philox(const uint32_t* ctr, uint64_t key, int64_t n, uint32_t* out, void* stream);

/* Exponentially scaled modified Bessel functions used by the ball kernels (supplemental
 * Sec. 1.1-1.2): which = 0: e^-x I0(x), 1: e^x K0(x), 2: e^-x I1(x), 3: e^x K1(x), at
 * x[i] > 0. device double [n]. */
wos_status wos_eval_bessel(int32_t which, int32_t precision, const double* x, int64_t n, double* out,
                           void* stream);

/* Off-centred kernels of the next-flight walk on the ball B(c, R) for Laplace - sigma_bar,
 * in the closed-form approximations of supplemental Sec. 1.2 (exact at the centre):
 * which = 0: G(x, y) |B| with u = x - c, v = y - c; which = 1: P(x, z) |dB| with u = x - c,
 * v = z - c on the sphere. u, v: device double [n][dim]; out: device double [n].
 * sigma_bar = 0 takes the harmonic kernels. */
wos_status wos_eval_offcentred(int32_t which, int32_t dim, int32_t precision, double R, double sigma_bar,
                               const double* u, const double* v, int64_t n, double* out, void* stream);

/* 1 if points[i] lies strictly inside the domain, else 0 (harness helper; not on the
 * walk's path). inside: device int8 [n]. */
wos_status wos_classify(const wos_problem* p, const double* points, int64_t n, int8_t* inside, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* WOS_H_ */
