// FP64 CPU oracle for the delta-tracking walk on spheres of
//   Sawhney, Seyb, Jarosz, Crane, "Grid-Free Monte Carlo for PDEs with
//   Spatially Varying Coefficients" (SIGGRAPH 2022).
//
// TEST INFRASTRUCTURE ONLY. This file is a plain, slow, deliberately unoptimised
// restatement of the method used to check the GPU library. Only the test suite,
// the smoke entry point and the benchmark's CPU-baseline leg may load it. It
// shares no code, header, table or constant with the GPU library.
//
// What it computes (each function cites the passage it follows):
//   * the PDE of Sec. 1 (eq. 1): div(alpha grad u) + omega.grad u - sigma u = -f,
//     u = g on the boundary, with omega = alpha grad(psi) (App. A needs the drift
//     to be a gradient field);
//   * the change of variables of Sec. 4.1 (eqs. 20-21) and App. A:
//     U = e^gamma u, gamma = (ln alpha + psi)/2, giving
//     Laplace(U) - sigma' U = -f', sigma' = sigma/alpha + Lap(gamma) + |grad gamma|^2,
//     f' = e^gamma f / alpha;
//   * the delta-tracking shift by a constant sigma_bar (eq. 23) and the
//     delta-tracking walk on spheres (Sec. 5.1, eq. 28, supplemental Alg. 1);
//   * the centred screened-Poisson Green's function of a ball, its integral |G|
//     and its Poisson kernel (supplemental Sec. 1.1), sampled here by numerical
//     inversion of the closed-form radial CDF (no rejection envelope);
//   * the next-flight walk on spheres (Sec. 5.2, supplemental Alg. 2) with the
//     off-centred Green's function and Poisson kernel approximations of supplemental
//     Sec. 1.2 and uniform points inside each ball;
//   * the static weight window of Sec. 6: Russian roulette below w- and expected-value
//     splitting above w+;
//   * the per-point Monte Carlo mean (Sec. 3.1, eqs. 17-18);
//   * domains given as a list of CSG operations on signed distance fields (Sec. 7.2).
//
// Readings of the paper taken here (where it is silent, ambiguous or garbled):
//   R1  the source sign in eq. 21 is taken as -f' (consistent with eq. 23 and App. A);
//   R2  with drift, gamma = (ln alpha + psi)/2 and the weights use e^{gamma(y)-gamma(x)}
//       (reduces to sqrt(alpha(y)/alpha(x)) of Alg. 1 when omega = 0);
//   R3  termination returns g(xbar) as printed in Alg. 1 (no e^gamma ratio);
//   R4  Alg. 1 (source estimated at every step) is the default; eq. 28 (source only on
//       volume events, weight 1/sigma_bar) is available as variant 1;
//   R5  Russian roulette: when |W| < w_lo the walk survives with probability |W|/w_lo
//       and then carries W = sign(W) w_lo; the estimate accumulated so far is kept;
//   R6  for s = R sqrt(sigma_bar) < 1e-4 the harmonic (sigma_bar -> 0) limits are used
//       for P_B = s^2/4 (2D), s^2/6 (3D) and for the radial law (relative error O(s^2));
//   R7  an SDF domain is {f < 0}; -f serves as the distance (a lower bound of the true
//       one for unions, exact for single primitives and intersections) and the walk
//       ends at x - f grad f.
//
// Pins (tests/test_oracle_*.py): every function here is checked against closed forms,
// quadrature, library routines or brute force. Whole-walk estimates on random coefficient
// fields (the star polygons, the perturbed icosphere, the high-contrast square's field
// families) are pinned by running the same fields with the data of a manufactured
// solution (f from eq. 1, g = u) against u itself. Parity unpinned: the next-flight walk
// with the approximate off-centred kernels (walk_next_flight, variant 2) is exact only
// where those kernels are (the centre, the harmonic case, sigma' = sigma_bar), elsewhere
// pinned through the exact-kernel variant 3 and the kernels' own pins.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key = (seed lo,
// seed hi), counter = (block index, walk index, point index, problem index); each
// uniform double takes 53 bits from two consecutive 32-bit words.
//
// Build: g++ -O2 -std=c++17 -fPIC -shared -pthread (oracle.py runs it).

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

const double kPi = 3.14159265358979323846;

// ------------------------------------------------------------------ Philox4x32-10

void philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k[0];
  const uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
    philox_round(c, k);
  }
  for (int i = 0; i < 4; ++i) out[i] = c[i];
}

struct Stream {
  uint32_t key[2];
  uint32_t ctr[4];
  uint32_t buf[4];
  int pos;
};

void stream_init(Stream* st, uint64_t seed, uint32_t walk, uint32_t point, uint32_t problem) {
  st->key[0] = (uint32_t)seed;
  st->key[1] = (uint32_t)(seed >> 32);
  st->ctr[0] = 0;
  st->ctr[1] = walk;
  st->ctr[2] = point;
  st->ctr[3] = problem;
  st->pos = 4;
}

uint32_t next_u32(Stream* st) {
  if (st->pos == 4) {
    philox4x32_10(st->ctr, st->key, st->buf);
    st->ctr[0] += 1;
    st->pos = 0;
  }
  return st->buf[st->pos++];
}

double uniform(Stream* st) {  // [0, 1)
  const uint64_t a = next_u32(st);
  const uint64_t b = next_u32(st);
  const uint64_t x = ((a << 32) | b) >> 11;
  return (double)x * (1.0 / 9007199254740992.0);
}

// ------------------------------------------------------------------ problem description

enum { B_NONE = 0, B_FOURIER = 1, B_BUMPS = 2, B_TANH = 3, B_TANH_DRIFT = 4, B_MANUFACTURED = 5 };
enum { T_AFFINE = 0, T_EXP = 1 };
enum { G_BALL = 0, G_BOX = 1, G_POLYGON = 2, G_TRIMESH = 3, G_SDF = 4 };
enum { U_EXPCOS = 1, U_QUADRATIC = 2 };

}  // namespace

extern "C" {

struct OField {
  int32_t base;
  int32_t transform;
  double c0, c1;
  int32_t n;       // number of terms (fourier modes / bumps)
  int32_t u_id;    // manufactured solution id
  const double* p; // fourier: per term k[dim], a, phi;  bumps: per term c[dim], w, amp
  double q[8];     // tanh: axis, x0, width;  tanh_drift: axis, x0, width, low, high, omega
};

struct OGeom {
  int32_t kind;
  int32_t pad;
  int64_t n_vertices;
  int64_t n_prims;
  const double* vertices;  // [n_vertices][dim]
  const int32_t* prims;    // trimesh: [n_prims][3]; polygon: unused (closed loop)
  double center[3];
  double radius;
  double lo[3];
  double hi[3];
};

struct OProblem {
  int32_t dim;
  int32_t pad;
  OGeom geom;
  OField alpha, psi, sigma, source, boundary;
  double epsilon;
  const void* accel;      // null: brute-force closest points; else the OBvh of the boundary
};

struct OOptions {
  double sigma_bar;       // > 0, or 0 only for sigma' == 0 problems
  uint64_t seed;
  uint64_t walk_offset;
  uint64_t n_walks;
  uint32_t problem_index;
  int32_t variant;        // 0: Alg. 1 (source every step), 1: eq. 28 (source on volume events),
                          // 2: next flight (Sec. 5.2, supplemental Alg. 2) with the closed-form
                          // off-centred kernels, 3: next flight with the exact series kernels
  int32_t russian_roulette;
  double ww_lo;
  double ww_hi;           // > 0: split walks whose |weight| exceeds it (Sec. 6); 0: no splitting
  uint64_t max_steps;
  int32_t threads;
  int32_t accel;          // 0: brute-force closest points (correctness mode); 1: the oracle's own
                          // axis-aligned BVH over segments or triangles (timing mode, Sec. 7.1)
};

}  // extern "C"

namespace {

// A scalar field with its gradient and Laplacian.
struct FVal {
  double v;
  double g[3];
  double lap;
};

double dot(const double* a, const double* b, int dim) {
  double s = 0;
  for (int i = 0; i < dim; ++i) s += a[i] * b[i];
  return s;
}

// Base B(x), grad B, Laplace B of the field families of the synthetic workloads.
FVal eval_base(const OField& f, const double* x, int dim) {
  FVal r = {0, {0, 0, 0}, 0};
  if (f.base == B_FOURIER) {
    // B = sum a cos(2 pi k.x + phi)
    const int stride = dim + 2;
    for (int j = 0; j < f.n; ++j) {
      const double* k = f.p + j * stride;
      const double a = f.p[j * stride + dim];
      const double phi = f.p[j * stride + dim + 1];
      const double arg = 2 * kPi * dot(k, x, dim) + phi;
      const double c = std::cos(arg), s = std::sin(arg);
      r.v += a * c;
      for (int i = 0; i < dim; ++i) r.g[i] += -a * s * 2 * kPi * k[i];
      r.lap += -a * c * 4 * kPi * kPi * dot(k, k, dim);
    }
  } else if (f.base == B_BUMPS) {
    // B = sum amp exp(-|x-c|^2 / (2 w^2))
    const int stride = dim + 2;
    for (int j = 0; j < f.n; ++j) {
      const double* c = f.p + j * stride;
      const double w = f.p[j * stride + dim];
      const double amp = f.p[j * stride + dim + 1];
      double d[3], r2 = 0;
      for (int i = 0; i < dim; ++i) {
        d[i] = x[i] - c[i];
        r2 += d[i] * d[i];
      }
      const double e = amp * std::exp(-r2 / (2 * w * w));
      r.v += e;
      for (int i = 0; i < dim; ++i) r.g[i] += -e * d[i] / (w * w);
      r.lap += e * (r2 / (w * w * w * w) - dim / (w * w));
    }
  } else if (f.base == B_TANH) {
    // B = (1 + tanh z)/2, z = (x_axis - x0)/width
    const int ax = (int)f.q[0];
    const double w = f.q[2];
    const double th = std::tanh((x[ax] - f.q[1]) / w);
    r.v = 0.5 * (1 + th);
    r.g[ax] = 0.5 * (1 - th * th) / w;
    r.lap = -th * (1 - th * th) / (w * w);
  } else if (f.base == B_TANH_DRIFT) {
    // psi with alpha psi' = omega, alpha = A + Bc tanh z, A = (lo+hi)/2, Bc = (hi-lo)/2,
    // psi = omega w [A z - Bc ln(A cosh z + Bc sinh z) + Bc ln A] / (A^2 - Bc^2)
    const int ax = (int)f.q[0];
    const double x0 = f.q[1], w = f.q[2], lo = f.q[3], hi = f.q[4], om = f.q[5];
    const double A = 0.5 * (lo + hi), Bc = 0.5 * (hi - lo);
    const double z = (x[ax] - x0) / w;
    const double az = std::fabs(z);
    const double sg = z >= 0 ? 1.0 : -1.0;
    const double lnmix = az + std::log(0.5 * (A + sg * Bc) + 0.5 * (A - sg * Bc) * std::exp(-2 * az));
    r.v = om * w * (A * z - Bc * lnmix + Bc * std::log(A)) / (A * A - Bc * Bc);
    const double th = std::tanh(z);
    const double al = A + Bc * th;
    const double dal = Bc * (1 - th * th) / w;
    r.g[ax] = om / al;
    r.lap = -om * dal / (al * al);
  }
  return r;
}

// Field value after its transform: affine c0 + c1 B, or exp(c0 + c1 B).
FVal eval_field(const OField& f, const double* x, int dim) {
  const FVal b = eval_base(f, x, dim);
  FVal r;
  if (f.transform == T_EXP) {
    r.v = std::exp(f.c0 + f.c1 * b.v);
    double gb2 = 0;
    for (int i = 0; i < 3; ++i) {
      r.g[i] = r.v * f.c1 * b.g[i];
      gb2 += b.g[i] * b.g[i];
    }
    r.lap = r.v * (f.c1 * b.lap + f.c1 * f.c1 * gb2);
  } else {
    r.v = f.c0 + f.c1 * b.v;
    for (int i = 0; i < 3; ++i) r.g[i] = f.c1 * b.g[i];
    r.lap = f.c1 * b.lap;
  }
  return r;
}

// Manufactured solutions u with grad u and Laplace u.
FVal eval_u(int id, const double* x) {
  FVal r = {0, {0, 0, 0}, 0};
  if (id == U_EXPCOS) {
    const double e = std::exp(x[0]);
    r.v = e * std::cos(x[1]);
    r.g[0] = e * std::cos(x[1]);
    r.g[1] = -e * std::sin(x[1]);
    r.lap = 0;
  } else if (id == U_QUADRATIC) {
    r.v = 1 + x[0] * x[0] + 0.5 * x[0] * x[1];
    r.g[0] = 2 * x[0] + 0.5 * x[1];
    r.g[1] = 0.5 * x[0];
    r.lap = 2;
  }
  return r;
}

// Everything the walk needs at a point (Sec. 4.1 eqs. 20-21 and App. A).
struct Coef {
  double alpha;
  double gamma;        // (ln alpha + psi) / 2
  double sigma_prime;  // sigma/alpha + Lap gamma + |grad gamma|^2
  double f;            // source of eq. 1
  double f_prime;      // e^gamma f / alpha
  double grad_gamma[3];
};

double source_value(const OProblem& P, const double* x, const FVal& al, const FVal& ps, double sg) {
  const OField& f = P.source;
  if (f.base == B_MANUFACTURED) {
    // f = -div(alpha grad u) - omega.grad u + sigma u, omega = alpha grad psi (eq. 1)
    const FVal u = eval_u(f.u_id, x);
    double ga_gu = 0, gp_gu = 0;
    for (int i = 0; i < P.dim; ++i) {
      ga_gu += al.g[i] * u.g[i];
      gp_gu += ps.g[i] * u.g[i];
    }
    return -(al.v * u.lap + ga_gu) - al.v * gp_gu + sg * u.v;
  }
  return eval_field(f, x, P.dim).v;
}

double boundary_value(const OProblem& P, const double* x) {
  const OField& g = P.boundary;
  if (g.base == B_MANUFACTURED) return eval_u(g.u_id, x).v;
  return eval_field(g, x, P.dim).v;
}

Coef coefficients(const OProblem& P, const double* x) {
  const int dim = P.dim;
  const FVal al = eval_field(P.alpha, x, dim);
  const FVal ps = eval_field(P.psi, x, dim);
  const double sg = eval_field(P.sigma, x, dim).v;
  // Eq. 20: dividing by alpha leaves Laplace u + b.grad u - (sigma/alpha) u = -f/alpha with
  // first-order coefficient b = grad(alpha)/alpha + omega/alpha = grad(ln alpha + psi).
  // App. A (generator Laplace/2): halve the equation, b/2 = grad(gamma) with
  // gamma = (ln alpha + psi)/2, and the Girsanov/Ito weight yields the zeroth-order
  // coefficient sigma/(2 alpha) + (Lap gamma + |grad gamma|^2)/2 and the source
  // e^gamma f/(2 alpha). Multiplying back by 2 gives the screened Poisson form below.
  double grad_gamma[3], lap_gamma;
  {
    double grad_ln_alpha[3];
    double ga2 = 0;
    for (int i = 0; i < 3; ++i) {
      grad_ln_alpha[i] = al.g[i] / al.v;
      ga2 += al.g[i] * al.g[i];
    }
    const double lap_ln_alpha = al.lap / al.v - ga2 / (al.v * al.v);
    for (int i = 0; i < 3; ++i) grad_gamma[i] = 0.5 * (grad_ln_alpha[i] + ps.g[i]);
    lap_gamma = 0.5 * (lap_ln_alpha + ps.lap);
  }
  Coef c;
  c.alpha = al.v;
  c.gamma = 0.5 * (std::log(al.v) + ps.v);
  c.sigma_prime = sg / al.v + lap_gamma + dot(grad_gamma, grad_gamma, 3);
  c.f = source_value(P, x, al, ps, sg);
  c.f_prime = std::exp(c.gamma) * c.f / al.v;
  for (int i = 0; i < 3; ++i) c.grad_gamma[i] = grad_gamma[i];
  return c;
}

// ------------------------------------------------------------------ distance to the boundary

void closest_on_segment(const double* p, const double* a, const double* b, int dim, double* out) {
  double ab[3], ap[3];
  for (int i = 0; i < dim; ++i) {
    ab[i] = b[i] - a[i];
    ap[i] = p[i] - a[i];
  }
  const double l2 = dot(ab, ab, dim);
  double t = l2 > 0 ? dot(ap, ab, dim) / l2 : 0.0;
  if (t < 0) t = 0;
  if (t > 1) t = 1;
  for (int i = 0; i < dim; ++i) out[i] = a[i] + t * ab[i];
}

double dist2(const double* a, const double* b, int dim) {
  double s = 0;
  for (int i = 0; i < dim; ++i) s += (a[i] - b[i]) * (a[i] - b[i]);
  return s;
}

// Closest point of a triangle: the projection onto its plane if that lies inside the
// triangle, otherwise the closest of the three edge points.
void closest_on_triangle(const double* p, const double* a, const double* b, const double* c, double* out) {
  double e0[3], e1[3], n[3], ap[3];
  for (int i = 0; i < 3; ++i) {
    e0[i] = b[i] - a[i];
    e1[i] = c[i] - a[i];
    ap[i] = p[i] - a[i];
  }
  n[0] = e0[1] * e1[2] - e0[2] * e1[1];
  n[1] = e0[2] * e1[0] - e0[0] * e1[2];
  n[2] = e0[0] * e1[1] - e0[1] * e1[0];
  const double nn = dot(n, n, 3);
  if (nn > 0) {
    const double h = dot(ap, n, 3) / nn;
    double q[3];
    for (int i = 0; i < 3; ++i) q[i] = p[i] - h * n[i];
    // barycentric test via signed sub-areas
    auto side = [&](const double* u, const double* v) {
      double uv[3], uq[3], cr[3];
      for (int i = 0; i < 3; ++i) {
        uv[i] = v[i] - u[i];
        uq[i] = q[i] - u[i];
      }
      cr[0] = uv[1] * uq[2] - uv[2] * uq[1];
      cr[1] = uv[2] * uq[0] - uv[0] * uq[2];
      cr[2] = uv[0] * uq[1] - uv[1] * uq[0];
      return dot(cr, n, 3);
    };
    if (side(a, b) >= 0 && side(b, c) >= 0 && side(c, a) >= 0) {
      for (int i = 0; i < 3; ++i) out[i] = q[i];
      return;
    }
  }
  double best = INFINITY, tmp[3];
  const double* V[3] = {a, b, c};
  for (int e = 0; e < 3; ++e) {
    closest_on_segment(p, V[e], V[(e + 1) % 3], 3, tmp);
    const double d2 = dist2(p, tmp, 3);
    if (d2 < best) {
      best = d2;
      for (int i = 0; i < 3; ++i) out[i] = tmp[i];
    }
  }
}

// ------------------------------------------------------------------ CSG signed distance fields
// Sec. 7.2 represents the domain by a list of CSG operations on signed distance fields.
// Reading: rows (op, shape, c[3], p[3]); the field starts as the empty set (+inf) and each
// row takes min (union), max (intersection) or max with the negated field (subtraction);
// the domain is {f < 0}, the ball radius is -f and the exit point is x - f grad f, the
// gradient being that of the row deciding f (the first on ties).

// Signed distance of one primitive and its gradient.
double sdf_primitive(const double* row, const double* x, int dim, double* grad) {
  const int shape = (int)row[1];
  const double* c = row + 2;
  const double* p = row + 5;
  if (shape == 0) {  // ball of radius p0 about c
    double r = std::sqrt(dist2(x, c, dim));
    for (int i = 0; i < dim; ++i) grad[i] = r > 0 ? (x[i] - c[i]) / r : (i == 0 ? 1.0 : 0.0);
    return r - p[0];
  }
  if (shape == 1) {  // box c +- p: distance to the nearest point of the box (outside) or
                     // minus the distance to the nearest face (inside)
    double q[3], out = 0, far = -INFINITY;
    int axis = 0;
    for (int i = 0; i < dim; ++i) {
      q[i] = std::fabs(x[i] - c[i]) - p[i];
      if (q[i] > 0) out += q[i] * q[i];
      if (q[i] > far) {
        far = q[i];
        axis = i;
      }
    }
    const bool outside = out > 0;
    out = std::sqrt(out);
    for (int i = 0; i < dim; ++i) {
      const double sg = x[i] >= c[i] ? 1.0 : -1.0;
      grad[i] = outside ? (q[i] > 0 ? sg * q[i] / out : 0.0) : (i == axis ? sg : 0.0);
    }
    return outside ? out : far;
  }
  // half-space {x . n < p0} with n = c / |c|
  double nn = std::sqrt(dot(c, c, dim));
  for (int i = 0; i < dim; ++i) grad[i] = c[i] / nn;
  return (dot(x, c, dim) - p[0]) / nn;
}

double sdf_field(const OGeom& g, const double* x, int dim, double* grad) {
  double f = INFINITY, gk[3];
  for (int64_t k = 0; k < g.n_vertices; ++k) {
    const double* row = g.vertices + 8 * k;
    const int op = (int)row[0];
    double fk = sdf_primitive(row, x, dim, gk);
    if (op == 2) {
      fk = -fk;
      for (int i = 0; i < dim; ++i) gk[i] = -gk[i];
    }
    const bool take = op == 0 ? fk < f : fk > f;
    if (take) {
      f = fk;
      for (int i = 0; i < dim; ++i) grad[i] = gk[i];
    }
  }
  return f;
}

// Boundary primitives of a polygon (segment j joins vertex j and j + 1 of the closed
// loop) or a triangle mesh.
int64_t n_boundary_prims(const OGeom& g) { return g.kind == G_POLYGON ? g.n_vertices : g.n_prims; }

void closest_on_prim(const OGeom& g, int64_t j, const double* x, double* q) {
  if (g.kind == G_POLYGON) {
    const int64_t n = g.n_vertices;
    closest_on_segment(x, g.vertices + 2 * j, g.vertices + 2 * ((j + 1) % n), 2, q);
  } else {
    const int32_t* t = g.prims + 3 * j;
    closest_on_triangle(x, g.vertices + 3 * t[0], g.vertices + 3 * t[1], g.vertices + 3 * t[2], q);
  }
}

// ------------------------------------------------------------------ BVH (timing mode)
// Sec. 7.1 answers closest-point queries with a basic axis-aligned BVH. This one is kept
// plain: each node covers a range of a permutation of the primitives; a node with more
// than 4 primitives is split at the median of their box centres along the longest axis
// of those centres. The nearest-primitive query visits the nearer child first and skips
// a box whose squared distance exceeds the best squared distance found so far (with a
// relative margin of 1e-9 against rounding in the per-primitive distance), so it returns
// the brute-force minimum: the same closest-point function runs on every primitive that
// could attain it.
struct OBvh {
  int dim = 2;
  std::vector<double> lo, hi;          // [node][dim] bounds
  std::vector<int32_t> left, right;    // children; -1 for a leaf
  std::vector<int64_t> first, count;   // leaf: range of `order`
  std::vector<int64_t> order;          // primitive indices
};

int32_t bvh_build_node(OBvh& b, const std::vector<double>& plo, const std::vector<double>& phi,
                       const std::vector<double>& cen, int64_t first, int64_t count) {
  const int dim = b.dim;
  const int32_t id = (int32_t)b.left.size();
  b.left.push_back(-1);
  b.right.push_back(-1);
  b.first.push_back(first);
  b.count.push_back(count);
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t k = first; k < first + count; ++k) {
    const int64_t j = b.order[k];
    for (int i = 0; i < dim; ++i) {
      lo[i] = std::fmin(lo[i], plo[j * dim + i]);
      hi[i] = std::fmax(hi[i], phi[j * dim + i]);
      clo[i] = std::fmin(clo[i], cen[j * dim + i]);
      chi[i] = std::fmax(chi[i], cen[j * dim + i]);
    }
  }
  for (int i = 0; i < dim; ++i) {
    b.lo.push_back(lo[i]);
    b.hi.push_back(hi[i]);
  }
  if (count <= 4) return id;
  int axis = 0;
  for (int i = 1; i < dim; ++i)
    if (chi[i] - clo[i] > chi[axis] - clo[axis]) axis = i;
  const int64_t half = count / 2;
  std::nth_element(b.order.begin() + first, b.order.begin() + first + half, b.order.begin() + first + count,
                   [&](int64_t u, int64_t v) { return cen[u * dim + axis] < cen[v * dim + axis]; });
  const int32_t l = bvh_build_node(b, plo, phi, cen, first, half);
  const int32_t r = bvh_build_node(b, plo, phi, cen, first + half, count - half);
  b.left[id] = l;
  b.right[id] = r;
  return id;
}

void bvh_build(const OGeom& g, int dim, OBvh& b) {
  const int64_t n = n_boundary_prims(g);
  const int nv = dim;   // vertices per primitive: 2 for segments, 3 for triangles
  std::vector<double> plo(n * dim), phi(n * dim), cen(n * dim);
  for (int64_t j = 0; j < n; ++j) {
    for (int i = 0; i < dim; ++i) {
      plo[j * dim + i] = INFINITY;
      phi[j * dim + i] = -INFINITY;
      cen[j * dim + i] = 0;
    }
    for (int v = 0; v < nv; ++v) {
      const double* p = g.kind == G_POLYGON ? g.vertices + 2 * ((j + v) % g.n_vertices)
                                            : g.vertices + 3 * g.prims[3 * j + v];
      for (int i = 0; i < dim; ++i) {
        plo[j * dim + i] = std::fmin(plo[j * dim + i], p[i]);
        phi[j * dim + i] = std::fmax(phi[j * dim + i], p[i]);
        cen[j * dim + i] += p[i] / nv;
      }
    }
  }
  b.dim = dim;
  b.order.resize(n);
  for (int64_t j = 0; j < n; ++j) b.order[j] = j;
  bvh_build_node(b, plo, phi, cen, 0, n);
}

double box_dist2(const OBvh& b, int32_t node, const double* x) {
  double s = 0;
  for (int i = 0; i < b.dim; ++i) {
    const double lo = b.lo[node * b.dim + i], hi = b.hi[node * b.dim + i];
    const double e = x[i] < lo ? lo - x[i] : (x[i] > hi ? x[i] - hi : 0.0);
    s += e * e;
  }
  return s;
}

double bvh_nearest(const OBvh& b, const OGeom& g, int dim, const double* x, double* xbar) {
  double best = INFINITY, q[3];
  int32_t stack[128];   // median splits: depth <= log2(n) + 1, at most one pending sibling per level
  int top = 0;
  stack[top++] = 0;
  while (top > 0) {
    const int32_t node = stack[--top];
    if (box_dist2(b, node, x) > best * (1.0 + 1e-9)) continue;
    if (b.left[node] < 0) {
      for (int64_t k = b.first[node]; k < b.first[node] + b.count[node]; ++k) {
        closest_on_prim(g, b.order[k], x, q);
        const double d2 = dist2(x, q, dim);
        if (d2 < best) {
          best = d2;
          for (int i = 0; i < dim; ++i) xbar[i] = q[i];
        }
      }
      continue;
    }
    int32_t near = b.left[node], far = b.right[node];
    if (box_dist2(b, far, x) < box_dist2(b, near, x)) std::swap(near, far);
    stack[top++] = far;   // popped after the nearer child
    stack[top++] = near;
  }
  return std::sqrt(best);
}

// Distance d and closest point xbar on the boundary (Alg. 1, first line): by brute force
// over all primitives, or with P.accel through the BVH above (the same minimum);
// unsigned for explicit boundaries, -f for SDF domains.
double distance_to_boundary(const OProblem& P, const double* x, double* xbar) {
  const OGeom& g = P.geom;
  const int dim = P.dim;
  if (g.kind == G_SDF) {
    double grad[3];
    const double f = sdf_field(g, x, dim, grad);
    for (int i = 0; i < dim; ++i) xbar[i] = x[i] - f * grad[i];
    return -f;
  }
  if (g.kind == G_BALL) {
    double v[3], r = 0;
    for (int i = 0; i < dim; ++i) {
      v[i] = x[i] - g.center[i];
      r += v[i] * v[i];
    }
    r = std::sqrt(r);
    for (int i = 0; i < dim; ++i) xbar[i] = r > 0 ? g.center[i] + g.radius * v[i] / r : g.center[i] + (i == 0 ? g.radius : 0);
    return std::fabs(g.radius - r);
  }
  if (g.kind == G_BOX) {
    double best = INFINITY;
    for (int i = 0; i < dim; ++i) {
      for (int side = 0; side < 2; ++side) {
        const double plane = side ? g.hi[i] : g.lo[i];
        double q[3];
        for (int j = 0; j < dim; ++j) q[j] = std::fmin(std::fmax(x[j], g.lo[j]), g.hi[j]);
        q[i] = plane;
        const double d2 = dist2(x, q, dim);
        if (d2 < best) {
          best = d2;
          for (int j = 0; j < dim; ++j) xbar[j] = q[j];
        }
      }
    }
    return std::sqrt(best);
  }
  if (P.accel) return bvh_nearest(*(const OBvh*)P.accel, g, dim, x, xbar);
  // polygon or triangle mesh: every primitive
  double best = INFINITY, q[3];
  for (int64_t j = 0; j < n_boundary_prims(g); ++j) {
    closest_on_prim(g, j, x, q);
    const double d2 = dist2(x, q, dim);
    if (d2 < best) {
      best = d2;
      for (int i = 0; i < dim; ++i) xbar[i] = q[i];
    }
  }
  return std::sqrt(best);
}

// ------------------------------------------------------------------ ball kernels (supp. Sec. 1.1)

double I0(double x) { return std::cyl_bessel_i(0.0, x); }
double I1(double x) { return std::cyl_bessel_i(1.0, x); }
double K0(double x) { return std::cyl_bessel_k(0.0, x); }
double K1(double x) { return std::cyl_bessel_k(1.0, x); }

const double kSmallS = 1e-4;  // reading R6

// P_B = sigma_bar |G| for the ball of radius R centred at x, s = R sqrt(sigma_bar).
double ball_pb(int dim, double s) {
  if (s < kSmallS) return dim == 2 ? s * s / 4 : s * s / 6;
  if (dim == 2) return 1.0 - 1.0 / I0(s);
  return 1.0 - s / std::sinh(s);
}

// |G| = integral of the centred Green's function over the ball.
double ball_gnorm(int dim, double R, double sigma_bar) {
  const double s = R * std::sqrt(sigma_bar);
  if (sigma_bar <= 0 || s < kSmallS) return dim == 2 ? R * R / 4 : R * R / 6;
  return ball_pb(dim, s) / sigma_bar;
}

// Radial CDF of y ~ G(x,.)/|G| in t = |y-x|/R, from integrating 2 pi r G (2D) or
// 4 pi r^2 G (3D) of supp. Sec. 1.1 in closed form.
//   2D: C(t) = [1 - ts K1(ts) - s (K0(s)/I0(s)) t I1(ts)] / (1 - 1/I0(s))
//   3D: C(t) = [1 - sinh(s(1-t))/sinh s - ts cosh(s(1-t))/sinh s] / (1 - s/sinh s)
// and their harmonic limits t^2 (1 - 2 ln t), 3t^2 - 2t^3.
double radial_cdf(int dim, double s, double t) {
  if (t <= 0) return 0.0;
  if (t >= 1) return 1.0;
  if (s < kSmallS) return dim == 2 ? t * t * (1 - 2 * std::log(t)) : t * t * (3 - 2 * t);
  if (dim == 2) {
    const double i0s = I0(s);
    const double ratio = K0(s) / i0s;
    const double ts = t * s;
    double num = 1.0 - ts * K1(ts);
    if (ratio > 0) num -= s * ratio * t * I1(ts);
    return num / (1.0 - 1.0 / i0s);
  }
  // sinh(s(1-t))/sinh(s) and cosh(s(1-t))/sinh(s), written with decaying exponentials
  // 1 - e^{-x} is formed with expm1 to avoid cancellation at small s
  const double one_m_em2s = -std::expm1(-2 * s);
  const double em2st = std::exp(-2 * s * (1 - t));
  const double est = std::exp(-s * t);
  const double sh_ratio = est * -std::expm1(-2 * s * (1 - t)) / one_m_em2s;
  const double ch_ratio = est * (1 + em2st) / one_m_em2s;
  const double num = 1.0 - sh_ratio - t * s * ch_ratio;
  return num / ball_pb(3, s);
}

// Radial density dC/dt.
double radial_pdf(int dim, double s, double t) {
  if (t <= 0 || t >= 1) return 0.0;
  if (s < kSmallS) return dim == 2 ? -4 * t * std::log(t) : 6 * t * (1 - t);
  if (dim == 2) {
    const double ts = t * s;
    return t * s * s * (K0(ts) - K0(s) / I0(s) * I0(ts)) / ball_pb(2, s);
  }
  const double sh_ratio = std::exp(-s * t) * std::expm1(-2 * s * (1 - t)) / std::expm1(-2 * s);
  return t * s * s * sh_ratio / ball_pb(3, s);
}

// Inverse of the radial CDF by safeguarded Newton iteration on [0, 1].
double radial_quantile(int dim, double s, double u) {
  double lo = 0.0, hi = 1.0, t = 0.5;
  for (int it = 0; it < 200; ++it) {
    const double c = radial_cdf(dim, s, t) - u;
    if (c < 0) lo = t; else hi = t;
    const double p = radial_pdf(dim, s, t);
    double tn = (p > 0) ? t - c / p : 0.5 * (lo + hi);
    if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
    if (std::fabs(tn - t) < 1e-15 || hi - lo < 1e-15) return tn;
    t = tn;
  }
  return t;
}

void uniform_direction(Stream* st, int dim, double* v) {
  if (dim == 2) {
    const double th = 2 * kPi * uniform(st);
    v[0] = std::cos(th);
    v[1] = std::sin(th);
    v[2] = 0;
  } else {
    const double z = 1 - 2 * uniform(st);
    const double ph = 2 * kPi * uniform(st);
    const double rr = std::sqrt(std::fmax(0.0, 1 - z * z));
    v[0] = rr * std::cos(ph);
    v[1] = rr * std::sin(ph);
    v[2] = z;
  }
}

// ------------------------------------------------------------------ one walk (Sec. 5.1, Alg. 1)

struct WalkResult {
  double value;
  uint64_t steps;   // distance queries
  int capped;
  int rr_killed;
  uint64_t inner;   // next flight: points sampled inside balls
};

// ------------------------------------------------------------------ gradient (supp. Sec. 2)
//
// grad_x G(x, y) and grad_x P(x, z) at the centre x of the ball (supplemental Sec. 1.3),
// as ratios to G(x, y) and P(x, z): the walk samples y ~ G/|G| and z uniform on the
// sphere, so these ratios are what multiplies the sampled terms. w = y - x or z - x.
void grad_ratio_green(int dim, const double* w, double R, double sb, double* out) {
  double r2 = 0;
  for (int i = 0; i < dim; ++i) r2 += w[i] * w[i];
  const double r = std::sqrt(r2);
  double f;
  if (!(sb > 0)) {
    f = dim == 2 ? (1 / r2 - 1 / (R * R)) / std::log(R / r) : (1 / (r2 * r) - 1 / (R * R * R)) / (1 / r - 1 / R);
  } else {
    const double k = std::sqrt(sb), s = R * k, a = r * k;
    if (dim == 2) {
      const double num = k / r * (K1(a) - K1(s) / I1(s) * I1(a));
      const double den = K0(a) - K0(s) / I0(s) * I0(a);
      f = num / den;
    } else {
      const double num = k / r2 * (std::exp(-a) * (1 + 1 / a) - (std::cosh(a) - std::sinh(a) / a) *
                                                                  std::exp(-s) * (1 + 1 / s) / (std::cosh(s) - std::sinh(s) / s));
      const double den = std::exp(-a) / r - std::exp(-s) / R * (std::sinh(a) / a) * (s / std::sinh(s));
      f = num / den;
    }
  }
  for (int i = 0; i < dim; ++i) out[i] = f * w[i];
}

void grad_ratio_poisson(int dim, const double* w, double R, double sb, double* out) {
  double f;
  if (!(sb > 0)) {
    f = (dim == 2 ? 2.0 : 3.0) / (R * R);
  } else {
    const double s = R * std::sqrt(sb);
    f = dim == 2 ? sb * I0(s) / (s * I1(s)) : sb * std::sinh(s) / (s * std::cosh(s) - std::sinh(s));
  }
  for (int i = 0; i < dim; ++i) out[i] = f * w[i];
}

// What the first ball of a walk leaves for the gradient estimate. With U = e^gamma u,
// U(x0) = S0 + w1 U(x1) for the first ball (source term S0, first step factor w1), and
// grad U(x0) has the same two terms with G replaced by grad_x G (and P by grad_x P on an
// exit): grad U ~ S0 a + (U - S0) b with a = grad G/G at y, b = a (volume) or grad P/P at
// z (exit). In u and relative to gamma(x0): grad u(x0) ~ A0 a + (A - A0) b - A grad gamma(x0).
struct FirstBall {
  bool set = false;
  double A0 = 0;
  double a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
};

// Streams of the branches of a split walk: branch b > 0 draws from the counter
// (block, walk, point, problem + b 2^16).
struct Family {
  uint64_t seed;
  uint32_t walk, point, problem;
  uint32_t branches = 0;   // branches started so far
};

double walk_branch(const OProblem& P, const OOptions& o, const double* x_start, double W, Coef cx, Stream* st,
                   Family& fam, WalkResult& res, FirstBall* first);

WalkResult walk(const OProblem& P, const OOptions& o, const double* x0, Stream* st, Family& fam,
                FirstBall* first = nullptr) {
  WalkResult res = {0, 0, 0, 0, 0};
  const Coef c0 = coefficients(P, x0);
  res.value = walk_branch(P, o, x0, 1.0, c0, st, fam, res, first);
  return res;
}

// One branch of a walk: from x with weight W (the product of the per-step factors that
// multiply the recursive estimate), returns its contribution sum_k W_k (source estimate
// at ball k) + W_K g(xbar_K). With ww_hi > 0 a branch whose |W| exceeds ww_hi splits into
// N branches of weight W/m, m = |W|/ww_hi, N = floor(m) with probability floor(m) + 1 - m
// and floor(m) + 1 otherwise (expected-value splitting, Sec. 6); E[N]/m = 1, so the
// estimate stays unbiased.
double walk_branch(const OProblem& P, const OOptions& o, const double* x_start, double W, Coef cx, Stream* st,
                   Family& fam, WalkResult& res, FirstBall* first) {
  const int dim = P.dim;
  const double sb = o.sigma_bar;
  double x[3] = {0, 0, 0};
  for (int i = 0; i < dim; ++i) x[i] = x_start[i];
  double A = 0.0;
  for (;;) {
    if (res.steps >= o.max_steps) {
      res.capped = 1;
      break;
    }
    double xbar[3] = {0, 0, 0};
    const double d = distance_to_boundary(P, x, xbar);
    res.steps++;
    if (d < P.epsilon) {               // epsilon shell: return g(xbar)  (R3)
      A += W * boundary_value(P, xbar);
      break;
    }
    const double R = d;                // largest ball centred at x inside the domain
    const double s = R * std::sqrt(sb);
    const double gnorm = ball_gnorm(dim, R, sb);
    const double pb = sb > 0 ? sb * gnorm : 0.0;  // probability of the volume term
    // y ~ G(x, .)/|G| : uniform direction and the radial law (supp. Sec. 1.4)
    double v[3];
    uniform_direction(st, dim, v);
    const double t = radial_quantile(dim, s, uniform(st));
    double y[3] = {0, 0, 0};
    for (int i = 0; i < dim; ++i) y[i] = x[i] + t * R * v[i];
    const Coef cy = coefficients(P, y);
    const double mu = uniform(st);
    const bool volume = mu < pb;
    // source estimate |G| f'(y) / (e^gamma(x)) = |G| e^{gamma(y)-gamma(x)} f(y)/alpha(y)
    const double A_before = A;
    if (o.variant == 0) {
      A += W * gnorm * std::exp(cy.gamma - cx.gamma) * cy.f / cy.alpha;
    } else if (volume) {
      A += W * std::exp(cy.gamma - cx.gamma) * cy.f / (cy.alpha * sb);
    }
    if (first && !first->set) {
      double w[3] = {0, 0, 0};
      for (int i = 0; i < dim; ++i) w[i] = y[i] - x[i];
      first->set = true;
      first->A0 = A - A_before;
      grad_ratio_green(dim, w, R, sb, first->a);
      for (int i = 0; i < 3; ++i) first->b[i] = first->a[i];
    }
    if (volume) {
      // null event: weight (1 - sigma'(y)/sigma_bar) e^{gamma(y) - gamma(x)}, continue at y
      W *= (1.0 - cy.sigma_prime / sb) * std::exp(cy.gamma - cx.gamma);
      for (int i = 0; i < dim; ++i) x[i] = y[i];
      cx = cy;
    } else {
      // boundary term: z uniform on the sphere, weight e^{gamma(z) - gamma(x)}
      double vz[3];
      uniform_direction(st, dim, vz);
      double z[3] = {0, 0, 0};
      for (int i = 0; i < dim; ++i) z[i] = x[i] + R * vz[i];
      if (first && res.steps == 1) {
        double w[3] = {0, 0, 0};
        for (int i = 0; i < dim; ++i) w[i] = R * vz[i];
        grad_ratio_poisson(dim, w, R, sb, first->b);
      }
      const Coef cz = coefficients(P, z);
      W *= std::exp(cz.gamma - cx.gamma);
      for (int i = 0; i < dim; ++i) x[i] = z[i];
      cx = cz;
    }
    if (o.russian_roulette && std::fabs(W) < o.ww_lo) {  // weight window, low side (R5)
      const double q = std::fabs(W) / o.ww_lo;
      if (uniform(st) < q) {
        W = (W < 0 ? -o.ww_lo : o.ww_lo);
      } else {
        res.rr_killed = 1;
        break;
      }
    } else if (o.ww_hi > 0 && std::fabs(W) > o.ww_hi && fam.branches < 65535) {  // high side
      const double m = std::fabs(W) / o.ww_hi;
      const double n = std::floor(m);
      const int N = uniform(st) < n + 1 - m ? (int)n : (int)n + 1;
      W /= m;
      for (int c = 1; c < N && fam.branches < 65535; ++c) {
        Stream child;
        stream_init(&child, fam.seed, fam.walk, fam.point, fam.problem + ((++fam.branches) << 16));
        A += walk_branch(P, o, x, W, cx, &child, fam, res, nullptr);
      }
    }
  }
  return A;
}

// ------------------------------------------------------------------ next flight (Sec. 5.2, Alg. 2)
//
// Off-centred Green's function and Poisson kernel of the ball B(c, R) for the operator
// Lap - sigma_bar, in the closed-form approximations of supplemental Sec. 1.2. With
// u = x - c, v = y - c, w = y - x and rho = (R^2 - u.v)/R:
//   G(x, y) = (Q(|w|) - Q(rho)) / (2 pi)                         (2D; 4 pi in 3D)
//   P(x, z) = (V(|w|) (|v|^2 - u.v)/(|w||v|) + V(rho) u.v/(R|v|)) / (2 pi)
// Q and V are the radial profiles of the centred Green's function and of its radial
// derivative (supplemental Sec. 1.1 and 1.2); at u = 0 both reduce to the centred
// expressions. sigma_bar = 0 takes the harmonic profiles Q = ln(R/r), V = 1/r (2D) and
// Q = 1/r - 1/R, V = 1/r^2 (3D).
double nf_Q(int dim, double r, double R, double sb) {
  if (sb <= 0) return dim == 2 ? std::log(R / r) : 1.0 / r - 1.0 / R;
  const double k = std::sqrt(sb);
  if (dim == 2) return K0(r * k) - K0(R * k) / I0(R * k) * I0(r * k);
  return std::exp(-r * k) / r - std::exp(-R * k) / R * (std::sinh(r * k) / (r * k)) * (R * k / std::sinh(R * k));
}

double nf_V(int dim, double r, double R, double sb) {
  if (sb <= 0) return dim == 2 ? 1.0 / r : 1.0 / (r * r);
  const double k = std::sqrt(sb);
  if (dim == 2) return k * (K1(r * k) + K0(R * k) / I0(R * k) * I1(r * k));
  const double a = r * k;
  return k / r * (std::exp(-a) * (1 + 1 / a) + std::exp(-R * k) / std::sinh(R * k) * (std::cosh(a) - std::sinh(a) / a));
}

double nf_green(int dim, const double* u, const double* v, double R, double sb) {
  double w2 = 0, uv = 0;
  for (int i = 0; i < dim; ++i) {
    w2 += (v[i] - u[i]) * (v[i] - u[i]);
    uv += u[i] * v[i];
  }
  const double rho = (R * R - uv) / R;
  const double c = dim == 2 ? 1.0 / (2 * kPi) : 1.0 / (4 * kPi);
  return c * (nf_Q(dim, std::sqrt(w2), R, sb) - nf_Q(dim, rho, R, sb));
}

double nf_poisson(int dim, const double* u, const double* v, double R, double sb) {
  double w2 = 0, uv = 0, v2 = 0;
  for (int i = 0; i < dim; ++i) {
    w2 += (v[i] - u[i]) * (v[i] - u[i]);
    uv += u[i] * v[i];
    v2 += v[i] * v[i];
  }
  const double w = std::sqrt(w2), vn = std::sqrt(v2);
  const double rho = (R * R - uv) / R;
  const double c = dim == 2 ? 1.0 / (2 * kPi) : 1.0 / (4 * kPi);
  return c * (nf_V(dim, w, R, sb) * (v2 - uv) / (w * vn) + nf_V(dim, rho, R, sb) * uv / (R * vn));
}

// Exact off-centred kernels, from the separable series of supplemental Sec. 1.2. They
// serve the oracle's exact-kernel next-flight walk (variant 3), which pins the walk's
// bookkeeping independently of the approximations. The free-space part of G is summed in
// closed form by the addition theorem of the screened kernel, so only the regular part
// is a series (theta: angle between u and v; a = |u|, b = |v|):
//   2D: G = (K0(k|w|) - sum_n c_n cos(n theta) I_n(ka) I_n(kb) K_n(kR)/I_n(kR)) / (2 pi)
//   3D: G = (e^{-k|w|}/|w| - (2k/pi) sum_n (2n+1) P_n(cos theta) i_n(ka) i_n(kb) k_n(kR)/i_n(kR)) / (4 pi)
//   2D: P = sum_n c_n cos(n theta) I_n(ka)/I_n(kR) / (2 pi R)
//   3D: P = sum_n (2n+1) P_n(cos theta) i_n(ka)/i_n(kR) / (4 pi R^2)
// with c_0 = 1, c_n = 2, i_n(x) = sqrt(pi/2x) I_{n+1/2}(x), k_n(x) = sqrt(pi/2x) K_{n+1/2}(x).
// Orders are stepped through ratios (I_v/I_{v-1} by backward recurrence, K_{v+1}/K_v by
// forward recurrence) in logarithms, so no term overflows.
const int kSeriesMax = 20000;

// log I_n(x) (2D) or log i_n(x) (3D), n = 0 .. N-1; at x = 0 only n = 0 is nonzero (= 1).
void log_i_orders(int dim, double x, int N, std::vector<double>& out) {
  out.assign(N, -1e300);
  if (x <= 0) {
    out[0] = 0.0;
    return;
  }
  const double v0 = dim == 2 ? 0.0 : 0.5;
  std::vector<double> r(N + 1, 0.0);   // r[n] = I_{v0+n}(x) / I_{v0+n-1}(x)
  double rr = 0.0;
  for (int n = N + 80; n >= 1; --n) {
    rr = 1.0 / (2.0 * (v0 + n) / x + rr);
    if (n <= N) r[n] = rr;
  }
  out[0] = std::log(std::cyl_bessel_i(v0, x)) + (dim == 3 ? 0.5 * std::log(kPi / (2 * x)) : 0.0);
  for (int n = 1; n < N; ++n) out[n] = out[n - 1] + std::log(r[n]);
}

// log K_n(x) (2D) or log k_n(x) (3D), n = 0 .. N-1, x > 0.
void log_k_orders(int dim, double x, int N, std::vector<double>& out) {
  out.assign(N, 0.0);
  const double v0 = dim == 2 ? 0.0 : 0.5;
  const double k0 = std::cyl_bessel_k(v0, x), k1 = std::cyl_bessel_k(v0 + 1.0, x);
  const double sh = dim == 3 ? 0.5 * std::log(kPi / (2 * x)) : 0.0;
  out[0] = std::log(k0) + sh;
  double s = k1 / k0;                  // K_{v0+n}/K_{v0+n-1}
  for (int n = 1; n < N; ++n) {
    if (n > 1) s = 1.0 / s + 2.0 * (v0 + n - 1) / x;
    out[n] = out[n - 1] + std::log(s);
  }
}

int series_terms(double q) {
  if (q <= 0) return 2;
  return std::min(kSeriesMax, 8 + (int)(std::log(1e-18) / std::log(std::fmin(q, 0.99999))));
}

// sum_n c_n cos(n theta) t_n (2D) or sum_n (2n+1) P_n(cos theta) t_n (3D)
double angular_sum(int dim, double cth, const std::vector<double>& logt) {
  const double theta = std::acos(cth);
  double tot = 0, pm2 = 1, pm1 = cth;
  for (size_t n = 0; n < logt.size(); ++n) {
    const double t = logt[n] < -700 ? 0.0 : std::exp(logt[n]);
    if (dim == 2) {
      tot += (n == 0 ? 1.0 : 2.0 * std::cos(n * theta)) * t;
    } else {
      double Pn = n == 0 ? 1.0 : cth;
      if (n >= 2) {
        Pn = ((2.0 * n - 1.0) * cth * pm1 - (n - 1.0) * pm2) / n;
        pm2 = pm1;
        pm1 = Pn;
      }
      tot += (2.0 * n + 1.0) * Pn * t;
    }
  }
  return tot;
}

double cos_angle(int dim, const double* u, const double* v) {
  double uv = 0, a2 = 0, b2 = 0;
  for (int i = 0; i < dim; ++i) {
    uv += u[i] * v[i];
    a2 += u[i] * u[i];
    b2 += v[i] * v[i];
  }
  if (a2 <= 0 || b2 <= 0) return 1.0;
  return std::fmax(-1.0, std::fmin(1.0, uv / std::sqrt(a2 * b2)));
}

double nf_green_exact(int dim, const double* u, const double* v, double R, double sb) {
  double w2 = 0, a2 = 0, b2 = 0;
  for (int i = 0; i < dim; ++i) {
    w2 += (v[i] - u[i]) * (v[i] - u[i]);
    a2 += u[i] * u[i];
    b2 += v[i] * v[i];
  }
  const double k = std::sqrt(sb), w = std::sqrt(w2), a = std::sqrt(a2), b = std::sqrt(b2);
  const int N = series_terms(a * b / (R * R));
  std::vector<double> la, lb, li, lk;
  log_i_orders(dim, k * a, N, la);
  log_i_orders(dim, k * b, N, lb);
  log_i_orders(dim, k * R, N, li);
  log_k_orders(dim, k * R, N, lk);
  for (int n = 0; n < N; ++n) la[n] += lb[n] + lk[n] - li[n];
  const double reg = angular_sum(dim, cos_angle(dim, u, v), la);
  if (dim == 2) return (K0(k * w) - reg) / (2 * kPi);
  return (std::exp(-k * w) / w - 2 * k / kPi * reg) / (4 * kPi);
}

double nf_poisson_exact(int dim, const double* u, const double* v, double R, double sb) {
  double a2 = 0;
  for (int i = 0; i < dim; ++i) a2 += u[i] * u[i];
  const double k = std::sqrt(sb), a = std::sqrt(a2);
  const int N = series_terms(a / R);
  std::vector<double> la, li;
  log_i_orders(dim, k * a, N, la);
  log_i_orders(dim, k * R, N, li);
  for (int n = 0; n < N; ++n) la[n] -= li[n];
  const double tot = angular_sum(dim, cos_angle(dim, u, v), la);
  return dim == 2 ? tot / (2 * kPi * R) : tot / (4 * kPi * R * R);
}

// Uniform point in the unit ball, by the radius law r = U^{1/n} and a uniform direction.
void uniform_in_ball(Stream* st, int dim, double* p) {
  double v[3];
  uniform_direction(st, dim, v);
  const double r = std::pow(uniform(st), 1.0 / dim);
  for (int i = 0; i < 3; ++i) p[i] = r * v[i];
}

// One walk of Alg. 2 in the transformed unknown U = e^gamma u (Sec. 4.1, App. A). For the
// ball B(x_k, R) with exit point z uniform on its sphere, the unrolled series
//   T_k = sum_j P(x^j, z) |dB| prod_{l<j} theta_l,
//   S_k = sum_{j>=1} f'(x^j)/(sigma_bar - sigma'(x^j)) prod_{l<j} theta_l,
//   theta_l = G(x^l, x^{l+1}) (sigma_bar - sigma'(x^{l+1})) |B|,
// with x^0 = x_k and x^{l+1} uniform in the ball, give U(x_k) ~ T_k U(z) + S_k; the number
// of terms is set by Russian roulette on the running throughput min(1, prod theta).
// The (sigma_bar - sigma') of the last theta cancels against the division in S (the
// term is f' G |B| times the previous throughput), so sigma' = sigma_bar needs no
// special case. Unrolled over the balls, with f' = e^gamma f/alpha:
//   u(x_0) ~ e^{-gamma(x_0)} [sum_k (prod_{i<k} T_i) S_k + (prod_{i<K} T_i) e^{gamma(x_K)} g(xbar_K)],
// kept here relative to gamma(x_0) so that no absolute e^gamma is formed.
WalkResult walk_next_flight(const OProblem& P, const OOptions& o, const double* x0, Stream* st) {
  const int dim = P.dim;
  const double sb = o.sigma_bar;
  const bool exact = o.variant == 3;   // exact series kernels instead of the approximations
  double x[3] = {0, 0, 0};
  for (int i = 0; i < dim; ++i) x[i] = x0[i];
  const double g0 = coefficients(P, x).gamma;
  const double unit_ball = dim == 2 ? kPi : 4.0 * kPi / 3.0;
  const double unit_sphere = dim == 2 ? 2 * kPi : 4 * kPi;
  double W = 1.0;   // prod_{i<k} T_i
  double A = 0.0;
  WalkResult res = {0, 0, 0, 0, 0};
  for (;;) {
    if (res.steps >= o.max_steps) {
      res.capped = 1;
      break;
    }
    double xbar[3] = {0, 0, 0};
    const double d = distance_to_boundary(P, x, xbar);
    res.steps++;
    if (d < P.epsilon) {
      A += W * std::exp(coefficients(P, x).gamma - g0) * boundary_value(P, xbar);
      break;
    }
    const double R = d;
    const double vol = unit_ball * std::pow(R, dim);
    const double area = unit_sphere * std::pow(R, dim - 1);
    double vz[3];
    uniform_direction(st, dim, vz);
    double zr[3] = {0, 0, 0};     // z - x_k
    for (int i = 0; i < dim; ++i) zr[i] = R * vz[i];
    double xc[3] = {0, 0, 0};     // current inner point, relative to x_k
    double T = 0, S = 0, beta = 1;
    for (;;) {
      T += (exact ? nf_poisson_exact(dim, xc, zr, R, sb) : nf_poisson(dim, xc, zr, R, sb)) * area * beta;
      const double prr = std::fmin(1.0, beta);
      if (prr < uniform(st)) break;
      beta /= prr;
      double xn[3] = {0, 0, 0};
      uniform_in_ball(st, dim, xn);
      for (int i = 0; i < dim; ++i) xn[i] *= R;
      double y[3] = {0, 0, 0};
      for (int i = 0; i < dim; ++i) y[i] = x[i] + xn[i];
      const Coef cy = coefficients(P, y);
      const double gv = (exact ? nf_green_exact(dim, xc, xn, R, sb) : nf_green(dim, xc, xn, R, sb)) * vol;
      S += beta * gv * std::exp(cy.gamma - g0) * cy.f / cy.alpha;
      beta *= gv * (sb - cy.sigma_prime);
      res.inner++;
      for (int i = 0; i < dim; ++i) xc[i] = xn[i];
    }
    A += W * S;
    W *= T;
    for (int i = 0; i < dim; ++i) x[i] += zr[i];
  }
  res.value = A;
  return res;
}

bool point_ok(const OProblem& P, const double* x) {
  for (int i = 0; i < P.dim; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

}  // namespace

// ====================================================================== C entry points

extern "C" {

void oracle_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  philox4x32_10(ctr, key, out);
}

// n uniform doubles of the stream of (seed, walk, point, problem).
void oracle_uniforms(uint64_t seed, uint32_t walk, uint32_t point, uint32_t problem, int64_t n, double* out) {
  Stream st;
  stream_init(&st, seed, walk, point, problem);
  for (int64_t i = 0; i < n; ++i) out[i] = uniform(&st);
}

// Off-centred Green's function G(x, y) and Poisson kernel P(x, z) of the ball B(c, R) for
// Lap - sigma_bar in the approximations of supplemental Sec. 1.2; u = x - c, v = y - c (or
// z - c). which: 0 = G, 1 = P, 2 = exact G, 3 = exact P (series). u, v: [n][dim].
void oracle_nf_kernel(int which, int dim, const double* u, const double* v, int64_t n, double R, double sigma_bar,
                      double* out) {
  for (int64_t i = 0; i < n; ++i)
    out[i] = which == 0 ? nf_green(dim, u + i * dim, v + i * dim, R, sigma_bar)
             : which == 1 ? nf_poisson(dim, u + i * dim, v + i * dim, R, sigma_bar)
             : which == 2 ? nf_green_exact(dim, u + i * dim, v + i * dim, R, sigma_bar)
                          : nf_poisson_exact(dim, u + i * dim, v + i * dim, R, sigma_bar);
}

// grad_x G(x, y)/G(x, y) (which = 0) or grad_x P(x, z)/P(x, z) (which = 1) at the centre
// x of the ball of radius R; w = y - x or z - x, out: [dim].
void oracle_grad_ratio(int which, int dim, const double* w, double R, double sigma_bar, double* out) {
  if (which == 0) grad_ratio_green(dim, w, R, sigma_bar, out);
  else grad_ratio_poisson(dim, w, R, sigma_bar, out);
}

double oracle_ball_pb(int dim, double s) { return ball_pb(dim, s); }
double oracle_ball_gnorm(int dim, double R, double sigma_bar) { return ball_gnorm(dim, R, sigma_bar); }
double oracle_radial_cdf(int dim, double s, double t) { return radial_cdf(dim, s, t); }
double oracle_radial_pdf(int dim, double s, double t) { return radial_pdf(dim, s, t); }
double oracle_radial_quantile(int dim, double s, double u) { return radial_quantile(dim, s, u); }
void oracle_radial_cdf_many(int dim, double s, const double* t, int64_t n, double* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = radial_cdf(dim, s, t[i]);
}
double oracle_bessel(int which, double x) {
  switch (which) {
    case 0: return I0(x);
    case 1: return I1(x);
    case 2: return K0(x);
    default: return K1(x);
  }
}

// Per point: alpha, gamma, sigma', f, f', g (boundary field evaluated at the point).
void oracle_coefficients(const OProblem* P, const double* pts, int64_t n, double* out) {
  for (int64_t i = 0; i < n; ++i) {
    const double* x = pts + i * P->dim;
    const Coef c = coefficients(*P, x);
    double* o = out + 6 * i;
    o[0] = c.alpha;
    o[1] = c.gamma;
    o[2] = c.sigma_prime;
    o[3] = c.f;
    o[4] = c.f_prime;
    o[5] = boundary_value(*P, x);
  }
}

// accel = 1 answers polygon and mesh queries through the oracle's BVH (same minimum).
void oracle_distance(const OProblem* P_in, const double* pts, int64_t n, double* d, double* xbar, int accel) {
  OProblem Pl = *P_in;
  OBvh bvh;
  Pl.accel = nullptr;
  if (accel && (Pl.geom.kind == G_POLYGON || Pl.geom.kind == G_TRIMESH)) {
    bvh_build(Pl.geom, Pl.dim, bvh);
    Pl.accel = &bvh;
  }
  for (int64_t i = 0; i < n; ++i) d[i] = distance_to_boundary(Pl, pts + i * Pl.dim, xbar + i * Pl.dim);
}

// sigma' min and max over the given sample points (the default majorant of Sec. 5.1 /
// Sec. 7.1 is max - min over the domain; the caller supplies interior samples).
void oracle_sigma_prime_range(const OProblem* P, const double* pts, int64_t n, double* mn, double* mx) {
  double lo = INFINITY, hi = -INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    const double sp = coefficients(*P, pts + i * P->dim).sigma_prime;
    lo = std::fmin(lo, sp);
    hi = std::fmax(hi, sp);
  }
  *mn = lo;
  *mx = hi;
}

// Monte Carlo solve: per point, walks j = walk_offset .. walk_offset + n_walks - 1.
// Outputs (per point): sum of estimates, sum of squares, total distance queries.
// counters: [0] invalid points, [1] capped walks, [2] Russian-roulette kills,
// [3] next flight: points sampled inside balls.
int oracle_solve_grad(const OProblem* P, const OOptions* o, const double* pts, int64_t n_points, double* sum,
                      double* sum_sq, uint64_t* steps, uint64_t* counters, double* gsum, double* gsum_sq);

int oracle_solve(const OProblem* P, const OOptions* o, const double* pts, int64_t n_points,
                 double* sum, double* sum_sq, uint64_t* steps, uint64_t* counters) {
  return oracle_solve_grad(P, o, pts, n_points, sum, sum_sq, steps, counters, nullptr, nullptr);
}

// As oracle_solve, and with gsum / gsum_sq (both [n][dim], or null) the sums of the
// per-walk gradient estimates and of their squares (supplemental Sec. 2; delta tracking
// only).
int oracle_solve_grad(const OProblem* P_in, const OOptions* o, const double* pts, int64_t n_points, double* sum,
                      double* sum_sq, uint64_t* steps, uint64_t* counters, double* gsum, double* gsum_sq) {
  // the timing mode's BVH lives for this call; the walk sees it through P->accel
  OProblem Pl = *P_in;
  OBvh bvh;
  Pl.accel = nullptr;
  if (o->accel && (Pl.geom.kind == G_POLYGON || Pl.geom.kind == G_TRIMESH)) {
    bvh_build(Pl.geom, Pl.dim, bvh);
    Pl.accel = &bvh;
  }
  const OProblem* P = &Pl;
  if (gsum && o->variant >= 2) return 1;
  if (o->sigma_bar < 0) return 1;
  if (o->variant < 0 || o->variant > 3) return 1;
  if (o->variant >= 2 && (o->russian_roulette || o->ww_hi > 0)) return 1;   // next flight has its own roulette
  if (o->ww_hi > 0 && (o->problem_index >= 65536 || (o->russian_roulette && !(o->ww_hi > o->ww_lo)))) return 1;
  if (o->variant == 3 && !(o->sigma_bar > 0)) return 1;    // exact kernels need sigma_bar > 0
  std::atomic<int64_t> next(0);
  std::atomic<uint64_t> bad(0), capped(0), killed(0), inner(0);
  auto worker = [&]() {
    for (;;) {
      const int64_t i = next.fetch_add(1);
      if (i >= n_points) break;
      const double* x0 = pts + i * P->dim;
      if (!point_ok(*P, x0)) {
        sum[i] = NAN;
        sum_sq[i] = NAN;
        steps[i] = 0;
        bad++;
        continue;
      }
      // Neumaier-compensated sums
      double s = 0, cs = 0, q = 0, cq = 0;
      double gs[3] = {0, 0, 0}, gq[3] = {0, 0, 0};
      const int dim = P->dim;
      const Coef c0 = coefficients(*P, x0);
      uint64_t nst = 0;
      for (uint64_t j = 0; j < o->n_walks; ++j) {
        Stream st;
        stream_init(&st, o->seed, (uint32_t)(o->walk_offset + j), (uint32_t)i, o->problem_index);
        Family fam;
        fam.seed = o->seed;
        fam.walk = (uint32_t)(o->walk_offset + j);
        fam.point = (uint32_t)i;
        fam.problem = o->problem_index;
        FirstBall fb;
        const WalkResult r = o->variant >= 2 ? walk_next_flight(*P, *o, x0, &st)
                                             : walk(*P, *o, x0, &st, fam, gsum ? &fb : nullptr);
        if (gsum) {
          for (int k = 0; k < dim; ++k) {
            const double g = fb.A0 * fb.a[k] + (r.value - fb.A0) * fb.b[k] - r.value * c0.grad_gamma[k];
            gs[k] += g;
            gq[k] += g * g;
          }
        }
        nst += r.steps;
        capped += r.capped;
        killed += r.rr_killed;
        inner += r.inner;
        const double v = r.value, v2 = r.value * r.value;
        double t = s + v;
        cs += std::fabs(s) >= std::fabs(v) ? (s - t) + v : (v - t) + s;
        s = t;
        t = q + v2;
        cq += std::fabs(q) >= std::fabs(v2) ? (q - t) + v2 : (v2 - t) + q;
        q = t;
      }
      sum[i] = s + cs;
      sum_sq[i] = q + cq;
      steps[i] = nst;
      if (gsum)
        for (int k = 0; k < dim; ++k) {
          gsum[i * dim + k] = gs[k];
          gsum_sq[i * dim + k] = gq[k];
        }
    }
  };
  int nt = o->threads > 0 ? o->threads : (int)std::thread::hardware_concurrency();
  if (nt < 1) nt = 1;
  std::vector<std::thread> pool;
  for (int k = 0; k < nt; ++k) pool.emplace_back(worker);
  for (auto& th : pool) th.join();
  counters[0] = bad;
  counters[1] = capped;
  counters[2] = killed;
  counters[3] = inner;
  return 0;
}

}  // extern "C"
