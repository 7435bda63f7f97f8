// Kernels around the walker (exact per-point sums, classification, sigma' sampling,
// diagnostics) and the host-side launchers; the walker itself is in wos_walker.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>

#include "wos_device.h"
#include "wos_launch.h"

namespace wos {

// ------------------------------------------------------------------ reduce (exact sums)

// Carries of limbs L[0..5] so that L[0..4] lie in [0, 2^32); the top limb keeps the sign.
__device__ __forceinline__ void fx_normalize(int64_t* L) {
#pragma unroll
  for (int k = 0; k < kFxLimbs - 1; ++k) {
    const int64_t c = L[k] >> 32;   // floor division by 2^32
    L[k] -= c * 4294967296ll;
    L[k + 1] += c;
  }
}

// The value sum_k L[k] 2^(32k - 96) of normalised limbs, summed in a fixed order with
// the Neumaier correction (each term is exact in double).
__device__ __forceinline__ double fx_value(const int64_t* L) {
  double s = 0, c = 0;
#pragma unroll
  for (int k = 0; k < kFxLimbs; ++k) {
    const double t = (double)L[k] * __builtin_ldexp(1.0, 32 * k - kFxFracBits);
    const double u = s + t;
    c += fabs(s) >= fabs(t) ? (s - u) + t : (t - u) + s;
    s = u;
  }
  return s + c;
}

// Adds the limbs of `words` (a slot field) to L and normalises.
__device__ __forceinline__ void fx_accumulate(int64_t* L, const uint64_t* words) {
#pragma unroll
  for (int k = 0; k < kFxLimbs; ++k) L[k] += (int64_t)words[k];
  fx_normalize(L);
}

// Per point: the exact sums of its slots (one per tile it was cut into), converted to
// double once and added into the caller's accumulators. With grad_dim > 0 also the sums
// of the gradient components (supplemental Sec. 2).
template <int GD>
__global__ void reduce_kernel(DevItem it, const uint64_t* __restrict__ slots, int slot_words) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t capped = 0, killed = 0;
  if (p < it.n_points) {
    const uint32_t spp = it.tiles_per_point > 0u ? it.tiles_per_point : 1u;
    if (!it.inside[p]) {
      const double nan = __builtin_nan("");
      it.sum[p] += nan;
      it.sum_sq[p] += nan;
#pragma unroll
      for (int c = 0; c < GD; ++c) {
        it.grad_sum[p * GD + c] += nan;
        it.grad_sum_sq[p * GD + c] += nan;
      }
    } else {
      int64_t S[kFxLimbs] = {0}, Q[kFxLimbs] = {0};
      int64_t GS[GD > 0 ? GD : 1][kFxLimbs], GQ[GD > 0 ? GD : 1][kFxLimbs];
#pragma unroll
      for (int c = 0; c < (GD > 0 ? GD : 1); ++c)
#pragma unroll
        for (int k = 0; k < kFxLimbs; ++k) GS[c][k] = GQ[c][k] = 0;
      uint64_t nst = 0, bad = 0;
      for (uint32_t k = 0; k < spp; ++k) {
        const uint64_t* w = slots + (size_t)(it.slot_base + (uint64_t)p * spp + k) * slot_words;
        fx_accumulate(S, w + kSlotSum);
        fx_accumulate(Q, w + kSlotSumSq);
        nst += w[kSlotSteps];
        const uint64_t f = w[kSlotFlags];
        capped += f & ((1ull << kFlagShiftKilled) - 1);
        killed += (f >> kFlagShiftKilled) & ((1ull << (kFlagShiftBad - kFlagShiftKilled)) - 1);
        bad += f >> kFlagShiftBad;
#pragma unroll
        for (int c = 0; c < GD; ++c) {
          fx_accumulate(GS[c], w + kSlotGrad + 2 * kFxLimbs * c);
          fx_accumulate(GQ[c], w + kSlotGrad + 2 * kFxLimbs * c + kFxLimbs);
        }
      }
      const double nan = __builtin_nan("");
      it.sum[p] += bad ? nan : fx_value(S);
      it.sum_sq[p] += bad ? nan : fx_value(Q);
#pragma unroll
      for (int c = 0; c < GD; ++c) {
        it.grad_sum[p * GD + c] += bad ? nan : fx_value(GS[c]);
        it.grad_sum_sq[p * GD + c] += bad ? nan : fx_value(GQ[c]);
      }
      it.n_steps[p] += nst;
    }
    it.n_walks[p] += it.walks;
  }
  if (it.counters) {
    for (int off = 32; off > 0; off >>= 1) {
      capped += __shfl_xor(capped, off);
      killed += __shfl_xor(killed, off);
    }
    if (__lane_id() == 0) {
      if (capped) atomicAdd((unsigned long long*)&it.counters[1], (unsigned long long)capped);
      if (killed) atomicAdd((unsigned long long*)&it.counters[2], (unsigned long long)killed);
    }
  }
}

// Zeroes the slots (and the tile counter) before a walker launch; a kernel rather than a
// memset node, so that it can be captured in the plan's graph.
__global__ void clear_kernel(uint64_t* __restrict__ p, uint64_t n, uint32_t* counter) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
}

__global__ void reset_kernel(uint32_t* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

__global__ void set_params_kernel(LaunchParams* lp, uint64_t seed, uint64_t add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    lp->seed = seed;
    lp->walk_offset_add = add;
  }
}

// ------------------------------------------------------------------ inside classification (FP64)

template <int DIM, int GEOM>
__device__ bool inside_point(G<DevGeometry<double>>& g, const double* x) {
#pragma unroll
  for (int i = 0; i < DIM; ++i)
    if (!isfinite(x[i])) return false;
  if (GEOM == GK_BALL) {
    double r2 = 0;
    for (int i = 0; i < DIM; ++i) r2 += (x[i] - g.center[i]) * (x[i] - g.center[i]);
    return r2 < g.radius * g.radius;
  } else if (GEOM == GK_BOX) {
    for (int i = 0; i < DIM; ++i)
      if (!(x[i] > g.lo[i] && x[i] < g.hi[i])) return false;
    return true;
  } else if (GEOM == GK_SDF) {
    int act;
    return sdf_value<double, DIM>(g, x, &act) < 0.0;
  } else if (GEOM == GK_POLYGON) {
    // even-odd crossing count of a horizontal ray
    bool in = false;
    for (int j = 0; j < g.n_prims; ++j) {
      const WOS_GLOBAL double* s = gptr(g.prims) + (size_t)j * kPrimStride2;
      const double ay = s[1], by = s[3];
      if ((ay > x[1]) != (by > x[1])) {
        const double xi = s[0] + (x[1] - ay) * (s[2] - s[0]) / (by - ay);
        if (x[0] < xi) in = !in;
      }
    }
    return in;
  } else {
    // generalized winding number: sum of signed solid angles / 4 pi
    // (Van Oosterom and Strackee: tan(Omega/2) = det[a b c] / (|a||b||c| + (a.b)|c| + (a.c)|b| + (b.c)|a|))
    double w = 0;
    for (int j = 0; j < g.n_prims; ++j) {
      const WOS_GLOBAL double* t = gptr(g.prims) + (size_t)j * kPrimStride3;
      double a[3], b[3], c[3];
      for (int i = 0; i < 3; ++i) {
        a[i] = t[i] - x[i];
        b[i] = t[3 + i] - x[i];
        c[i] = t[6 + i] - x[i];
      }
      const double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
      const double lb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
      const double lc = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
      const double det = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                         a[2] * (b[0] * c[1] - b[1] * c[0]);
      const double ab = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
      const double ac = a[0] * c[0] + a[1] * c[1] + a[2] * c[2];
      const double bc = b[0] * c[0] + b[1] * c[1] + b[2] * c[2];
      w += 2.0 * atan2(det, la * lb * lc + ab * lc + ac * lb + bc * la);
    }
    return fabs(w) > 2.0 * M_PI;
  }
}

template <int DIM, int GEOM>
__global__ void classify_kernel(const DevProblem<double>* P, const double* pts, int64_t n, int8_t* inside,
                                uint64_t* counters) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  if (i < n) {
    const bool in = inside_point<DIM, GEOM>(gptr(P)->geom, pts + i * DIM);
    inside[i] = in ? 1 : 0;
    bad = !in;
  }
  if (counters) {
    const uint64_t m = __ballot(bad);
    if (__lane_id() == 0 && m) atomicAdd((unsigned long long*)&counters[0], (unsigned long long)__popcll(m));
  }
}

// ------------------------------------------------------------------ sigma' sampling (FP64)
// out per block: [min sigma', max sigma', min alpha, min sigma, #non-finite, #samples]

template <int DIM, int GEOM>
__global__ void sigma_sample_kernel(const DevProblem<double>* P, double lo0, double lo1, double lo2, double h0,
                                    double h1, double h2, int grid, double* out) {
  const double lo[3] = {lo0, lo1, lo2}, h[3] = {h0, h1, h2};
  double mn = __builtin_huge_val(), mx = -__builtin_huge_val(), amin = __builtin_huge_val(),
         smin = __builtin_huge_val(), bad = 0, cnt = 0;
  const int64_t total = DIM == 2 ? (int64_t)grid * grid : (int64_t)grid * grid * grid;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = k;
    double x[DIM];
    for (int i = 0; i < DIM; ++i) {
      x[i] = lo[i] + h[i] * ((double)(r % grid) + 0.5);
      r /= grid;
    }
    G<DevProblem<double>>& PR = *gptr(P);
    if (!inside_point<DIM, GEOM>(PR.geom, x)) continue;
    const PointCoef<double> c = point_coef<double, DIM, false>(PR, x);
    const double sig = field_eval<double, DIM, false>(PR.sigma, x).v;
    cnt += 1;
    if (!isfinite(c.sigma_prime) || !isfinite(c.alpha)) {
      bad += 1;
      continue;
    }
    mn = fmin(mn, c.sigma_prime);
    mx = fmax(mx, c.sigma_prime);
    amin = fmin(amin, c.alpha);
    smin = fmin(smin, sig);
  }
  __shared__ double red[6][256];
  const int t = threadIdx.x;
  red[0][t] = mn; red[1][t] = mx; red[2][t] = amin; red[3][t] = smin; red[4][t] = bad; red[5][t] = cnt;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) {
      red[0][t] = fmin(red[0][t], red[0][t + s]);
      red[1][t] = fmax(red[1][t], red[1][t + s]);
      red[2][t] = fmin(red[2][t], red[2][t + s]);
      red[3][t] = fmin(red[3][t], red[3][t + s]);
      red[4][t] += red[4][t + s];
      red[5][t] += red[5][t + s];
    }
    __syncthreads();
  }
  if (t == 0)
    for (int k = 0; k < 6; ++k) out[blockIdx.x * 6 + k] = red[k][0];
}

// ------------------------------------------------------------------ diagnostics

template <typename T, int DIM>
__global__ void coef_kernel(const DevProblem<T>* P, const double* pts, int64_t n, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T x[DIM];
  for (int k = 0; k < DIM; ++k) x[k] = (T)pts[i * DIM + k];
  G<DevProblem<T>>& PR = *gptr(P);
  const PointCoef<T> c = point_coef<T, DIM, true>(PR, x);
  double* o = out + i * 6;
  o[0] = c.alpha;
  o[1] = c.gamma;
  o[2] = c.sigma_prime;
  o[3] = (double)c.f_over_alpha * (double)c.alpha;
  o[4] = (double)m_exp(c.gamma) * (double)c.f_over_alpha;
  o[5] = boundary_value<T, DIM>(PR, x);
}

// gamma(x0) of every interior query point: the same for all walks of a point, so each
// walk starts from it instead of spending an iteration of the walker on it.
template <typename T, int DIM>
__global__ void gamma0_kernel(const DevProblem<T>* P, const double* pts, int64_t n, const int8_t* inside, T* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T g = 0;
  if (inside[i]) {
    T x[DIM];
    for (int k = 0; k < DIM; ++k) x[k] = (T)pts[i * DIM + k];
    g = point_gamma<T, DIM>(*gptr(P), x);
  }
  out[i] = g;
}

template <typename T, int DIM, int GEOM>
__global__ void distance_kernel(const DevProblem<T>* P, const double* pts, int64_t n, double* d, double* xb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T x[DIM], q[DIM];
  for (int k = 0; k < DIM; ++k) x[k] = (T)pts[i * DIM + k];
  int prim;
  d[i] = boundary_distance<T, DIM, GEOM>(gptr(P)->geom, x, &prim);
  closest_point<T, DIM, GEOM>(gptr(P)->geom, x, prim, q);
  for (int k = 0; k < DIM; ++k) xb[i * DIM + k] = q[k];
}

template <typename T, int DIM>
__global__ void ball_kernel(const double* s, int64_t n, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // unit radius: sigma_bar = s^2
  const T si = (T)s[i];
  const bool harmonic = !(si > (T)0);
  const Ball<T, DIM> b = ball_terms<T, DIM>((T)1, si, harmonic ? (T)0 : (T)1 / (si * si), harmonic);
  out[2 * i] = b.pb;
  out[2 * i + 1] = b.gnorm;
}

template <typename T, int DIM>
__global__ void sample_kernel(double s, int64_t n, uint64_t seed, double* t, uint64_t* trials) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t tr = 0;
  if (i < n) {
    Rng rng;
    rng.set_key(seed);
    rng.init((uint32_t)i, 0, 0);
    const T sv = (T)s;
    const bool harmonic = !(sv > (T)0);
    const Ball<T, DIM> b = ball_terms<T, DIM>((T)1, sv, harmonic ? (T)0 : (T)1 / (sv * sv), harmonic);
    t[i] = sample_radius<T, DIM>(rng, sv, b, harmonic, tr);
  }
  if (trials) {
    uint64_t v = tr;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (__lane_id() == 0 && v) atomicAdd((unsigned long long*)trials, (unsigned long long)v);
  }
}

__global__ void philox_kernel(const uint32_t* ctr, uint64_t key, int64_t n, uint32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint4 c = make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
  const uint4 r = philox4x32_10(c, make_uint2((uint32_t)key, (uint32_t)(key >> 32)));
  out[4 * i] = r.x;
  out[4 * i + 1] = r.y;
  out[4 * i + 2] = r.z;
  out[4 * i + 3] = r.w;
}

template <typename T>
__global__ void bessel_kernel(int which, const double* x, int64_t n, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T v = (T)x[i];
  out[i] = which == 0 ? (double)bessel_i0e<T>(v)
           : which == 1 ? (double)bessel_k0e<T>(v)
           : which == 2 ? (double)bessel_i1e<T>(v)
                        : (double)bessel_k1e<T>(v);
}

// Off-centred kernels of the next-flight walk at explicit points: which 0 = G(x, y) |B|,
// 1 = P(x, z) |dB|, for u = x - c, v = y - c (rows of [n][DIM]).
template <typename T, int DIM>
__global__ void offcentred_kernel(int which, T R, T sigma_bar, const double* u, const double* v, int64_t n,
                                  double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T uu[DIM], vv[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    uu[k] = (T)u[i * DIM + k];
    vv[k] = (T)v[i * DIM + k];
  }
  const bool harmonic = !(sigma_bar > (T)0);
  const T k = harmonic ? (T)0 : m_sqrt(sigma_bar);
  const Ball<T, DIM> b = ball_terms<T, DIM>(R, R * k, harmonic ? (T)0 : (T)1 / sigma_bar, harmonic);
  const NfBall<T, DIM> nb = nf_ball<T, DIM>(R, k, b.c2d);
  out[i] = which == 0 ? (double)nf_green_vol<T, DIM>(nb, uu, vv) : (double)nf_poisson_area<T, DIM>(nb, uu, vv);
}

__global__ void finalize_kernel(const double* sum, const double* sum_sq, const uint64_t* nw, int64_t n, double* mean,
                                double* se) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double N = (double)nw[i];
  const double m = sum[i] / N;
  const double var = N > 1 ? fmax(sum_sq[i] / N - m * m, 0.0) * N / (N - 1) : __builtin_nan("");
  mean[i] = m;
  se[i] = sqrt(var / N);
}

// ====================================================================== static scratch
//
// Scratch memory of wos_solve_static, for callers that cannot allocate: a file-scope device
// array, of which every GPU the library runs on holds its own copy until the process
// ends. Host code never uses the array's name as an address: the device address of the
// current GPU's copy is looked up once per device (hipGetSymbolAddress) and kept.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mutex;
std::map<int, void*> g_scratch_ptr;
}  // namespace

hipError_t static_scratch(int device, void** ptr) {
  std::lock_guard<std::mutex> lk(g_scratch_mutex);
  auto it = g_scratch_ptr.find(device);
  if (it == g_scratch_ptr.end()) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    it = g_scratch_ptr.emplace(device, p).first;
  }
  *ptr = it->second;
  return hipSuccess;
}

// ====================================================================== launchers

static inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_walker(const WalkerLaunch& L, hipStream_t st) {
  if (L.fp64) return L.dim == 2 ? launch_walker_f64_2d(L, st) : launch_walker_f64_3d(L, st);
  return L.dim == 2 ? launch_walker_f32_2d(L, st) : launch_walker_f32_3d(L, st);
}

int walker_mode(int variant, bool grad, bool split) { return variant == 2 ? 2 : (grad || split) ? 1 : 0; }

const void* walker_symbol(int fp64, int dim, int geom, int mode) {
  if (fp64) return dim == 2 ? walker_symbol_f64_2d(geom, mode) : walker_symbol_f64_3d(geom, mode);
  return dim == 2 ? walker_symbol_f32_2d(geom, mode) : walker_symbol_f32_3d(geom, mode);
}

hipError_t launch_reduce(int grad_dim, const DevItem& it, const uint64_t* slots, int slot_words, hipStream_t st) {
  if (it.n_points == 0) return hipSuccess;
  const dim3 g(blocks_for(it.n_points, 256)), b(256);
  if (grad_dim == 2) hipLaunchKernelGGL(reduce_kernel<2>, g, b, 0, st, it, slots, slot_words);
  else if (grad_dim == 3) hipLaunchKernelGGL(reduce_kernel<3>, g, b, 0, st, it, slots, slot_words);
  else hipLaunchKernelGGL(reduce_kernel<0>, g, b, 0, st, it, slots, slot_words);
  return hipGetLastError();
}

hipError_t launch_clear(uint64_t* p, uint64_t n, uint32_t* counter, hipStream_t st) {
  const unsigned blocks = (unsigned)std::min<uint64_t>(std::max<uint64_t>((n + 255) / 256, 1), 4096);
  hipLaunchKernelGGL(clear_kernel, dim3(blocks), dim3(256), 0, st, p, n, counter);
  return hipGetLastError();
}

hipError_t launch_set_params(LaunchParams* lp, uint64_t seed, uint64_t walk_offset_add, hipStream_t st) {
  hipLaunchKernelGGL(set_params_kernel, dim3(1), dim3(64), 0, st, lp, seed, walk_offset_add);
  return hipGetLastError();
}

hipError_t launch_reset(uint32_t* counter, hipStream_t st) {
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, st, counter);
  return hipGetLastError();
}

template <int DIM, int GEOM>
static hipError_t classify_t(const void* P, const double* pts, int64_t n, int8_t* inside, uint64_t* counters,
                             hipStream_t st) {
  hipLaunchKernelGGL((classify_kernel<DIM, GEOM>), dim3(blocks_for(n, 256)), dim3(256), 0, st,
                     (const DevProblem<double>*)P, pts, n, inside, counters);
  return hipGetLastError();
}

hipError_t launch_classify(int dim, int geom, const void* P64, const double* pts, int64_t n, int8_t* inside,
                           uint64_t* counters, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (dim == 2) {
    switch (geom) {
      case GK_BALL: return classify_t<2, GK_BALL>(P64, pts, n, inside, counters, st);
      case GK_BOX: return classify_t<2, GK_BOX>(P64, pts, n, inside, counters, st);
      case GK_POLYGON: return classify_t<2, GK_POLYGON>(P64, pts, n, inside, counters, st);
      case GK_SDF: return classify_t<2, GK_SDF>(P64, pts, n, inside, counters, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (geom) {
    case GK_BALL: return classify_t<3, GK_BALL>(P64, pts, n, inside, counters, st);
    case GK_BOX: return classify_t<3, GK_BOX>(P64, pts, n, inside, counters, st);
    case GK_TRIMESH: return classify_t<3, GK_TRIMESH>(P64, pts, n, inside, counters, st);
    case GK_SDF: return classify_t<3, GK_SDF>(P64, pts, n, inside, counters, st);
    default: return hipErrorInvalidValue;
  }
}

template <int DIM, int GEOM>
static hipError_t sigma_t(const void* P, const double* lo, const double* h, int grid, int nblocks, double* out,
                          hipStream_t st) {
  hipLaunchKernelGGL((sigma_sample_kernel<DIM, GEOM>), dim3(nblocks), dim3(256), 0, st, (const DevProblem<double>*)P,
                     lo[0], lo[1], lo[2], h[0], h[1], h[2], grid, out);
  return hipGetLastError();
}

hipError_t launch_sigma_sample(int dim, int geom, const void* P64, const double* lo, const double* h, int grid,
                               int nblocks, double* out, hipStream_t st) {
  if (dim == 2) {
    switch (geom) {
      case GK_BALL: return sigma_t<2, GK_BALL>(P64, lo, h, grid, nblocks, out, st);
      case GK_BOX: return sigma_t<2, GK_BOX>(P64, lo, h, grid, nblocks, out, st);
      case GK_POLYGON: return sigma_t<2, GK_POLYGON>(P64, lo, h, grid, nblocks, out, st);
      case GK_SDF: return sigma_t<2, GK_SDF>(P64, lo, h, grid, nblocks, out, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (geom) {
    case GK_BALL: return sigma_t<3, GK_BALL>(P64, lo, h, grid, nblocks, out, st);
    case GK_BOX: return sigma_t<3, GK_BOX>(P64, lo, h, grid, nblocks, out, st);
    case GK_TRIMESH: return sigma_t<3, GK_TRIMESH>(P64, lo, h, grid, nblocks, out, st);
    case GK_SDF: return sigma_t<3, GK_SDF>(P64, lo, h, grid, nblocks, out, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gamma0(int fp64, int dim, const void* P, const double* pts, int64_t n, const int8_t* inside,
                         void* out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const dim3 g(blocks_for(n, 256)), b(256);
  if (fp64) {
    if (dim == 2)
      hipLaunchKernelGGL((gamma0_kernel<double, 2>), g, b, 0, st, (const DevProblem<double>*)P, pts, n, inside, (double*)out);
    else
      hipLaunchKernelGGL((gamma0_kernel<double, 3>), g, b, 0, st, (const DevProblem<double>*)P, pts, n, inside, (double*)out);
  } else {
    if (dim == 2)
      hipLaunchKernelGGL((gamma0_kernel<float, 2>), g, b, 0, st, (const DevProblem<float>*)P, pts, n, inside, (float*)out);
    else
      hipLaunchKernelGGL((gamma0_kernel<float, 3>), g, b, 0, st, (const DevProblem<float>*)P, pts, n, inside, (float*)out);
  }
  return hipGetLastError();
}

hipError_t launch_coefficients(int fp64, int dim, const void* P, const double* pts, int64_t n, double* out,
                               hipStream_t st) {
  if (n == 0) return hipSuccess;
  const dim3 g(blocks_for(n, 256)), b(256);
  if (fp64) {
    if (dim == 2) hipLaunchKernelGGL((coef_kernel<double, 2>), g, b, 0, st, (const DevProblem<double>*)P, pts, n, out);
    else hipLaunchKernelGGL((coef_kernel<double, 3>), g, b, 0, st, (const DevProblem<double>*)P, pts, n, out);
  } else {
    if (dim == 2) hipLaunchKernelGGL((coef_kernel<float, 2>), g, b, 0, st, (const DevProblem<float>*)P, pts, n, out);
    else hipLaunchKernelGGL((coef_kernel<float, 3>), g, b, 0, st, (const DevProblem<float>*)P, pts, n, out);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t distance_t(int dim, int geom, const void* P, const double* pts, int64_t n, double* d, double* xb,
                             hipStream_t st) {
  const dim3 g(blocks_for(n, 256)), b(256);
  const DevProblem<T>* p = (const DevProblem<T>*)P;
  if (dim == 2) {
    if (geom == GK_BALL) hipLaunchKernelGGL((distance_kernel<T, 2, GK_BALL>), g, b, 0, st, p, pts, n, d, xb);
    else if (geom == GK_BOX) hipLaunchKernelGGL((distance_kernel<T, 2, GK_BOX>), g, b, 0, st, p, pts, n, d, xb);
    else if (geom == GK_SDF) hipLaunchKernelGGL((distance_kernel<T, 2, GK_SDF>), g, b, 0, st, p, pts, n, d, xb);
    else hipLaunchKernelGGL((distance_kernel<T, 2, GK_POLYGON>), g, b, 0, st, p, pts, n, d, xb);
  } else {
    if (geom == GK_BALL) hipLaunchKernelGGL((distance_kernel<T, 3, GK_BALL>), g, b, 0, st, p, pts, n, d, xb);
    else if (geom == GK_BOX) hipLaunchKernelGGL((distance_kernel<T, 3, GK_BOX>), g, b, 0, st, p, pts, n, d, xb);
    else if (geom == GK_SDF) hipLaunchKernelGGL((distance_kernel<T, 3, GK_SDF>), g, b, 0, st, p, pts, n, d, xb);
    else hipLaunchKernelGGL((distance_kernel<T, 3, GK_TRIMESH>), g, b, 0, st, p, pts, n, d, xb);
  }
  return hipGetLastError();
}

hipError_t launch_distance(int fp64, int dim, int geom, const void* P, const double* pts, int64_t n, double* d,
                           double* xb, hipStream_t st) {
  if (n == 0) return hipSuccess;
  return fp64 ? distance_t<double>(dim, geom, P, pts, n, d, xb, st) : distance_t<float>(dim, geom, P, pts, n, d, xb, st);
}

hipError_t launch_ball(int fp64, int dim, const double* s, int64_t n, double* out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const dim3 g(blocks_for(n, 256)), b(256);
  if (fp64) {
    if (dim == 2) hipLaunchKernelGGL((ball_kernel<double, 2>), g, b, 0, st, s, n, out);
    else hipLaunchKernelGGL((ball_kernel<double, 3>), g, b, 0, st, s, n, out);
  } else {
    if (dim == 2) hipLaunchKernelGGL((ball_kernel<float, 2>), g, b, 0, st, s, n, out);
    else hipLaunchKernelGGL((ball_kernel<float, 3>), g, b, 0, st, s, n, out);
  }
  return hipGetLastError();
}

hipError_t launch_sample(int fp64, int dim, double s, int64_t n, uint64_t seed, double* t, uint64_t* trials,
                         hipStream_t st) {
  if (n == 0) return hipSuccess;
  const dim3 g(blocks_for(n, 256)), b(256);
  if (fp64) {
    if (dim == 2) hipLaunchKernelGGL((sample_kernel<double, 2>), g, b, 0, st, s, n, seed, t, trials);
    else hipLaunchKernelGGL((sample_kernel<double, 3>), g, b, 0, st, s, n, seed, t, trials);
  } else {
    if (dim == 2) hipLaunchKernelGGL((sample_kernel<float, 2>), g, b, 0, st, s, n, seed, t, trials);
    else hipLaunchKernelGGL((sample_kernel<float, 3>), g, b, 0, st, s, n, seed, t, trials);
  }
  return hipGetLastError();
}

hipError_t launch_philox(const uint32_t* ctr, uint64_t key, int64_t n, uint32_t* out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(philox_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, ctr, key, n, out);
  return hipGetLastError();
}

hipError_t launch_offcentred(int fp64, int dim, int which, double R, double sigma_bar, const double* u,
                             const double* v, int64_t n, double* out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const dim3 g(blocks_for(n, 256)), b(256);
  if (fp64) {
    if (dim == 2) hipLaunchKernelGGL((offcentred_kernel<double, 2>), g, b, 0, st, which, R, sigma_bar, u, v, n, out);
    else hipLaunchKernelGGL((offcentred_kernel<double, 3>), g, b, 0, st, which, R, sigma_bar, u, v, n, out);
  } else {
    if (dim == 2)
      hipLaunchKernelGGL((offcentred_kernel<float, 2>), g, b, 0, st, which, (float)R, (float)sigma_bar, u, v, n, out);
    else
      hipLaunchKernelGGL((offcentred_kernel<float, 3>), g, b, 0, st, which, (float)R, (float)sigma_bar, u, v, n, out);
  }
  return hipGetLastError();
}

hipError_t launch_bessel(int fp64, int which, const double* x, int64_t n, double* out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const dim3 g(blocks_for(n, 256)), b(256);
  if (fp64) hipLaunchKernelGGL((bessel_kernel<double>), g, b, 0, st, which, x, n, out);
  else hipLaunchKernelGGL((bessel_kernel<float>), g, b, 0, st, which, x, n, out);
  return hipGetLastError();
}

// Per component of [n][dim] sums, with the walk count of its point.
__global__ void finalize_components_kernel(const double* sum, const double* sum_sq, const uint64_t* nw, int64_t n,
                                           int dim, double* mean, double* se) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * dim) return;
  const double N = (double)nw[i / dim];
  const double m = sum[i] / N;
  const double var = N > 1 ? fmax(sum_sq[i] / N - m * m, 0.0) * N / (N - 1) : __builtin_nan("");
  mean[i] = m;
  se[i] = sqrt(var / N);
}

hipError_t launch_finalize_components(const double* sum, const double* sum_sq, const uint64_t* nw, int64_t n, int dim,
                                      double* mean, double* se, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_components_kernel, dim3(blocks_for(n * dim, 256)), dim3(256), 0, st, sum, sum_sq, nw,
                     n, dim, mean, se);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* sum, const double* sum_sq, const uint64_t* nw, int64_t n, double* mean,
                           double* se, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, sum, sum_sq, nw, n, mean, se);
  return hipGetLastError();
}

}  // namespace wos
