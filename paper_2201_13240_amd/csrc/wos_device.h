// Device functions of the delta-tracking walk on spheres (gfx950).
//
// Everything here is templated on the arithmetic type T (float or double) so the FP32
// and FP64 walkers are one source. Citations refer to Sawhney, Seyb, Jarosz, Crane,
// "Grid-Free Monte Carlo for PDEs with Spatially Varying Coefficients" (2022) and its
// supplemental material.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bessel_tables.h"
#include "proposal_bound.h"
#include "wos_types.h"

namespace wos {

// Problem tables, BVHs, query points and work tables never change while a kernel runs,
// so they are read through constant-address-space references: the compiler then serves
// wave-uniform reads with scalar loads and lane-varying ones with global loads (a
// generic pointer would force flat loads for both).
#define WOS_GLOBAL __attribute__((address_space(4)))
template <typename T>
using G = const WOS_GLOBAL T;
template <typename T>
__device__ __forceinline__ const WOS_GLOBAL T* gptr(const T* p) {
  return (const WOS_GLOBAL T*)p;
}

// ------------------------------------------------------------------ math wrappers

__device__ __forceinline__ float m_exp(float x) { return __expf(x); }
__device__ __forceinline__ double m_exp(double x) { return ::exp(x); }
__device__ __forceinline__ float m_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double m_exp2(double x) { return ::exp2(x); }
__device__ __forceinline__ float m_expm1(float x) { return ::expm1f(x); }
__device__ __forceinline__ double m_expm1(double x) { return ::expm1(x); }
__device__ __forceinline__ float m_log(float x) { return __logf(x); }
__device__ __forceinline__ double m_log(double x) { return ::log(x); }
// ln x of a positive normal x (uniforms, their products, clamped arguments): the hardware
// base-2 logarithm times ln 2, without the subnormal scaling and the two-part product with
// ln 2 of the library logarithm (about 1 ulp more error, 2 instructions instead of 13)
__device__ __forceinline__ float m_logn(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
__device__ __forceinline__ double m_logn(double x) { return ::log(x); }
// hardware square root (within 1 ulp; no rescaling of inputs below 2^-96)
__device__ __forceinline__ float m_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double m_sqrt(double x) { return ::sqrt(x); }
__device__ __forceinline__ float m_tanh(float x) { return ::tanhf(x); }
__device__ __forceinline__ double m_tanh(double x) { return ::tanh(x); }
__device__ __forceinline__ float m_cbrt(float x) { return ::cbrtf(x); }
__device__ __forceinline__ double m_cbrt(double x) { return ::cbrt(x); }
// Reciprocal and quotient: FP32 takes the hardware reciprocal (1 ulp) instead of the
// correctly rounded division sequence; FP64 divides exactly.
__device__ __forceinline__ float m_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double m_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float m_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double m_div(double a, double b) { return a / b; }
__device__ __forceinline__ float m_fabs(float x) { return ::fabsf(x); }
__device__ __forceinline__ double m_fabs(double x) { return ::fabs(x); }
__device__ __forceinline__ float m_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double m_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
// sin and cos of 2*pi*r (r in revolutions). FP32: the hardware sine and cosine take
// revolutions directly; r is first reduced to [0, 1) by the hardware fraction (exact,
// r - floor(r)), inside their input range. m_sincospi2_unit takes an r already in (0, 1)
// (a uniform) as it is.
__device__ __forceinline__ void m_sincospi2(float r, float* s, float* c) {
  const float f = __builtin_amdgcn_fractf(r);
  *s = __builtin_amdgcn_sinf(f);
  *c = __builtin_amdgcn_cosf(f);
}
__device__ __forceinline__ void m_sincospi2_unit(float r, float* s, float* c) {
  *s = __builtin_amdgcn_sinf(r);
  *c = __builtin_amdgcn_cosf(r);
}
__device__ __forceinline__ void m_sincospi2(double r, double* s, double* c) { ::sincospi(2.0 * r, s, c); }
__device__ __forceinline__ void m_sincospi2_unit(double r, double* s, double* c) { ::sincospi(2.0 * r, s, c); }
// cos(2 pi r), r in revolutions
__device__ __forceinline__ float m_cospi2(float r) { return __builtin_amdgcn_cosf(__builtin_amdgcn_fractf(r)); }
__device__ __forceinline__ double m_cospi2(double r) { return ::cospi(2.0 * r); }
__device__ __forceinline__ void m_sincos(float x, float* s, float* c) { ::sincosf(x, s, c); }
__device__ __forceinline__ void m_sincos(double x, double* s, double* c) { ::sincos(x, s, c); }

template <typename T> struct Consts;
template <> struct Consts<float> {
  static constexpr float kInf = __builtin_huge_valf();
  static constexpr float kEulerGamma = 0.5772156649015329f;
  static constexpr float kTiny = 1e-30f;
};
template <> struct Consts<double> {
  static constexpr double kInf = __builtin_huge_val();
  static constexpr double kEulerGamma = 0.57721566490153286061;
  static constexpr double kTiny = 1e-300;
};

// Work counters of one lane, kept only by the event-counting build of the walker.
struct Tally {
  uint32_t nodes;        // BVH inner nodes visited
  uint32_t prims;        // primitives whose distance was computed
  uint32_t trials_free;  // radius proposals drawn from the free-space law
  uint32_t cells;        // candidate-grid lookups
};

// ------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11).

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
    }
    // 32 x 32 -> 64-bit products: one v_mad_u64_u32 each instead of a mul_lo / mul_hi pair
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k.x, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k.y, (uint32_t)p0);
  }
  return c;
}

// Per-walk counter-based stream: key = seed, counter = (block, walk, point, problem).
// The walker draws the words of one iteration in lockstep across the wave at the top of
// the iteration (refill<NB>: NB Philox blocks, 4 words each), so the cipher never runs
// inside the divergent branches that consume them. Every consumer reads its own fixed
// word slot (a compile-time index), so no lane-varying word position has to be tracked.
// Words a lane does not consume in an iteration are skipped, which keeps the stream of a
// walk a fixed function of (seed, walk, point, problem) whatever the schedule.
constexpr int kMaxRngBlocks = 5;

struct Rng {
  uint2 key;        // the seed: one key for every stream of a launch, set once by set_key so
                    // that it stays wave-uniform (the round keys then come from scalar adds)
  uint32_t walk, point, problem;
  uint32_t block;   // next block index
  uint32_t w[4 * kMaxRngBlocks];

  __device__ __forceinline__ void set_key(uint64_t seed) { key = make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)); }
  __device__ __forceinline__ void init(uint32_t wk, uint32_t p, uint32_t prob) {
    walk = wk;
    point = p;
    problem = prob;
    block = 0;
  }
  template <int NB>
  __device__ __forceinline__ void refill() {
    static_assert(NB >= 1 && NB <= kMaxRngBlocks, "block count");
    // the round keys are formed here by scalar adds: an empty asm statement keeps the
    // compiler from hoisting all twenty of them out of the walker's loop into scalar
    // registers, which it would then spill
    uint32_t kx = key.x, ky = key.y;
    asm volatile("" : "+s"(kx), "+s"(ky));
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const uint4 q = philox4x32_10(make_uint4(block + j, walk, point, problem), make_uint2(kx, ky));
      w[4 * j] = q.x;
      w[4 * j + 1] = q.y;
      w[4 * j + 2] = q.z;
      w[4 * j + 3] = q.w;
    }
    block += NB;
  }
};

// Uniform from slot S of the current draw. FP32: (k + 1/2) 2^-21 for the 21-bit field k
// of the slot, in (0, 1) (never 0 or 1, so a logarithm is finite and nonzero: a
// free-space radius proposal 2 sqrt(ln u1 ln u2) is never 0), six uniforms per Philox
// block: slot 6b + j is bits 21j .. 21j + 20 of the 128-bit block b (words 4b .. 4b + 3,
// least significant first), so one block serves a 2D delta-tracking step. FP64: 53 bits
// of words 2S and 2S + 1, plus 2^-53, in (0, 1].
constexpr int kFp32UniformBits = 21;

template <int S>
__device__ __forceinline__ uint32_t uniform_bits_fp32(const Rng& r) {
  constexpr int b = S / 6, o = 21 * (S % 6), i = 4 * b + o / 32, sh = o % 32;
  constexpr uint32_t mask = (1u << kFp32UniformBits) - 1u;
  if constexpr (sh + kFp32UniformBits <= 32) {
    return (r.w[i] >> sh) & mask;
  } else {
    return __builtin_amdgcn_alignbit(r.w[i + 1], r.w[i], sh) & mask;
  }
}

template <typename T, int S>
__device__ __forceinline__ T uniform01(const Rng& r) {
  if constexpr (sizeof(T) == 4) {
    // (2k + 1) 2^-22 = 1.m - 1 with the 23-bit mantissa m = 4k + 2 (exact)
    return __uint_as_float((uniform_bits_fp32<S>(r) << 2) | 0x3F800002u) - 1.0f;
  } else {
    const uint64_t a = r.w[2 * S], b = r.w[2 * S + 1];
    return (double)((((a << 32) | b) >> 11) + 1ull) * 1.1102230246251565404e-16;  // 2^-53
  }
}

// Uniform slots of one iteration of the walker. Delta tracking: ball direction, radius
// proposal (3 uniforms in 2D, 4 in 3D), volume/exit choice, exit direction, roulette.
// Next flight: roulette on the throughput, exit direction of a new ball, inner point
// (direction and radius). Blocks: Philox blocks per iteration with the roulette slot
// (kBlocks) and without it (kBlocksPlain: no weight window; FP32 2D: one block).
template <typename T, int DIM>
struct Slots {
  static constexpr int kDir = 0;
  static constexpr int kTrial = kDir + DIM - 1;
  static constexpr int kMu = kTrial + (DIM == 2 ? 3 : 4);
  static constexpr int kExitDir = kMu + 1;
  static constexpr int kRoulette = kExitDir + DIM - 1;
  static constexpr int kCount = kRoulette + 1;
  static constexpr int kNfRoulette = 0;
  static constexpr int kNfExitDir = 1;
  static constexpr int kNfInner = kNfExitDir + DIM - 1;
  static constexpr int kNfCount = kNfInner + DIM;
  static constexpr int blocks(int slots) { return sizeof(T) == 4 ? (slots + 5) / 6 : (2 * slots + 3) / 4; }
  static constexpr int kBlocks = blocks(kCount);
  static constexpr int kBlocksPlain = blocks(kCount - 1);
  static constexpr int kNfBlocks = blocks(kNfCount);
  static_assert(kBlocks <= kMaxRngBlocks && kNfBlocks <= kMaxRngBlocks, "slot layout exceeds the buffer");
};

// Draws of one delta-tracking iteration for the FP64 walker taking the FP32 walker's
// uniforms (common random numbers): the FP32 slot layout's Philox blocks are drawn (with
// or without the roulette slot, as the FP32 walker does), and the uniform of FP32 slot
// S, (2k + 1) 2^-22, is re-encoded into words 2S and 2S + 1 so that the FP64
// construction (53 bits, plus 2^-53) returns exactly that value. Slots are rewritten from
// the last down: FP32 slot S reads only words below 2S + 2, and slot S' < S writes words
// 2S' and 2S' + 1, above every word a lower slot reads, so no word is overwritten before
// it is read.
template <int S>
__device__ __forceinline__ void reencode_fp32_slots(Rng& r) {
  if constexpr (S >= 0) {
    // (2k + 1) 2^(53 - 22) - 1 < 2^53
    const uint64_t x = ((((uint64_t)uniform_bits_fp32<S>(r) << 1) | 1ull) << (52 - kFp32UniformBits)) - 1ull;
    const uint64_t y = x << 11;
    r.w[2 * S] = (uint32_t)(y >> 32);
    r.w[2 * S + 1] = (uint32_t)y;
    reencode_fp32_slots<S - 1>(r);
  }
}

template <int DIM, int NB>
__device__ __forceinline__ void refill_fp32_draws(Rng& r) {
  using S32 = Slots<float, DIM>;
  r.refill<NB>();
  reencode_fp32_slots<(NB == S32::kBlocks ? S32::kCount : S32::kCount - 1) - 1>(r);
}

// ------------------------------------------------------------------ modified Bessel functions

template <typename T>
__device__ __forceinline__ T chebyshev(const double* c, int n, T t) {
  // Clenshaw recurrence for sum_j c_j T_j(t)
  T b1 = 0, b2 = 0;
  const T t2 = t + t;
  for (int j = n - 1; j >= 1; --j) {
    const T b0 = m_fma(t2, b1, (T)c[j] - b2);
    b2 = b1;
    b1 = b0;
  }
  return m_fma(t, b1, (T)c[0] - b2);
}

// Horner's rule for sum_j p_j t^j, one FMA per term
template <typename T>
__device__ __forceinline__ T horner(const double* p, int n, T t) {
  T acc = (T)p[n - 1];
  for (int j = n - 2; j >= 0; --j) acc = m_fma(acc, t, (T)p[j]);
  return acc;
}

// A polynomial given both as a Chebyshev series and as a power series: FP32 takes Horner's
// rule (half the instructions), FP64 the Chebyshev recurrence (with Horner's rule the FP64
// 2D walker no longer fits 256 VGPRs without spills)
template <typename T>
__device__ __forceinline__ T envelope_series(const double* cheb, const double* pw, int n, T u) {
  if constexpr (sizeof(T) == 4) return horner<T>(pw, n, u);
  else return chebyshev<T>(cheb, n, u);
}

template <typename T> struct BesselTerms;
template <> struct BesselTerms<float> {
  static constexpr int kI0Wide = WOS_I0E_WIDE_TAIL_NH32, kK0Wide = WOS_K0E_WIDE_TAIL_NH32;
  static constexpr int kSeries = 7, kI0Mid = WOS_I0E_MID_N32, kI0Tail = WOS_I0E_TAIL_N32,
                       kK0Low = WOS_K0E_LOW_N32, kK0Mid = WOS_K0E_MID_N32, kK0Tail = WOS_K0E_TAIL_N32,
                       kI1Mid = WOS_I1E_MID_N32, kI1Tail = WOS_I1E_TAIL_N32, kK1Low = WOS_K1E_LOW_N32,
                       kK1Mid = WOS_K1E_MID_N32, kK1Tail = WOS_K1E_TAIL_N32;
};
template <> struct BesselTerms<double> {
  static constexpr int kSeries = 15, kI0Mid = WOS_I0E_MID_N64, kI0Tail = WOS_I0E_TAIL_N64,
                       kK0Low = WOS_K0E_LOW_N64, kK0Mid = WOS_K0E_MID_N64, kK0Tail = WOS_K0E_TAIL_N64,
                       kI1Mid = WOS_I1E_MID_N64, kI1Tail = WOS_I1E_TAIL_N64, kK1Low = WOS_K1E_LOW_N64,
                       kK1Mid = WOS_K1E_MID_N64, kK1Tail = WOS_K1E_TAIL_N64;
};

// Coefficients of the power series below: 1/(k!)^2, H_k = 1 + 1/2 + ... + 1/k and their
// product
struct BesselSeriesCoef {
  double a[16], h[16], b[16];
};
constexpr BesselSeriesCoef make_bessel_series_coef() {
  BesselSeriesCoef c{};
  double f = 1, h = 0;
  for (int k = 1; k < 16; ++k) {
    f /= (double)k * (double)k;
    h += 1.0 / k;
    c.a[k] = f;
    c.h[k] = h;
    c.b[k] = f * h;
  }
  return c;
}
static constexpr BesselSeriesCoef kBesselSeries = make_bessel_series_coef();

// Power series of I0 and K0 for x <= 2 (for K0 near x = 2 the two parts cancel to about a
// tenth, which costs FP32 a few units in the last place); FP32 takes both as polynomials
// in q by Horner's rule, FP64 sums the terms upward. FP32 stops at k = 7 (the terms
// dropped sum to less than 2e-9 at q = 1, 2e-8 of K0(2)), FP64 at k = 15:
//   I0(x) - 1 = sum_{k>=1} q^k/(k!)^2,  q = x^2/4
//   K0(x) = -(ln(x/2) + gamma_E) I0(x) + sum_{k>=1} q^k/(k!)^2 H_k
template <typename T>
__device__ __forceinline__ void bessel_series(T x, T* i0m1, T* k0) {
  constexpr int n = BesselTerms<T>::kSeries;
  const T q = (T)0.25 * x * x;
  T s_i, s_k;
  if constexpr (sizeof(T) == 4) {
    s_i = (T)kBesselSeries.a[n];
    s_k = (T)kBesselSeries.b[n];
    for (int k = n - 1; k >= 1; --k) {
      s_i = m_fma(s_i, q, (T)kBesselSeries.a[k]);
      s_k = m_fma(s_k, q, (T)kBesselSeries.b[k]);
    }
    s_i *= q;
    s_k *= q;
  } else {
    T term = 1;
    s_i = 0;
    s_k = 0;
    for (int k = 1; k <= n; ++k) {
      term *= q * (T)(1.0 / (k * k));
      s_i += term;
      s_k = m_fma(term, (T)kBesselSeries.h[k], s_k);
    }
  }
  *i0m1 = s_i;
  if (k0) {
    // x/2 clamped to the smallest normal number, where the logarithm is the hardware's
    const T hx = sizeof(T) == 4 ? fmax((T)0.5 * x, (T)1.17549435e-38f) : (T)0.5 * x;
    *k0 = -(m_logn(hx) + Consts<T>::kEulerGamma) * ((T)1 + s_i) + s_k;
  }
}

// e^-x I0(x), x >= 0
template <typename T>
__device__ T bessel_i0e(T x) {
  if (x <= (T)2) {
    T i0m1;
    bessel_series<T>(x, &i0m1, nullptr);
    return ((T)1 + i0m1) * m_exp(-x);
  }
  if (x <= (T)8) return chebyshev<T>(WOS_I0E_MID, BesselTerms<T>::kI0Mid, (x - (T)5) * (T)(1.0 / 3.0));
  return m_div(chebyshev<T>(WOS_I0E_TAIL, BesselTerms<T>::kI0Tail, (T)16 * m_rcp(x) - (T)1), m_sqrt(x));
}

// e^x K0(x), x > 0
template <typename T>
__device__ T bessel_k0e(T x) {
  if (x <= (T)1) {
    T i0m1, k0;
    bessel_series<T>(x, &i0m1, &k0);
    return k0 * m_exp(x);
  }
  if (x <= (T)3) return chebyshev<T>(WOS_K0E_LOW, BesselTerms<T>::kK0Low, x - (T)2);
  if (x <= (T)8) return chebyshev<T>(WOS_K0E_MID, BesselTerms<T>::kK0Mid, ((T)2 * x - (T)11) * (T)0.2);
  return m_div(chebyshev<T>(WOS_K0E_TAIL, BesselTerms<T>::kK0Tail, (T)16 * m_rcp(x) - (T)1), m_sqrt(x));
}

// I0 and K0 at x > 0 for the 2D ball terms and radius proposals, in one function so that
// lanes of a wavefront whose arguments fall in different ranges still share its two code
// paths: below 2 the series gives *a = I0 - 1 and *k = K0 (returns false); from 2 on the
// Chebyshev fits give *a = e^-x I0 and *k = e^x K0 (returns true). In FP32 each function
// has a single fit from 2 on (in t = 4/x - 1, of sqrt(x) e^-x I0 and sqrt(x) e^x K0), so
// every lane with x >= 2 runs the same two polynomials, as power series in t by Horner's
// rule; FP64 keeps the narrower ranges, whose fits reach double precision with fewer terms.
template <typename T>
__device__ __forceinline__ bool bessel_i0k0(T x, T* a, T* k) {
  if (x < (T)2) {
    bessel_series<T>(x, a, k);
    return false;
  }
  if constexpr (sizeof(T) == 4) {
    const T rs = __builtin_amdgcn_rsqf(x);
    const T t = m_fma((T)4, rs * rs, (T)-1);   // 4/x - 1
    *a = horner<T>(WOS_I0E_WIDE_TAIL_POW32, BesselTerms<T>::kI0Wide, t) * rs;
    *k = horner<T>(WOS_K0E_WIDE_TAIL_POW32, BesselTerms<T>::kK0Wide, t) * rs;
    return true;
  }
  if (x <= (T)8) {
    *a = chebyshev<T>(WOS_I0E_MID, BesselTerms<T>::kI0Mid, (x - (T)5) * (T)(1.0 / 3.0));
  } else {
    *a = m_div(chebyshev<T>(WOS_I0E_TAIL, BesselTerms<T>::kI0Tail, (T)16 * m_rcp(x) - (T)1), m_sqrt(x));
  }
  if (x <= (T)3) {
    *k = chebyshev<T>(WOS_K0E_LOW, BesselTerms<T>::kK0Low, x - (T)2);
  } else if (x <= (T)8) {
    *k = chebyshev<T>(WOS_K0E_MID, BesselTerms<T>::kK0Mid, ((T)2 * x - (T)11) * (T)0.2);
  } else {
    *k = m_div(chebyshev<T>(WOS_K0E_TAIL, BesselTerms<T>::kK0Tail, (T)16 * m_rcp(x) - (T)1), m_sqrt(x));
  }
  return true;
}

// Power series of I1 and K1 for small x (x <= 2 for I1, x <= 1 for K1), q = x^2/4:
//   I1(x) = (x/2) sum_{k>=0} q^k/(k!(k+1)!)
//   K1(x) = 1/x + ln(x/2) I1(x) - (x/4) sum_{k>=0} (psi(k+1) + psi(k+2)) q^k/(k!(k+1)!)
// with psi(k+1) + psi(k+2) = H_k + H_{k+1} - 2 gamma_E.
template <typename T>
__device__ __forceinline__ void bessel_series1(T x, T* i1, T* k1) {
  const T q = (T)0.25 * x * x;
  T term = 1, s_i = 1, h = 0, s_k = -(T)2 * Consts<T>::kEulerGamma + (T)1;   // k = 0: H_0 + H_1 = 1
  for (int k = 1; k <= BesselTerms<T>::kSeries; ++k) {
    term *= q * (T)(1.0 / (k * (k + 1)));
    const T hk = h + (T)1 / (T)k;                 // H_k
    const T hk1 = hk + (T)1 / (T)(k + 1);         // H_{k+1}
    h = hk;
    s_i += term;
    s_k = m_fma(term, hk + hk1 - (T)2 * Consts<T>::kEulerGamma, s_k);
  }
  const T hx = (T)0.5 * x;
  *i1 = hx * s_i;
  if (k1) *k1 = m_rcp(x) + m_log(hx) * (*i1) - (T)0.5 * hx * s_k;
}

// e^-x I1(x), x >= 0
template <typename T>
__device__ T bessel_i1e(T x) {
  if (x <= (T)2) {
    T i1;
    bessel_series1<T>(x, &i1, nullptr);
    return i1 * m_exp(-x);
  }
  if (x <= (T)8) return chebyshev<T>(WOS_I1E_MID, BesselTerms<T>::kI1Mid, (x - (T)5) * (T)(1.0 / 3.0));
  return m_div(chebyshev<T>(WOS_I1E_TAIL, BesselTerms<T>::kI1Tail, (T)16 * m_rcp(x) - (T)1), m_sqrt(x));
}

// e^x K1(x), x > 0
template <typename T>
__device__ T bessel_k1e(T x) {
  if (x <= (T)1) {
    T i1, k1;
    bessel_series1<T>(x, &i1, &k1);
    return k1 * m_exp(x);
  }
  if (x <= (T)3) return chebyshev<T>(WOS_K1E_LOW, BesselTerms<T>::kK1Low, x - (T)2);
  if (x <= (T)8) return chebyshev<T>(WOS_K1E_MID, BesselTerms<T>::kK1Mid, ((T)2 * x - (T)11) * (T)0.2);
  return m_div(chebyshev<T>(WOS_K1E_TAIL, BesselTerms<T>::kK1Tail, (T)16 * m_rcp(x) - (T)1), m_sqrt(x));
}

// ------------------------------------------------------------------ ball kernels
// 1/(2k+3)!, k = 0..8: the power series of (sinh s - s)/s^3 in s^2
struct SinhSeriesCoef {
  double c[9];
};
constexpr SinhSeriesCoef make_sinh_series_coef() {
  SinhSeriesCoef r{};
  double f = 6;
  for (int k = 0; k < 9; ++k) {
    r.c[k] = 1.0 / f;
    f *= (double)(2 * k + 4) * (double)(2 * k + 5);
  }
  return r;
}
static constexpr SinhSeriesCoef kSinhSeries = make_sinh_series_coef();

// Centred Green's function of Laplace - sigma_bar on the ball of radius R (supp. Sec. 1.1):
//   |G| = P_B / sigma_bar with P_B = 1 - 1/I0(s) (2D), 1 - s/sinh(s) (3D), s = R sqrt(sigma_bar),
// and the Poisson kernel (1 - P_B)/|dB|, so P_B is the probability of the volume term
// (Sec. 5.1). Small s uses the series of I0 - 1 and sinh(s) - s to avoid cancellation.
template <typename T, int DIM>
struct Ball {
  T pb;        // P_B = sigma_bar |G|
  T gnorm;     // |G|
  T c2d;       // 2D: K0(s)/I0(s) (s < 2) or e^{2s} K0(s)/I0(s) = K0e/I0e (s >= 2)
};

template <typename T, int DIM>
__device__ __forceinline__ Ball<T, DIM> ball_terms(T R, T s, T inv_sigma_bar, bool harmonic) {
  Ball<T, DIM> b;
  b.c2d = 0;
  if (harmonic) {  // sigma_bar = 0: harmonic Green's function, |G| = R^2/(2n)
    b.pb = 0;
    b.gnorm = R * R * (T)(DIM == 2 ? 0.25 : 1.0 / 6.0);
    return b;
  }
  if (DIM == 2) {
    // s < 2: a = I0 - 1, k = K0; from s = 2 on: a = e^-s I0, k = e^s K0 (one reciprocal
    // for both cases)
    T a, k;
    const bool scaled = bessel_i0k0<T>(s, &a, &k);
    const T ii0 = m_rcp(scaled ? a : (T)1 + a);
    b.pb = scaled ? (T)1 - m_exp(-s) * ii0 : a * ii0;
    b.c2d = k * ii0;
  } else {
    if (s < (T)1) {
      // (sinh s - s) = s^3 sum_{k>=0} s^{2k} / (2k+3)!, a polynomial in s^2 by Horner
      constexpr int n = sizeof(T) == 4 ? 4 : 8;
      const T s2 = s * s;
      T acc = (T)kSinhSeries.c[n];
      for (int k = n - 1; k >= 0; --k) acc = m_fma(acc, s2, (T)kSinhSeries.c[k]);
      const T shm = s * s2 * acc;
      b.pb = m_div(shm, s + shm);
    } else {
      // 1 - s/sinh(s) = 1 - 2 s e^{-s} / (1 - e^{-2s})
      b.pb = (T)1 + m_div((T)2 * s * m_exp(-s), m_expm1((T)-2 * s));
    }
  }
  b.gnorm = b.pb * inv_sigma_bar;
  return b;
}

// ------------------------------------------------------------------ kernel gradients
// grad_x G(x, y) and grad_x P(x, z) at the centre x of the ball (supplemental Sec. 1.3)
// as ratios to G(x, y) and P(x, z), so that they multiply the walk's sampled terms
// (y ~ G/|G|, z uniform on the sphere): a = f_G (y - x), b = f_P (z - x). Growing
// exponentials are carried scaled (r <= R, so e^{2(r - R) k} <= 1).
template <typename T, int DIM>
__device__ __forceinline__ T grad_ratio_green(T r, T R, T k) {
  if (!(k > (T)0)) {
    return DIM == 2 ? m_div(m_rcp(r * r) - m_rcp(R * R), m_log(R / r))
                    : m_div(m_rcp(r * r * r) - m_rcp(R * R * R), m_rcp(r) - m_rcp(R));
  }
  const T a = r * k, s = R * k;
  if (DIM == 2) {
    // (k/r) (K1(a) - (K1(s)/I1(s)) I1(a)) / (K0(a) - (K0(s)/I0(s)) I0(a)), times e^a / e^a
    const T sh = m_exp((T)2 * (a - s));
    const T c0 = m_div(bessel_k0e<T>(s), bessel_i0e<T>(s)), c1 = m_div(bessel_k1e<T>(s), bessel_i1e<T>(s));
    const T num = bessel_k1e<T>(a) - c1 * bessel_i1e<T>(a) * sh;
    const T den = bessel_k0e<T>(a) - c0 * bessel_i0e<T>(a) * sh;
    return k * m_div(num, r * den);
  }
  // 3D: (k/r^2) N / Q with N = e^{-a} (1 + 1/a) - C(a) e^{-s} (1 + 1/s) / C(s),
  // Q = (e^{-a} - e^{-s} sinh(a)/sinh(s)) / r and C(x) = cosh x - sinh(x)/x; both times e^a:
  //   N e^a = (1 + 1/a) - e^a C(a) e^{-s} (1 + 1/s) / C(s)
  //   Q e^a = (1 - (e^{2a} - 1)/(e^{2s} - 1)) / r
  const T e2s = m_exp((T)-2 * s);
  T prod;   // e^a C(a) e^{-s} (1 + 1/s) / C(s)
  if (a >= (T)0.5) {
    // e^a C(a) = (e^{2a} (1 - 1/a) + (1 + 1/a)) / 2 and C(s) = e^s ((1 - 1/s) + e^{-2s} (1 + 1/s)) / 2
    const T dsn = ((T)1 - m_rcp(s)) + e2s * ((T)1 + m_rcp(s));
    prod = m_div((m_exp((T)2 * (a - s)) * ((T)1 - m_rcp(a)) + e2s * ((T)1 + m_rcp(a))) * ((T)1 + m_rcp(s)), dsn);
  } else {
    const T a2 = a * a;
    const T ca = a2 * ((T)(1.0 / 3.0) + a2 * ((T)(1.0 / 30.0) + a2 * ((T)(1.0 / 840.0) + a2 * (T)(1.0 / 45360.0))));
    T cs;
    if (s < (T)0.5) {
      const T s2 = s * s;
      cs = s2 * ((T)(1.0 / 3.0) + s2 * ((T)(1.0 / 30.0) + s2 * ((T)(1.0 / 840.0) + s2 * (T)(1.0 / 45360.0))));
      prod = m_exp(a - s) * ca * m_div((T)1 + m_rcp(s), cs);
    } else {
      const T dsn = ((T)1 - m_rcp(s)) + e2s * ((T)1 + m_rcp(s));
      prod = (T)2 * m_exp(a - (T)2 * s) * ca * m_div((T)1 + m_rcp(s), dsn);
    }
  }
  const T num = ((T)1 + m_rcp(a)) - prod;
  const T ratio = s <= (T)10 ? m_div(m_expm1((T)2 * a), m_expm1((T)2 * s))
                             : m_div(m_exp((T)2 * (a - s)) - e2s, (T)1 - e2s);
  return k * m_div(num, r * ((T)1 - ratio));
}

template <typename T, int DIM>
__device__ __forceinline__ T grad_ratio_poisson(T R, T k) {
  if (!(k > (T)0)) return (T)(DIM == 2 ? 2.0 : 3.0) * m_rcp(R * R);
  const T s = R * k;
  if (DIM == 2) return k * k * m_div(bessel_i0e<T>(s), s * bessel_i1e<T>(s));
  // sigma sinh(s) / (s cosh(s) - sinh(s))
  if (s < (T)0.5) {
    const T s2 = s * s;
    const T num = (T)1 + s2 * ((T)(1.0 / 6.0) + s2 * ((T)(1.0 / 120.0) + s2 * (T)(1.0 / 5040.0)));
    const T den = s2 * ((T)(1.0 / 3.0) + s2 * ((T)(1.0 / 30.0) + s2 * ((T)(1.0 / 840.0) + s2 * (T)(1.0 / 45360.0))));
    return k * k * m_div(num, den);
  }
  const T e2s = m_exp((T)-2 * s);
  return k * k * m_div((T)1 - e2s, s * ((T)1 + e2s) - ((T)1 - e2s));
}

// ------------------------------------------------------------------ off-centred kernels
// Closed-form approximations of the off-centred Green's function and Poisson kernel of
// the ball B(c, R) for Lap - sigma_bar (supplemental Sec. 1.2), used by the next-flight
// walk (Sec. 5.2). With u = x - c, v = y - c, w = y - x and rho = (R^2 - u.v)/R:
//   G(x, y) |B|   = (Q(|w|) - Q(rho)) R^2/2            (2D; R^3/3 in 3D)
//   P(x, z) |dB|  = R^{n-1} (V(|w|) (R^2 - u.v)/(|w| R) + V(rho) u.v / R^2)     (|z - c| = R)
// Q and V are the radial profiles of the centred kernels (V = -Q'):
//   2D: Q = K0(kr) - (K0(kR)/I0(kR)) I0(kr),   V = k (K1(kr) + (K0(kR)/I0(kR)) I1(kr))
//   3D: Q = (e^{-kr} - e^{-kR} sinh(kr)/sinh(kR)) / r,
//       V = (k/r) (e^{-kr} (1 + 1/(kr)) + e^{-kR}/sinh(kR) (cosh(kr) - sinh(kr)/(kr)))
// and for sigma_bar = 0 the harmonic profiles Q = ln(R/r), V = 1/r (2D), Q = 1/r - 1/R,
// V = 1/r^2 (3D). Growing exponentials are carried as e^{kr - 2kR} (kr <= 2kR), so no
// term overflows in FP32.
template <typename T, int DIM>
struct NfBall {
  T R, k, s;
  T c;        // 2D: K0(s)/I0(s) (s < 2) or e^{2s} K0(s)/I0(s) (s >= 2); 3D: 1/(1 - e^{-2s})
  T shift;    // 2D: 0 (s < 2) or 2s; 3D: 2s
  bool harmonic;
};

template <typename T, int DIM>
__device__ __forceinline__ NfBall<T, DIM> nf_ball(T R, T sqrt_sigma_bar, T c2d) {
  NfBall<T, DIM> b;
  b.R = R;
  b.k = sqrt_sigma_bar;
  b.s = R * sqrt_sigma_bar;
  b.harmonic = !(sqrt_sigma_bar > (T)0);
  if (DIM == 2) {
    b.c = c2d;      // as produced by ball_terms
    b.shift = b.s < (T)2 ? (T)0 : (T)2 * b.s;
  } else {
    b.c = (T)-1 / m_expm1((T)-2 * b.s);
    b.shift = (T)2 * b.s;
  }
  return b;
}

template <typename T, int DIM>
__device__ __forceinline__ T nf_Q(const NfBall<T, DIM>& b, T r) {
  r = fmax(r, Consts<T>::kTiny);
  if (b.harmonic) return DIM == 2 ? m_log(b.R / r) : (T)1 / r - (T)1 / b.R;
  const T x = r * b.k;
  if (DIM == 2) {
    T k0;
    if (x <= (T)1) {
      T i0m1;
      bessel_series<T>(x, &i0m1, &k0);
    } else {
      k0 = bessel_k0e<T>(x) * m_exp(-x);
    }
    return k0 - b.c * bessel_i0e<T>(x) * m_exp(x - b.shift);
  }
  // e^{-s} sinh(x)/sinh(s) = (e^{x-2s} - e^{-x-2s}) / (1 - e^{-2s})
  T img;
  if (b.s < (T)1) {
    const T shx = (T)0.5 * (m_expm1(x) - m_expm1(-x));
    const T shs = (T)0.5 * (m_expm1(b.s) - m_expm1(-b.s));
    img = m_exp(-b.s) * shx / shs;
  } else {
    img = (m_exp(x - b.shift) - m_exp(-x - b.shift)) * b.c;
  }
  return (m_exp(-x) - img) / r;
}

template <typename T, int DIM>
__device__ __forceinline__ T nf_V(const NfBall<T, DIM>& b, T r) {
  r = fmax(r, Consts<T>::kTiny);
  if (b.harmonic) return DIM == 2 ? (T)1 / r : (T)1 / (r * r);
  const T x = r * b.k;
  if (DIM == 2) {
    T k1;
    if (x <= (T)1) {
      T i1;
      bessel_series1<T>(x, &i1, &k1);
    } else {
      k1 = bessel_k1e<T>(x) * m_exp(-x);
    }
    return b.k * (k1 + b.c * bessel_i1e<T>(x) * m_exp(x - b.shift));
  }
  // e^{-s}/sinh(s) (cosh x - sinh(x)/x) = 2 e^{-2s}/(1 - e^{-2s}) (cosh x - sinh(x)/x)
  T reg;
  if (x < (T)0.5) {
    const T x2 = x * x;   // cosh x - sinh(x)/x = x^2/3 + x^4/30 + x^6/840 + x^8/45360
    const T ser = x2 * ((T)(1.0 / 3.0) + x2 * ((T)(1.0 / 30.0) + x2 * ((T)(1.0 / 840.0) + x2 * (T)(1.0 / 45360.0))));
    reg = (T)2 * m_exp(-b.shift) * b.c * ser;
  } else {
    const T ix = (T)1 / x;
    reg = (m_exp(x - b.shift) * ((T)1 - ix) + m_exp(-x - b.shift) * ((T)1 + ix)) * b.c;
  }
  return b.k / r * (m_exp(-x) * ((T)1 + (T)1 / x) + reg);
}

// G(x, y) |B| for u = x - c, v = y - c.
template <typename T, int DIM>
__device__ __forceinline__ T nf_green_vol(const NfBall<T, DIM>& b, const T* u, const T* v) {
  T w2 = 0, uv = 0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    const T d = v[i] - u[i];
    w2 = m_fma(d, d, w2);
    uv = m_fma(u[i], v[i], uv);
  }
  const T rho = (b.R * b.R - uv) / b.R;
  const T vol = DIM == 2 ? (T)0.5 * b.R * b.R : b.R * b.R * b.R * (T)(1.0 / 3.0);
  return (nf_Q<T, DIM>(b, m_sqrt(w2)) - nf_Q<T, DIM>(b, rho)) * vol;
}

// P(x, z) |dB| for u = x - c and z - c = v on the sphere.
template <typename T, int DIM>
__device__ __forceinline__ T nf_poisson_area(const NfBall<T, DIM>& b, const T* u, const T* v) {
  T w2 = 0, uv = 0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    const T d = v[i] - u[i];
    w2 = m_fma(d, d, w2);
    uv = m_fma(u[i], v[i], uv);
  }
  const T R = b.R, w = fmax(m_sqrt(w2), Consts<T>::kTiny);
  const T rho = (R * R - uv) / R;
  const T p = nf_V<T, DIM>(b, w) * (R * R - uv) / (w * R) + nf_V<T, DIM>(b, rho) * uv / (R * R);
  return DIM == 2 ? p * R : p * R * R;
}

// Radius fraction t = |y - x|/R of y ~ G(x, .)/|G| (supp. Sec. 1.4). Exact rejection
// sampling with two proposals whose envelopes follow from two inequalities:
//  * the screened Green's function never exceeds the harmonic one on the same ball,
//    so the harmonic radial law (2D: t = sqrt(U1 U2), density 4 t ln(1/t); 3D: Beta(2,2))
//    is a proposal with acceptance G^s/G^0 = (K0(ts) - c I0(ts))/ln(1/t) (2D) or
//    sinh(s(1-t)) / ((1-t) sinh s) (3D) and mean cost (R^2/2n)/|G| trials;
//  * it never exceeds the free-space Green's function, whose radial law is u = ts =
//    2 sqrt(E1 E2) (2D) or E1 + E2 (3D) with E ~ Exp(1); acceptance is G^s/G^free on
//    u < s, mean cost 1/P_B trials.
// The cheaper proposal is used: s < 2 (2D) or s < sqrt 6 (3D) takes the harmonic one.
// `trials` counts proposals drawn. Acceptance per proposal is >= 0.56, so kMaxTrials is
// never reached for finite s; a non-finite s returns -1 after kMaxTrials proposals.
constexpr uint32_t kMaxTrials = 256;

// One proposal and its accept/reject test; returns t in (0, 1] on acceptance and -1 on
// rejection. The walker calls it once per iteration and lane, so a rejected lane retries
// at the next iteration instead of holding its whole wavefront in a rejection loop.
// 2D: below s = WOS_PROP_SMAX the proposal is a harmonic-law draw t0 = sqrt(U1 U2) mapped
// to t = t0^a, a = 1 + WOS_PROP_KAPPA s^2 (density proportional to t^(2/a - 1) ln(1/t)),
// accepted with t^(2 - 2/a) G(t) / (C ln(1/t)), G the screened Green's function of the unit
// disk and C >= the supremum of that ratio (proposal_bound.h): 88-100% of proposals are
// accepted there, against 56% for either proposal alone at s = 2. From WOS_PROP_SMAX on
// the free-space proposal u = 2 sqrt(E1 E2), accepted with G_ball/G_free on u < s (86% and
// more). 3D likewise with the Beta(2, 2) harmonic law below s = WOS_PROP3_SMAX (acceptance
// 0.88-1.0, against 0.57-0.97 for the harmonic law alone below sqrt 6).
template <typename T, int DIM, int S, bool COUNT = false>
__device__ __forceinline__ T radius_trial(const Rng& rng, T s, const Ball<T, DIM>& b, bool harmonic,
                                        Tally* tally = nullptr) {
  if (DIM == 2) {
    const T u1 = uniform01<T, S>(rng), u2 = uniform01<T, S + 1>(rng);
    if (harmonic) return m_sqrt(u1 * u2);
    const T u3 = uniform01<T, S + 2>(rng);
    const bool pprop = s < (T)WOS_PROP_SMAX;
    T t, x, la = 0, ae = 1, w = 1;
    if (pprop) {
      ae = m_fma((T)WOS_PROP_KAPPA * s, s, (T)1);
      w = u1 * u2;                        // t0^2
      la = (T)-0.5 * m_logn(w);           // ln(1/t0)
      t = m_exp(-ae * la);
      x = t * s;
    } else {
      if constexpr (COUNT) ++tally->trials_free;
      x = (T)2 * m_sqrt(m_logn(u1) * m_logn(u2));
      t = m_div(x, s);
    }
    T a, k;
    const bool scaled = bessel_i0k0<T>(x, &a, &k);
    if (pprop) {
      // G(t) = K0(x) - K0(s) I0(x) / I0(s). From x = 2 on the Bessel values are scaled
      // (K0(x) = k e^-x, I0(x) = a e^x), and so is the ball's c2d from s = 2 on (K0(s)/I0(s)
      // = c2d e^-2s); x <= s, so the two exponentials of the second term combine into one
      const T k0x = scaled ? k * m_exp(-x) : k;
      const T e2 = m_exp((s >= (T)2 ? (T)-2 * s : (T)0) + (scaled ? x : (T)0));
      const T g = k0x - b.c2d * (scaled ? a : (T)1 + a) * e2;
      const T C = envelope_series<T>(WOS_PROP_C, WOS_PROP_P, WOS_PROP_N, s * (T)(2.0 / WOS_PROP_SMAX) - (T)1);
      // accept if u3 C ln(1/t) <= t^(2 - 2/a) G(t), with ln(1/t) = a ln(1/t0) and
      // t^(2 - 2/a) = t0^(2a - 2) = t^2 / t0^2, multiplied through by t0^2
      return u3 * C * ae * la * w <= t * t * g ? t : (T)-1;
    }
    // 1 - G_ball/G_free = c2d I0(x)/K0(x) e^{-2s} with c2d = e^{2s} K0(s)/I0(s)
    const T r = b.c2d * m_div(scaled ? a : (T)1 + a, k) * m_exp(scaled ? (T)2 * (x - s) : (T)-2 * s);
    return (x < s && u3 <= (T)1 - r) ? t : (T)-1;
  } else {
    if (harmonic || s < (T)WOS_PROP3_SMAX) {
      // Beta(2,2) = median of three uniforms, t0; below s = WOS_PROP3_SMAX mapped to
      // t = t0^a, a = 1 + WOS_PROP3_KAPPA s^2 (proposal density proportional to
      // t^(2/a - 1) (1 - t^(1/a))), accepted with t^(2 - 2/a) sinh(s (1 - t)) /
      // (C sinh(s) (1 - t0)), C >= its supremum over t: a s / sinh(s) below
      // WOS_PROP3_SK, the series of proposal_bound.h above
      const T a = uniform01<T, S>(rng), c = uniform01<T, S + 1>(rng), d = uniform01<T, S + 2>(rng);
      const T t0 = fmax(fmin(a, c), fmin(fmax(a, c), d));
      if (harmonic) return t0;
      const T u4 = uniform01<T, S + 3>(rng);
      const T ae = m_fma((T)WOS_PROP3_KAPPA * s, s, (T)1);
      const T lt0 = m_logn(t0);
      const T t = m_exp(ae * lt0);
      const T omt = (T)1 - t;
      // sinh(s(1-t)) / sinh(s) = e^{-st} (1 - e^{-2s(1-t)}) / (1 - e^{-2s})
      const T e2s = m_expm1((T)-2 * s);
      const T sr = omt > (T)0 ? m_div(m_exp(-s * t) * m_expm1((T)-2 * s * omt), e2s) : (T)0;
      const T C = s < (T)WOS_PROP3_SK
                      ? ae * m_div((T)-2 * s * m_exp(-s), e2s) * (T)1.00001
                      : envelope_series<T>(WOS_PROP3_C, WOS_PROP3_P, WOS_PROP3_N,
                                     (s - (T)WOS_PROP3_SK) * (T)(2.0 / (WOS_PROP3_SMAX - WOS_PROP3_SK)) - (T)1);
      // u4 C <= t0^(2a - 2) sr / (1 - t0), with t0^(2a - 2) = t^2 / t0^2, multiplied through
      // by t0^2 (1 - t0)
      return u4 * C * (t0 * t0) * ((T)1 - t0) <= t * t * sr ? t : (T)-1;
    }
    if constexpr (COUNT) ++tally->trials_free;
    const T u = -m_logn(uniform01<T, S>(rng) * uniform01<T, S + 1>(rng));
    const T u3 = uniform01<T, S + 2>(rng);
    if (!(u < s)) return (T)-1;
    // G^s/G^free = 1 - e^{u-s} sinh(u)/sinh(s) = 1 - e^{2(u-s)} (1 - e^{-2u})/(1 - e^{-2s})
    const T r = m_div(m_exp((T)2 * (u - s)) * m_expm1((T)-2 * u), m_expm1((T)-2 * s));
    return u3 <= (T)1 - r ? m_div(u, s) : (T)-1;
  }
}

// Trials until acceptance (at most kMaxTrials; -1 if none is accepted), each on a fresh
// draw of the stream.
template <typename T, int DIM, bool COUNT = false>
__device__ __forceinline__ T sample_radius(Rng& rng, T s, const Ball<T, DIM>& b, bool harmonic, uint32_t& trials,
                                         Tally* tally = nullptr) {
  for (uint32_t k = 0; k < kMaxTrials; ++k) {
    ++trials;
    rng.refill<Slots<T, DIM>::blocks(4)>();
    const T t = radius_trial<T, DIM, 0, COUNT>(rng, s, b, harmonic, tally);
    if (t >= (T)0) return t;
  }
  return (T)-1;
}

// Uniform direction on the unit sphere from uniform slots S .. S + DIM - 2.
template <typename T, int DIM, int S>
__device__ __forceinline__ void uniform_direction(const Rng& rng, T* v) {
  if (DIM == 2) {
    T sn, cs;
    m_sincospi2_unit(uniform01<T, S>(rng), &sn, &cs);
    v[0] = cs;
    v[1] = sn;
  } else {
    const T z = (T)1 - (T)2 * uniform01<T, S>(rng);
    T sn, cs;
    m_sincospi2_unit(uniform01<T, S + 1>(rng), &sn, &cs);
    const T rr = m_sqrt(fmax((T)0, (T)1 - z * z));
    v[0] = rr * cs;
    v[1] = rr * sn;
    v[2] = z;
  }
}

// Uniform point in the ball of radius R centred at the origin: uniform direction and
// radius R U^{1/n}, from uniform slots S .. S + DIM - 1.
template <typename T, int DIM, int S>
__device__ __forceinline__ void uniform_in_ball(const Rng& rng, T R, T* p) {
  uniform_direction<T, DIM, S>(rng, p);
  const T u = uniform01<T, S + DIM - 1>(rng);
  const T r = R * (DIM == 2 ? m_sqrt(u) : m_cbrt(u));
#pragma unroll
  for (int i = 0; i < DIM; ++i) p[i] *= r;
}

// ------------------------------------------------------------------ coefficient fields

template <typename T, int DIM>
struct FV {
  T v;
  T g[DIM];
  T lap;
};

template <typename T, int DIM>
__device__ __forceinline__ T axis_component(const T* x, int ax) {
  T v = x[0];
#pragma unroll
  for (int i = 1; i < DIM; ++i) v = ax == i ? x[i] : v;
  return v;
}

// Base function B of a field at x, with gradient and Laplacian when D is true.
template <typename T, int DIM, bool D>
__device__ __forceinline__ FV<T, DIM> field_base(G<DevField<T>>& f, const T* x) {
  FV<T, DIM> r;
  r.v = 0;
  r.lap = 0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) r.g[i] = 0;
  const int base = f.base;
  if (base == FB_FOURIER) {
    const WOS_GLOBAL T* p = gptr(f.terms);
    for (int j = 0; j < f.n; ++j, p += kTermStride) {
      if (!D) {
        // value alone: a cos(2 pi (k.x + phi / 2 pi)), one cosine
        T th = m_fma(p[0], x[0], m_fma(p[1], x[1], p[7]));
        if (DIM == 3) th = m_fma(p[2], x[2], th);
        r.v = m_fma(p[6], m_cospi2(th), r.v);
        continue;
      }
      // phase k.x in revolutions (k in cycles per unit length)
      T th = p[0] * x[0] + p[1] * x[1];
      if (DIM == 3) th = m_fma(p[2], x[2], th);
      T sn, cs;
      m_sincospi2(th, &sn, &cs);
      const T ac = p[3], as = p[4];
      const T val = ac * cs - as * sn;                 // a cos(2 pi k.x + phi)
      r.v += val;
      if (D) {
        constexpr T kTwoPi = (T)6.283185307179586476925286766559;
        const T dval = -(ac * sn + as * cs) * kTwoPi;   // -2 pi a sin(2 pi k.x + phi)
#pragma unroll
        for (int i = 0; i < DIM; ++i) r.g[i] = m_fma(dval, p[i], r.g[i]);
        r.lap = m_fma(-val, p[5], r.lap);                // Laplacian: -|2 pi k|^2 B_j
      }
    }
  } else if (base == FB_BUMPS) {
    const WOS_GLOBAL T* p = gptr(f.terms);
    for (int j = 0; j < f.n; ++j, p += kTermStride) {
      T d[DIM], r2 = 0;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        d[i] = x[i] - p[i];
        r2 = m_fma(d[i], d[i], r2);
      }
      const T e = p[4] * m_exp2(-r2 * p[3]);   // p[3] = log2(e) / (2 w^2)
      r.v += e;
      if (D) {
        const T iw2 = p[5];
#pragma unroll
        for (int i = 0; i < DIM; ++i) r.g[i] = m_fma(-e * iw2, d[i], r.g[i]);
        r.lap = m_fma(e, iw2 * (r2 * iw2 - (T)DIM), r.lap);
      }
    }
  } else if (base == FB_TANH) {
    // the axis is a run-time value: select with compile-time indices so that x and r
    // stay in registers (a dynamic index would place them in scratch memory)
    const int ax = (int)f.prm[0];
    const T iw = f.prm[2];
    const T th = m_tanh((axis_component<T, DIM>(x, ax) - f.prm[1]) * iw);
    r.v = (T)0.5 * ((T)1 + th);
    if (D) {
      const T sech2 = (T)1 - th * th;
      const T ga = (T)0.5 * sech2 * iw;
#pragma unroll
      for (int i = 0; i < DIM; ++i) r.g[i] = i == ax ? ga : (T)0;
      r.lap = -th * sech2 * iw * iw;
    }
  } else if (base == FB_TANH_DRIFT) {
    // psi = K [A z - B ln(A cosh z + B sinh z) + B ln A], alpha psi' = omega along the axis
    const int ax = (int)f.prm[0];
    const T iw = f.prm[2], A = f.prm[3], B = f.prm[4], K = f.prm[5], lnA = f.prm[6], om = f.prm[7];
    const T z = (axis_component<T, DIM>(x, ax) - f.prm[1]) * iw;
    const T az = m_fabs(z);
    const T sg = z >= (T)0 ? (T)1 : (T)-1;
    const T lnmix = az + m_log((T)0.5 * (A + sg * B) + (T)0.5 * (A - sg * B) * m_exp((T)-2 * az));
    r.v = K * (A * z - B * lnmix + B * lnA);
    if (D) {
      const T th = m_tanh(z);
      const T al = A + B * th;
      const T dal = B * ((T)1 - th * th) * iw;
      const T ga = om / al;
#pragma unroll
      for (int i = 0; i < DIM; ++i) r.g[i] = i == ax ? ga : (T)0;
      r.lap = -om * dal / (al * al);
    }
  }
  return r;
}

// Bases of the Fourier fields of a 2D problem from the dense table (slots 0, 1, 2), with
// gradient and Laplacian for the first ND slots when D is true. The table is in product
// form, B = sum_a psi_a(x) (M phi(y))_a: for each row a one dot product with the seven y
// basis functions per slot (and per derivative in y), then one multiply-add with psi_a;
// the x derivatives come from the same row sums with the derivatives of psi_a. Only two
// sincos calls per point; the rest are fused multiply-adds on wave-uniform coefficients.
template <typename T>
__device__ __forceinline__ T spectral_dot(const WOS_GLOBAL T* r, const T* phi) {
  T v = r[0];
#pragma unroll
  for (int b = 1; b < kSpecRow; ++b) v = m_fma(r[b], phi[b], v);
  return v;
}

// Values of the three slots with the gradient and Laplacian of slot 0 alone. The x
// derivatives come from the row sums V_a = (M phi)_a as in spectral2d; the y derivatives
// from the column sums T_b = (psi^T M)_b of the value table, accumulated over the same row
// pairs (two multiply-adds per column and row pair), as sum_b T_b phi'_b and
// sum_b T_b phi''_b, with phi' and phi'' the y derivatives of the basis. This replaces the
// two extra dot products per row of the derivative tables (about a fifth fewer
// multiply-adds, and the derivative rows are not loaded).
template <typename T>
__device__ __forceinline__ void spectral2d_first_slot(G<Spectral2D<T>>& sp, const T* x, const T* phi,
                                                      FV<T, 2>* out) {
  T tb[kSpecRow];
#pragma unroll
  for (int b = 0; b < kSpecRow; ++b) tb[b] = sp.m[0][0][0][b];
#pragma unroll
  for (int s = 0; s < 3; ++s) out[s].v = spectral_dot<T>(sp.m[0][s][0], phi);
  T cx1, sx1;
  m_sincospi2(x[0], &sx1, &cx1);
  T c = cx1, sn = sx1, gx = 0, lx = 0, fn = 0;
#pragma unroll 1
  for (int n = 1; n <= kSpecK; ++n) {
    fn += (T)1;
    const WOS_GLOBAL T* rc = sp.m[2 * n - 1][0][0];
    const WOS_GLOBAL T* rs = sp.m[2 * n][0][0];
    const T vc = spectral_dot<T>(rc, phi);
    const T vs = spectral_dot<T>(rs, phi);
    const T u = m_fma(vc, c, vs * sn);
    out[0].v += u;
    gx = m_fma(fn, m_fma(vs, c, -vc * sn), gx);
    lx = m_fma(-fn * fn, u, lx);
#pragma unroll
    for (int b = 0; b < kSpecRow; ++b) tb[b] = m_fma(rc[b], c, m_fma(rs[b], sn, tb[b]));
#pragma unroll
    for (int s = 1; s < 3; ++s) {
      const T wc = spectral_dot<T>(sp.m[2 * n - 1][s][0], phi);
      const T ws = spectral_dot<T>(sp.m[2 * n][s][0], phi);
      out[s].v = m_fma(wc, c, m_fma(ws, sn, out[s].v));
    }
    const T t = m_fma(c, cx1, -sn * sx1);
    sn = m_fma(sn, cx1, c * sx1);
    c = t;
  }
  // phi'_{2n-1} = -w sin, phi'_{2n} = w cos; phi'' = -w^2 phi (w = 2 pi n)
  constexpr T kTwoPi = (T)6.283185307179586476925286766559;
  constexpr T kFourPi2 = (T)39.478417604357434475337963999505;
  T gy = 0, lyy = 0;
#pragma unroll
  for (int n = 1; n <= kSpecK; ++n) {
    const T cn = phi[2 * n - 1], snn = phi[2 * n];
    gy = m_fma((T)n, m_fma(tb[2 * n], cn, -tb[2 * n - 1] * snn), gy);
    lyy = m_fma((T)(-n * n), m_fma(tb[2 * n - 1], cn, tb[2 * n] * snn), lyy);
  }
  out[0].g[0] = kTwoPi * gx;
  out[0].g[1] = kTwoPi * gy;
  out[0].lap = kFourPi2 * (lx + lyy);
}

template <typename T, bool D, int ND = 2>
__device__ __forceinline__ void spectral2d(G<Spectral2D<T>>& sp, const T* x, FV<T, 2>* out) {
  // phi(y) = 1, cos 2 pi y, sin 2 pi y, cos 4 pi y, sin 4 pi y, cos 6 pi y, sin 6 pi y
  T phi[kSpecRow];
  phi[0] = 1;
  m_sincospi2(x[1], &phi[2], &phi[1]);
#pragma unroll
  for (int n = 2; n <= kSpecK; ++n) {
    const T pc = phi[2 * n - 3], ps = phi[2 * n - 2];
    phi[2 * n - 1] = m_fma(pc, phi[1], -ps * phi[2]);
    phi[2 * n] = m_fma(ps, phi[1], pc * phi[2]);
  }
  if constexpr (D && ND == 1) {
    spectral2d_first_slot<T>(sp, x, phi, out);
    return;
  }
  // row a = 0 (psi_0 = 1)
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    out[s].v = spectral_dot<T>(sp.m[0][s][0], phi);
    if (D && s < ND) {
      out[s].g[0] = 0;
      out[s].g[1] = spectral_dot<T>(sp.m[0][s][1], phi);
      out[s].lap = spectral_dot<T>(sp.m[0][s][2], phi);
    }
  }
  T cx1, sx1;
  m_sincospi2(x[0], &sx1, &cx1);
  T c = cx1, sn = sx1;   // cos and sin of 2 pi n x
  T gx[ND > 0 ? ND : 1], lx[ND > 0 ? ND : 1];
#pragma unroll
  for (int s = 0; s < ND; ++s) {
    gx[s] = 0;
    lx[s] = 0;
  }
  // rows 2n - 1 (cos 2 pi n x) and 2n (sin 2 pi n x); the loop is kept rolled so that one
  // pair of rows of coefficients (scalar loads) is live at a time
#pragma unroll 1
  for (int n = 1; n <= kSpecK; ++n) {
    const T fn = (T)n;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const T vc = spectral_dot<T>(sp.m[2 * n - 1][s][0], phi);
      const T vs = spectral_dot<T>(sp.m[2 * n][s][0], phi);
      const T u = m_fma(vc, c, vs * sn);
      out[s].v += u;
      if (D && s < ND) {
        // d/dx: 2 pi n (vs cos - vc sin); d2/dx2: -(2 pi n)^2 u (2 pi factors applied below)
        gx[s] = m_fma(fn, m_fma(vs, c, -vc * sn), gx[s]);
        lx[s] = m_fma(-fn * fn, u, lx[s]);
        const T wc = spectral_dot<T>(sp.m[2 * n - 1][s][1], phi);
        const T ws = spectral_dot<T>(sp.m[2 * n][s][1], phi);
        out[s].g[1] += m_fma(wc, c, ws * sn);
        const T zc = spectral_dot<T>(sp.m[2 * n - 1][s][2], phi);
        const T zs = spectral_dot<T>(sp.m[2 * n][s][2], phi);
        out[s].lap += m_fma(zc, c, zs * sn);
      }
    }
    const T t = m_fma(c, cx1, -sn * sx1);
    sn = m_fma(sn, cx1, c * sx1);
    c = t;
  }
  constexpr T kTwoPi = (T)6.283185307179586476925286766559;
  constexpr T kFourPi2 = (T)39.478417604357434475337963999505;
#pragma unroll
  for (int s = 0; s < ND; ++s) {
    if (D) {
      out[s].g[0] = kTwoPi * gx[s];
      out[s].lap = m_fma(kFourPi2, lx[s], out[s].lap);
    }
  }
}

// Field after its transform (c0 + c1 B or exp(c0 + c1 B)) from its base B; `log` of the
// exp transform is available without a logarithm.
template <typename T, int DIM, bool D>
__device__ __forceinline__ FV<T, DIM> field_transform(G<DevField<T>>& f, const FV<T, DIM>& b,
                                                      T* log_value = nullptr) {
  FV<T, DIM> r;
  const T c1 = f.c1;
  if (f.transform == FT_EXP) {
    const T lv = m_fma(c1, b.v, f.c0);
    if (log_value) *log_value = lv;
    r.v = m_exp(lv);
    if (D) {
      T gb2 = 0;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        r.g[i] = r.v * c1 * b.g[i];
        gb2 = m_fma(b.g[i], b.g[i], gb2);
      }
      r.lap = r.v * (c1 * b.lap + c1 * c1 * gb2);
    }
  } else {
    r.v = m_fma(c1, b.v, f.c0);
    if (D) {
#pragma unroll
      for (int i = 0; i < DIM; ++i) r.g[i] = c1 * b.g[i];
      r.lap = c1 * b.lap;
    }
  }
  return r;
}

template <typename T, int DIM, bool D>
__device__ __forceinline__ FV<T, DIM> field_eval(G<DevField<T>>& f, const T* x, T* log_value = nullptr) {
  return field_transform<T, DIM, D>(f, field_base<T, DIM, D>(f, x), log_value);
}

// Manufactured solutions u (value, gradient, Laplacian).
template <typename T, int DIM>
__device__ __forceinline__ FV<T, DIM> solution(int id, const T* x) {
  FV<T, DIM> u;
#pragma unroll
  for (int i = 0; i < DIM; ++i) u.g[i] = 0;
  if (id == SOL_EXPCOS) {
    const T e = m_exp(x[0]);
    T sn, cs;
    m_sincos(x[1], &sn, &cs);
    u.v = e * cs;
    u.g[0] = e * cs;
    u.g[1] = -e * sn;
    u.lap = 0;
  } else {
    u.v = (T)1 + x[0] * x[0] + (T)0.5 * x[0] * x[1];
    u.g[0] = (T)2 * x[0] + (T)0.5 * x[1];
    u.g[1] = (T)0.5 * x[0];
    u.lap = 2;
  }
  return u;
}

// What one step needs at a point after the change of variables (Sec. 4.1, App. A):
//   gamma = (ln alpha + psi)/2, sigma' = sigma/alpha + Lap(gamma) + |grad gamma|^2 and
//   f/alpha (the source enters as e^{gamma(y) - gamma(x)} f(y)/alpha(y)).
template <typename T>
struct PointCoef {
  T gamma;
  T sigma_prime;
  T f_over_alpha;
  T alpha;
};

// Bases of alpha, psi and sigma at x: from the dense 2D table where the problem has one,
// else field by field.
template <typename T, int DIM, bool D>
__device__ __forceinline__ void coefficient_bases(G<DevProblem<T>>& P, const T* x, FV<T, DIM>* b) {
  const int sp = DIM == 2 ? P.spectral : 0;
  if constexpr (DIM == 2) {
    if (sp) spectral2d<T, D>(P.spec, x, b);
  }
  if (!(sp & 1)) b[0] = field_base<T, DIM, D>(P.alpha, x);
  if (!(sp & 2)) b[1] = field_base<T, DIM, D>(P.psi, x);
  if (!(sp & 4)) b[2] = field_base<T, DIM, false>(P.sigma, x);
}

// gamma with its gradient and Laplacian, alpha, 1/alpha and sigma at x.
template <typename T, int DIM>
__device__ __forceinline__ void gamma_alpha_sigma(G<DevProblem<T>>& P, const T* x, FV<T, DIM>& gam, T& alpha,
                                                  T& inv_alpha, T& sigma) {
  if constexpr (DIM == 2) {
    if (P.spectral & kSpecGammaMerged) {
      // the table holds gamma itself (slot 0) and the base of alpha = exp(c0 + c1 B) (slot 1)
      FV<T, 2> b[3];
      spectral2d<T, true, 1>(P.spec, x, b);
      gam = b[0];
      const T la = m_fma(P.alpha.c1, b[1].v, P.alpha.c0);
      alpha = m_exp(la);
      inv_alpha = m_exp(-la);   // (the walker uses 1/alpha alone: one exponential)
      if (!(P.spectral & 4)) b[2] = field_base<T, 2, false>(P.sigma, x);
      sigma = field_transform<T, 2, false>(P.sigma, b[2]).v;
      return;
    }
  }
  FV<T, DIM> base[3];
  coefficient_bases<T, DIM, true>(P, x, base);
  // ln alpha with its gradient and Laplacian: grad ln a = grad a / a,
  // Lap ln a = Lap a / a - |grad ln a|^2 (for the exp transform ln a = c0 + c1 B directly)
  T lnal;
  const FV<T, DIM> al = field_transform<T, DIM, true>(P.alpha, base[0], &lnal);
  if (P.alpha.transform != FT_EXP) lnal = m_log(al.v);
  const T inv_al = m_rcp(al.v);
  T gl[DIM], ga2 = 0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    gl[i] = al.g[i] * inv_al;
    ga2 = m_fma(gl[i], gl[i], ga2);
  }
  const T lapl = m_fma(al.lap, inv_al, -ga2);
  if (P.psi.base == FB_NONE && P.psi.transform == FT_AFFINE) {
    gam.v = (T)0.5 * (lnal + P.psi.c0);
#pragma unroll
    for (int i = 0; i < DIM; ++i) gam.g[i] = (T)0.5 * gl[i];
    gam.lap = (T)0.5 * lapl;
  } else {
    const FV<T, DIM> ps = field_transform<T, DIM, true>(P.psi, base[1]);
    gam.v = (T)0.5 * (lnal + ps.v);
#pragma unroll
    for (int i = 0; i < DIM; ++i) gam.g[i] = (T)0.5 * (gl[i] + ps.g[i]);
    gam.lap = (T)0.5 * (lapl + ps.lap);
  }
  alpha = al.v;
  inv_alpha = inv_al;
  sigma = field_transform<T, DIM, false>(P.sigma, base[2]).v;
}

template <typename T, int DIM, bool WITH_SOURCE>
__device__ __forceinline__ PointCoef<T> point_coef(G<DevProblem<T>>& P, const T* x, T* grad_gamma = nullptr) {
  FV<T, DIM> gam;
  T alpha, inv_al, sig;
  gamma_alpha_sigma<T, DIM>(P, x, gam, alpha, inv_al, sig);
  T g2 = 0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) g2 = m_fma(gam.g[i], gam.g[i], g2);
  if (grad_gamma) {
#pragma unroll
    for (int i = 0; i < DIM; ++i) grad_gamma[i] = gam.g[i];
  }
  PointCoef<T> c;
  c.gamma = gam.v;
  c.alpha = alpha;
  c.sigma_prime = m_fma(sig, inv_al, gam.lap + g2);
  c.f_over_alpha = 0;
  if (WITH_SOURCE) {
    if (P.source.base == FB_MANUFACTURED) {
      // f = -div(alpha grad u) - omega.grad u + sigma u = -alpha (Lap u + 2 grad(gamma).grad u) + sigma u
      const FV<T, DIM> u = solution<T, DIM>(P.source.sol, x);
      T gu = 0;
#pragma unroll
      for (int i = 0; i < DIM; ++i) gu = m_fma(gam.g[i], u.g[i], gu);
      c.f_over_alpha = -(u.lap + (T)2 * gu) + sig * inv_al * u.v;
    } else {
      c.f_over_alpha = field_eval<T, DIM, false>(P.source, x).v * inv_al;
    }
  }
  return c;
}

template <typename T, int DIM>
__device__ __forceinline__ T boundary_value(G<DevProblem<T>>& P, const T* x) {
  if (P.boundary.base == FB_MANUFACTURED) return solution<T, DIM>(P.boundary.sol, x).v;
  return field_eval<T, DIM, false>(P.boundary, x).v;
}

// gamma alone (exit points of walks that need the full weight, and the last point)
template <typename T, int DIM>
__device__ __forceinline__ T point_gamma(G<DevProblem<T>>& P, const T* x) {
  T lnal, ps = P.psi.c0;
  const bool has_psi = !(P.psi.base == FB_NONE && P.psi.transform == FT_AFFINE);
  if (DIM == 2 && P.spectral) {
    FV<T, DIM> base[3];
    if constexpr (DIM == 2) spectral2d<T, false>(P.spec, x, base);
    if (P.spectral & kSpecGammaMerged) return base[0].v;
    if (!(P.spectral & 1)) base[0] = field_base<T, DIM, false>(P.alpha, x);
    if (has_psi && !(P.spectral & 2)) base[1] = field_base<T, DIM, false>(P.psi, x);
    const FV<T, DIM> al = field_transform<T, DIM, false>(P.alpha, base[0], &lnal);
    if (P.alpha.transform != FT_EXP) lnal = m_log(al.v);
    if (has_psi) ps = field_transform<T, DIM, false>(P.psi, base[1]).v;
  } else {
    const FV<T, DIM> al = field_eval<T, DIM, false>(P.alpha, x, &lnal);
    if (P.alpha.transform != FT_EXP) lnal = m_log(al.v);
    if (has_psi) ps = field_eval<T, DIM, false>(P.psi, x).v;
  }
  return (T)0.5 * (lnal + ps);
}

// ------------------------------------------------------------------ distance queries

template <typename T, int DIM, typename PT>
__device__ __forceinline__ T box_dist2(const T* x, PT lo, PT hi) {
  T d2 = 0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    const T e = fmax(fmax(lo[i] - x[i], x[i] - hi[i]), (T)0);
    d2 = m_fma(e, e, d2);
  }
  return d2;
}

template <typename T, typename PT>
__device__ __forceinline__ T segment_dist2(const T* x, PT s, T* tpar) {
  const T ex = s[2] - s[0], ey = s[3] - s[1];
  const T px = x[0] - s[0], py = x[1] - s[1];
  const T l2 = m_fma(ex, ex, ey * ey);
  T t = l2 > (T)0 ? m_div(m_fma(px, ex, py * ey), l2) : (T)0;
  t = fmin(fmax(t, (T)0), (T)1);
  const T dx = px - t * ex, dy = py - t * ey;
  *tpar = t;
  return m_fma(dx, dx, dy * dy);
}

// The same for a segment given as start point, edge vector and 1/|e|^2 (0 for a point).
template <typename T, typename PT>
__device__ __forceinline__ T segment_dist2_pre(const T* x, PT s, T inv_len2) {
  const T px = x[0] - s[0], py = x[1] - s[1];
  T t = m_fma(px, s[2], py * s[3]) * inv_len2;
  t = fmin(fmax(t, (T)0), (T)1);
  const T dx = m_fma(-t, s[2], px), dy = m_fma(-t, s[3], py);
  return m_fma(dx, dx, dy * dy);
}

// Closest point of triangle (a, b, c) = (tri[0..2], tri[3..5], tri[6..8]) to p, by the
// Voronoi regions of its vertices, edges and face (Ericson, Real-Time Collision
// Detection, Sec. 5.1.5).
template <typename T, typename PT>
__device__ __forceinline__ void triangle_closest(const T* p, PT tri, T* q) {
  const T a[3] = {tri[0], tri[1], tri[2]};
  T ab[3], ac[3];
  for (int i = 0; i < 3; ++i) {
    ab[i] = tri[3 + i] - a[i];
    ac[i] = tri[6 + i] - a[i];
  }
  T ap[3];
  for (int i = 0; i < 3; ++i) ap[i] = p[i] - a[i];
  const T d1 = ab[0] * ap[0] + ab[1] * ap[1] + ab[2] * ap[2];
  const T d2 = ac[0] * ap[0] + ac[1] * ap[1] + ac[2] * ap[2];
  if (d1 <= (T)0 && d2 <= (T)0) { for (int i = 0; i < 3; ++i) q[i] = a[i]; return; }
  T bp[3];
  for (int i = 0; i < 3; ++i) bp[i] = ap[i] - ab[i];
  const T d3 = ab[0] * bp[0] + ab[1] * bp[1] + ab[2] * bp[2];
  const T d4 = ac[0] * bp[0] + ac[1] * bp[1] + ac[2] * bp[2];
  if (d3 >= (T)0 && d4 <= d3) { for (int i = 0; i < 3; ++i) q[i] = a[i] + ab[i]; return; }
  const T vc = d1 * d4 - d3 * d2;
  if (vc <= (T)0 && d1 >= (T)0 && d3 <= (T)0) {
    const T v = m_div(d1, d1 - d3);
    for (int i = 0; i < 3; ++i) q[i] = a[i] + v * ab[i];
    return;
  }
  T cp[3];
  for (int i = 0; i < 3; ++i) cp[i] = ap[i] - ac[i];
  const T d5 = ab[0] * cp[0] + ab[1] * cp[1] + ab[2] * cp[2];
  const T d6 = ac[0] * cp[0] + ac[1] * cp[1] + ac[2] * cp[2];
  if (d6 >= (T)0 && d5 <= d6) { for (int i = 0; i < 3; ++i) q[i] = a[i] + ac[i]; return; }
  const T vb = d5 * d2 - d1 * d6;
  if (vb <= (T)0 && d2 >= (T)0 && d6 <= (T)0) {
    const T w = m_div(d2, d2 - d6);
    for (int i = 0; i < 3; ++i) q[i] = a[i] + w * ac[i];
    return;
  }
  const T va = d3 * d6 - d5 * d4;
  if (va <= (T)0 && (d4 - d3) >= (T)0 && (d5 - d6) >= (T)0) {
    const T w = m_div(d4 - d3, (d4 - d3) + (d5 - d6));
    for (int i = 0; i < 3; ++i) q[i] = a[i] + ab[i] + w * (ac[i] - ab[i]);
    return;
  }
  const T denom = m_rcp(va + vb + vc);
  const T v = vb * denom, w = vc * denom;
  for (int i = 0; i < 3; ++i) q[i] = a[i] + ab[i] * v + ac[i] * w;
}

template <typename T, typename PT>
__device__ __forceinline__ T triangle_dist2(const T* p, PT tri) {
  T q[3];
  triangle_closest<T>(p, tri, q);
  const T dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
  return m_fma(dx, dx, m_fma(dy, dy, dz * dz));
}

constexpr int kPrimStride2 = 4;    // segment: x0 y0 x1 y1
constexpr int kPrimStride3 = 12;   // triangle: a, b, c, (pad)
constexpr int kStackDepth = 48;     // private (scratch) stack: any tree the host accepts
// LDS stack depths of the walker. The walker's LDS must leave room for five 256-thread
// blocks per CU: the mesh walker takes trees of depth <= 15 (30 KB in FP32), the polygon
// walker, whose candidate grid answers most queries, trees of depth <= 12 (24 KB; up to
// about 8000 edges). Deeper trees use the private stack.
constexpr int kLdsStackDepth = 15;
constexpr int kLdsStackDepthPolygon = 12;

// Traversal stack of far children with their box distances, either in LDS (one column
// per lane: entry k of lane t at k * stride + t, conflict-free) for trees of depth <= depth,
// or in private memory.
template <typename T>
struct LdsStack {
  int32_t* node;   // null: use the private stack
  T* dist;
  int stride;
  int depth;
};

// Nearest primitive by BVH traversal; returns squared distance and primitive index.
template <typename T, int DIM>
__device__ __forceinline__ T prim_dist2(const WOS_GLOBAL T* prims, const T* x, int pi) {
  if (DIM == 2) {
    T tp;
    return segment_dist2<T>(x, prims + (size_t)pi * kPrimStride2, &tp);
  }
  return triangle_dist2<T>(x, prims + (size_t)pi * kPrimStride3);
}

// Nearest primitive by BVH traversal; returns squared distance and primitive index.
// `hint` (>= 0) is a primitive whose distance seeds the bound: a walk moves by at most
// the previous distance per step, so the previous closest primitive is usually still
// closest or nearly so, and the traversal then prunes all but a few nodes. The result
// is the exact nearest distance either way.
template <typename T, int DIM, bool COUNT = false>
__device__ __forceinline__ T bvh_nearest(G<DevGeometry<T>>& g, const T* x, int* best_prim, Tally* tally = nullptr,
                                         LdsStack<T> lds = LdsStack<T>{nullptr, nullptr, 0, 0}, int hint = -1) {
  if (lds.node && g.depth <= lds.depth) {
    const WOS_GLOBAL BvhNode<T, DIM>* nodes = (const WOS_GLOBAL BvhNode<T, DIM>*)g.nodes;
    const WOS_GLOBAL T* prims = gptr(g.prims);
    T best = Consts<T>::kInf;
    int bp = -1;
    if (hint >= 0) {
      best = prim_dist2<T, DIM>(prims, x, hint);
      bp = hint;
      if constexpr (COUNT) ++tally->prims;
    }
    int sp = 0;
    int cur = g.root;
    T cur_d = 0;
    for (;;) {
      if (cur_d < best) {
        if (cur < 0) {
          const int code = -1 - cur;
          const int first = code >> 3, cnt = code & 7;
          if constexpr (COUNT) tally->prims += cnt;
          for (int k = 0; k < cnt; ++k) {
            const int pi = first + k;
            T d2;
            if (DIM == 2) {
              T tp;
              d2 = segment_dist2<T>(x, prims + (size_t)pi * kPrimStride2, &tp);
            } else {
              d2 = triangle_dist2<T>(x, prims + (size_t)pi * kPrimStride3);
            }
            if (d2 < best) {
              best = d2;
              bp = pi;
            }
          }
        } else {
          G<BvhNode<T, DIM>>& n = nodes[cur];
          if constexpr (COUNT) ++tally->nodes;
          const T da = box_dist2<T, DIM>(x, n.lo[0], n.hi[0]);
          const T db = box_dist2<T, DIM>(x, n.lo[1], n.hi[1]);
          const int ca = n.child[0], cb = n.child[1];
          const bool a_first = da <= db;
          const int near_c = a_first ? ca : cb, far_c = a_first ? cb : ca;
          const T near_d = a_first ? da : db, far_d = a_first ? db : da;
          if (far_d < best) {  // at most one entry per level above the current node
            lds.node[sp * lds.stride] = far_c;
            lds.dist[sp * lds.stride] = far_d;
            ++sp;
          }
          cur = near_c;
          cur_d = near_d;
          continue;
        }
      }
      if (sp == 0) break;
      --sp;
      cur = lds.node[sp * lds.stride];
      cur_d = lds.dist[sp * lds.stride];
    }
    *best_prim = bp;
    return best;
  }
  const WOS_GLOBAL BvhNode<T, DIM>* nodes = (const WOS_GLOBAL BvhNode<T, DIM>*)g.nodes;
  const WOS_GLOBAL T* prims = gptr(g.prims);
  T best = Consts<T>::kInf;
  int bp = -1;
  int stack[kStackDepth];
  T stack_d[kStackDepth];
  int sp = 0;
  int cur = g.root;
  T cur_d = 0;
  for (;;) {
    if (cur_d < best) {
      if (cur < 0) {
        const int code = -1 - cur;
        const int first = code >> 3, cnt = code & 7;
        if constexpr (COUNT) tally->prims += cnt;
        for (int k = 0; k < cnt; ++k) {
          const int pi = first + k;
          T d2;
          if (DIM == 2) {
            T tp;
            d2 = segment_dist2<T>(x, prims + (size_t)pi * kPrimStride2, &tp);
          } else {
            d2 = triangle_dist2<T>(x, prims + (size_t)pi * kPrimStride3);
          }
          if (d2 < best) {
            best = d2;
            bp = pi;
          }
        }
      } else {
        G<BvhNode<T, DIM>>& n = nodes[cur];
        if constexpr (COUNT) ++tally->nodes;
        const T da = box_dist2<T, DIM>(x, n.lo[0], n.hi[0]);
        const T db = box_dist2<T, DIM>(x, n.lo[1], n.hi[1]);
        const int ca = n.child[0], cb = n.child[1];
        const bool a_first = da <= db;
        const int near_c = a_first ? ca : cb, far_c = a_first ? cb : ca;
        const T near_d = a_first ? da : db, far_d = a_first ? db : da;
        if (far_d < best && sp < kStackDepth) {
          stack[sp] = far_c;
          stack_d[sp] = far_d;
          ++sp;
        }
        cur = near_c;
        cur_d = near_d;
        continue;
      }
    }
    if (sp == 0) break;
    --sp;
    cur = stack[sp];
    cur_d = stack_d[sp];
  }
  *best_prim = bp;
  return best;
}

// A polygon grid query returns its candidate list position tagged with kGridPrimTag
// instead of the primitive, so no load waits for the primitive index on every step.
constexpr int kGridPrimTag = 1 << 30;

template <typename T>
__device__ __forceinline__ int resolve_prim(G<DevGeometry<T>>& g, int prim) {
  return (prim >= 0 && (prim & kGridPrimTag)) ? gptr(g.cell_prim)[prim & (kGridPrimTag - 1)] : prim;
}

// ------------------------------------------------------------------ CSG signed distance fields
// (Sec. 7.2: the domain as a list of CSG operations on signed distance fields). The rows
// sit at wave-uniform addresses, so their loads are scalar; each lane evaluates every row.

// Signed distance of one primitive at x; with GRAD also its gradient.
template <typename T, int DIM, bool GRAD>
__device__ __forceinline__ T sdf_shape(const WOS_GLOBAL T* r, const T* x, T* gr) {
  const int shape = (int)r[1];
  T e[DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i) e[i] = x[i] - r[2 + i];
  if (shape == 0) {
    T r2 = 0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) r2 = m_fma(e[i], e[i], r2);
    const T len = m_sqrt(r2);
    if constexpr (GRAD) {
      const T inv = len > (T)0 ? (T)1 / len : (T)0;
#pragma unroll
      for (int i = 0; i < DIM; ++i) gr[i] = len > (T)0 ? e[i] * inv : (i == 0 ? (T)1 : (T)0);
    }
    return len - r[5];
  } else if (shape == 1) {
    // |max(q, 0)| outside, max_i q_i inside, q = |x - c| - h
    T q[DIM], out2 = 0, qmax = -Consts<T>::kInf;
    int amax = 0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      q[i] = fabs(e[i]) - r[5 + i];
      if (q[i] > (T)0) out2 = m_fma(q[i], q[i], out2);
      if (q[i] > qmax) {
        qmax = q[i];
        amax = i;
      }
    }
    if (out2 > (T)0) {
      const T len = m_sqrt(out2);
      if constexpr (GRAD) {
#pragma unroll
        for (int i = 0; i < DIM; ++i) gr[i] = q[i] > (T)0 ? copysign(q[i] / len, e[i]) : (T)0;
      }
      return len;
    }
    if constexpr (GRAD) {
#pragma unroll
      for (int i = 0; i < DIM; ++i) gr[i] = i == amax ? copysign((T)1, e[i]) : (T)0;
    }
    return qmax;
  } else {
    T f = -r[5];
#pragma unroll
    for (int i = 0; i < DIM; ++i) f = m_fma(x[i], r[2 + i], f);
    if constexpr (GRAD) {
#pragma unroll
      for (int i = 0; i < DIM; ++i) gr[i] = r[2 + i];
    }
    return f;
  }
}

// Combined field f of the operation list (from f = +inf: union min, intersection max,
// subtraction max(f, -f_k)); *active = 2 k + (row k entered negated) for the row that
// decides f (the first one on ties).
template <typename T, int DIM>
__device__ __forceinline__ T sdf_value(G<DevGeometry<T>>& g, const T* x, int* active) {
  const WOS_GLOBAL T* rows = gptr(g.prims);
  T f = Consts<T>::kInf;
  int act = 0;
  for (int k = 0; k < g.n_prims; ++k) {
    const WOS_GLOBAL T* r = rows + (size_t)k * kSdfStride;
    const int op = (int)r[0];
    T fk = sdf_shape<T, DIM, false>(r, x, nullptr);
    if (op == 0) {
      if (fk < f) {
        f = fk;
        act = 2 * k;
      }
    } else {
      if (op == 2) fk = -fk;
      if (fk > f) {
        f = fk;
        act = 2 * k + (op == 2 ? 1 : 0);
      }
    }
  }
  *active = act;
  return f;
}

// Distance d from x to the boundary (Alg. 1, first step); prim receives what
// closest_point needs to recover xbar. With BOUND, a polygon or a triangle mesh may
// answer with a certified lower bound of d instead (at least grid_lb_min: a quarter cell
// and twice epsilon) where the truncated list of its grid cell cannot decide the nearest
// primitive
// (points deep inside, where many primitives are nearly equidistant): the ball of that
// radius still lies inside the domain, which is all the walk's step needs, and a walk
// never ends on such a value.
template <typename T, int DIM, int GEOM, bool COUNT = false, bool BOUND = false>
__device__ __forceinline__ T boundary_distance(G<DevGeometry<T>>& g, const T* x, int* prim, Tally* tally = nullptr,
                                               LdsStack<T> lds = LdsStack<T>{nullptr, nullptr, 0, 0}, int hint = -1) {
  if (GEOM == GK_BALL) {
    T r2 = 0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      const T e = x[i] - g.center[i];
      r2 = m_fma(e, e, r2);
    }
    *prim = 0;
    return g.radius - m_sqrt(r2);
  } else if (GEOM == GK_BOX) {
    T d = Consts<T>::kInf;
    int best = 0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      const T dl = x[i] - g.lo[i], dh = g.hi[i] - x[i];
      if (dl < d) { d = dl; best = 2 * i; }
      if (dh < d) { d = dh; best = 2 * i + 1; }
    }
    *prim = best;
    return d;
  } else if (GEOM == GK_SDF) {
    if constexpr (COUNT) tally->prims += g.n_prims;
    return -sdf_value<T, DIM>(g, x, prim);
  } else {
    if constexpr (GEOM == GK_POLYGON) {
      if (g.grid_nx > 0) {
        // candidate grid: scan the list of the cell that contains x
        const T fx = (x[0] - g.grid_lo[0]) * g.grid_inv_h;
        const T fy = (x[1] - g.grid_lo[1]) * g.grid_inv_h;
        if (fx >= (T)0 && fy >= (T)0 && fx < (T)g.grid_nx && fy < (T)g.grid_ny) {
          const int ix = (int)fx, iy = (int)fy;
          const WOS_GLOBAL CellRec<T>* rec = (const WOS_GLOBAL CellRec<T>*)g.cells + (iy * g.grid_nx + ix);
          const uint32_t n = rec->count, st = rec->start;
          if (n > 0) {
            // the inline candidates are tested unconditionally (their loads do not wait
            // for the count); entries past a shorter list repeat its last candidate, which
            // ties and so never replaces it
            T best = Consts<T>::kInf;
            uint32_t bk = 0;
#pragma unroll
            for (int k = 0; k < kCellInline; ++k) {
              const T d2 = segment_dist2_pre<T>(x, rec->seg[k], rec->inv_len2[k]);
              if (d2 < best) {
                best = d2;
                bk = (uint32_t)k;
              }
            }
            uint32_t k = kCellInline;
            T lb = Consts<T>::kInf;
            if (n > (uint32_t)kCellInline) {
              // the rest of the list, nearest to the cell centre first: stop once a
              // candidate's centre distance exceeds |x - centre| + best
              const WOS_GLOBAL T* segs = gptr(g.cell_segs) + (size_t)st * 4;
              const WOS_GLOBAL T* dc = gptr(g.cell_dc) + st;
              const T ox = x[0] - m_fma((T)ix + (T)0.5, g.grid_h, g.grid_lo[0]);
              const T oy = x[1] - m_fma((T)iy + (T)0.5, g.grid_h, g.grid_lo[1]);
              const T r_pc = m_sqrt(m_fma(ox, ox, oy * oy));
              for (; k < n; ++k) {
                const T lim = dc[k] - r_pc;
                if (lim > (T)0 && lim * lim >= best) break;
                T tp;
                const T d2 = segment_dist2<T>(x, segs + (size_t)k * 4, &tp);
                if (d2 < best) {
                  best = d2;
                  bk = k;
                }
              }
              // a truncated list scanned to its end: the segments left off lie at
              // least tail - r_pc from x (complete lists have tail = +inf)
              if (k >= n) lb = rec->tail - r_pc;
            }
            if constexpr (COUNT) {
              ++tally->cells;
              tally->prims += k < n ? k : n;
            }
            const T d = m_sqrt(best);
            if (d <= lb) {
              *prim = kGridPrimTag | (int)(st + bk);   // resolved through cell_prim when needed
              return d;
            }
            if (BOUND && lb >= g.grid_lb_min) {
              *prim = kGridPrimTag | (int)(st + bk);
              return lb;
            }
          }
        }
      }
    }
    if constexpr (GEOM == GK_TRIMESH && DIM == 3) {
      if (g.grid_nx > 0) {
        // candidate grid: scan the list of the cell that contains x, nearest to the cell
        // centre first, until a candidate's centre distance exceeds |x - centre| + best
        T f[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) f[i] = (x[i] - g.grid_lo[i]) * g.grid_inv_h;
        if (f[0] >= (T)0 && f[1] >= (T)0 && f[2] >= (T)0 && f[0] < (T)g.grid_nx && f[1] < (T)g.grid_ny &&
            f[2] < (T)g.grid_nz) {
          const int ix = (int)f[0], iy = (int)f[1], iz = (int)f[2];
          const WOS_GLOBAL MeshCell<T>* rec =
              (const WOS_GLOBAL MeshCell<T>*)g.cells + ((iz * g.grid_ny + iy) * g.grid_nx + ix);
          const uint32_t n = rec->count, st = rec->start;
          const T tail = rec->tail;
          if (n > 0) {
            const WOS_GLOBAL int32_t* cp = gptr(g.cell_prim) + st;
            const WOS_GLOBAL T* dc = gptr(g.cell_dc) + st;
            const WOS_GLOBAL T* prims = gptr(g.prims);
            const T ox = x[0] - m_fma((T)ix + (T)0.5, g.grid_h, g.grid_lo[0]);
            const T oy = x[1] - m_fma((T)iy + (T)0.5, g.grid_h, g.grid_lo[1]);
            const T oz = x[2] - m_fma((T)iz + (T)0.5, g.grid_h, g.grid_lo[2]);
            const T r_pc = m_sqrt(m_fma(ox, ox, m_fma(oy, oy, oz * oz)));
            T best = Consts<T>::kInf;
            int bp = 0;
            uint32_t k = 0;
            for (; k < n; ++k) {
              const T lim = dc[k] - r_pc;
              if (lim > (T)0 && lim * lim >= best) break;
              const int pi = cp[k];
              const T d2 = triangle_dist2<T>(x, prims + (size_t)pi * kPrimStride3);
              if (d2 < best) {
                best = d2;
                bp = pi;
              }
            }
            if constexpr (COUNT) {
              ++tally->cells;
              tally->prims += k;
            }
            // every triangle left off the list lies at least tail - r_pc from x
            const T d = m_sqrt(best);
            const T lb = tail - r_pc;
            if (k < n || d <= lb) {
              *prim = bp;
              return d;
            }
            if (BOUND && lb >= g.grid_lb_min) {
              *prim = bp;
              return lb;
            }
          }
        }
      }
    }
    return m_sqrt(bvh_nearest<T, DIM, COUNT>(g, x, prim, tally, lds, resolve_prim(g, hint)));
  }
}

template <typename T, int DIM, int GEOM>
__device__ __forceinline__ void closest_point(G<DevGeometry<T>>& g, const T* x, int prim, T* xb) {
  prim = resolve_prim(g, prim);
  if (GEOM == GK_BALL) {
    T e[DIM], r2 = 0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      e[i] = x[i] - g.center[i];
      r2 = m_fma(e[i], e[i], r2);
    }
    const T r = m_sqrt(r2);
    const T sc = r > (T)0 ? g.radius / r : (T)0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) xb[i] = g.center[i] + (r > (T)0 ? sc * e[i] : (i == 0 ? g.radius : (T)0));
  } else if (GEOM == GK_BOX) {
    const int ax = prim >> 1;
#pragma unroll
    for (int i = 0; i < DIM; ++i) xb[i] = i == ax ? ((prim & 1) ? g.hi[i] : g.lo[i]) : x[i];
  } else if (GEOM == GK_SDF) {
    // x - f grad f with the deciding row's field; a negated row flips both factors
    T gr[DIM];
    const T fk = sdf_shape<T, DIM, true>(gptr(g.prims) + (size_t)(prim >> 1) * kSdfStride, x, gr);
#pragma unroll
    for (int i = 0; i < DIM; ++i) xb[i] = m_fma(-fk, gr[i], x[i]);
  } else if (DIM == 2) {
    const WOS_GLOBAL T* s = gptr(g.prims) + (size_t)prim * kPrimStride2;
    T t;
    segment_dist2<T>(x, s, &t);
    xb[0] = s[0] + t * (s[2] - s[0]);
    xb[1] = s[1] + t * (s[3] - s[1]);
  } else {
    triangle_closest<T>(x, gptr(g.prims) + (size_t)prim * kPrimStride3, xb);
  }
}

}  // namespace wos
