// Host-side launchers of the kernels in wos_kernels.hip (internal interface).
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>

#include "wos_types.h"

namespace wos {

struct WalkerLaunch {
  int fp64;
  int dim;
  int geom;
  unsigned grid;
  unsigned block;
  const DevItem* items;
  int n_items;
  uint32_t n_tiles;   // tiles of all items
  uint32_t* tile_counter;
  uint64_t* slots;    // accumulation slots, slot_words(grad dim) words each, zeroed before the launch
  int slot_words;
  const LaunchParams* lp;
  uint64_t max_steps;
  int variant;
  int compensated;
  int fp32_draws;     // FP64 walker with the FP32 walker's uniforms
  int rr;
  double ww_lo;
  double ww_hi;       // 0: no splitting
  void* grad;         // gradient records (T[grid lane][1 + 3 dim]) or null
  uint64_t* events;   // non-null selects the event-counting build of the walker
};

hipError_t launch_walker(const WalkerLaunch& L, hipStream_t st);
// The walkers of one precision and dimension (wos_walker_{f32,f64}_{2d,3d}.hip).
hipError_t launch_walker_f32_2d(const WalkerLaunch& L, hipStream_t st);
hipError_t launch_walker_f32_3d(const WalkerLaunch& L, hipStream_t st);
hipError_t launch_walker_f64_2d(const WalkerLaunch& L, hipStream_t st);
hipError_t launch_walker_f64_3d(const WalkerLaunch& L, hipStream_t st);
const void* walker_symbol_f32_2d(int geom, int mode);
const void* walker_symbol_f32_3d(int geom, int mode);
const void* walker_symbol_f64_2d(int geom, int mode);
const void* walker_symbol_f64_3d(int geom, int mode);
// Bytes of the scratch array of wos_solve_static, one copy per GPU.
constexpr size_t kStaticScratchBytes = 128ull << 20;
// Device address of `device`'s copy of that array (looked up on the first call for the
// device, with the device current, and kept).
hipError_t static_scratch(int device, void** ptr);
// 0 delta tracking, 1 delta tracking with splitting or gradient records, 2 next flight
int walker_mode(int variant, bool grad, bool split);
const void* walker_symbol(int fp64, int dim, int geom, int mode);
// Per-point sums of one item from its slots, added into the item's outputs.
hipError_t launch_reduce(int grad_dim, const DevItem& it, const uint64_t* slots, int slot_words, hipStream_t st);
// Zeroes n words at p and the tile counter (a kernel, so that it can sit in a captured graph).
hipError_t launch_clear(uint64_t* p, uint64_t n, uint32_t* counter, hipStream_t st);
hipError_t launch_finalize_components(const double* sum, const double* sum_sq, const uint64_t* nw, int64_t n, int dim,
                                      double* mean, double* se, hipStream_t st);
hipError_t launch_reset(uint32_t* counter, hipStream_t st);
hipError_t launch_set_params(LaunchParams* lp, uint64_t seed, uint64_t walk_offset_add, hipStream_t st);
hipError_t launch_classify(int dim, int geom, const void* P64, const double* pts, int64_t n, int8_t* inside,
                           uint64_t* counters, hipStream_t st);
hipError_t launch_sigma_sample(int dim, int geom, const void* P64, const double* lo, const double* h, int grid,
                               int nblocks, double* out, hipStream_t st);
hipError_t launch_gamma0(int fp64, int dim, const void* P, const double* pts, int64_t n, const int8_t* inside,
                         void* out, hipStream_t st);
hipError_t launch_coefficients(int fp64, int dim, const void* P, const double* pts, int64_t n, double* out,
                               hipStream_t st);
hipError_t launch_distance(int fp64, int dim, int geom, const void* P, const double* pts, int64_t n, double* d,
                           double* xb, hipStream_t st);
hipError_t launch_ball(int fp64, int dim, const double* s, int64_t n, double* out, hipStream_t st);
hipError_t launch_sample(int fp64, int dim, double s, int64_t n, uint64_t seed, double* t, uint64_t* trials,
                         hipStream_t st);
hipError_t launch_philox(const uint32_t* ctr, uint64_t key, int64_t n, uint32_t* out, hipStream_t st);
hipError_t launch_bessel(int fp64, int which, const double* x, int64_t n, double* out, hipStream_t st);
hipError_t launch_offcentred(int fp64, int dim, int which, double R, double sigma_bar, const double* u,
                             const double* v, int64_t n, double* out, hipStream_t st);
hipError_t launch_finalize(const double* sum, const double* sum_sq, const uint64_t* nw, int64_t n, double* mean,
                           double* se, hipStream_t st);

}  // namespace wos
