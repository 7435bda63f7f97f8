// The persistent walker of the walk on spheres (delta tracking, Sec. 5.1 and supplemental
// Alg. 1; next flight, Sec. 5.2 and supplemental Alg. 2): device code, kernel entry points
// and launch templates. Each of wos_walker_{f32,f64}_{2d,3d}.hip includes it and
// instantiates the walkers of one precision and dimension, so that the variants compile in
// parallel.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "wos_device.h"
#include "wos_launch.h"

#ifndef WOS_WAVES_FP32
#define WOS_WAVES_FP32 5
#endif
#ifndef WOS_WAVES_FP64
#define WOS_WAVES_FP64 2
#endif

namespace wos {

// ------------------------------------------------------------------ wave helpers (wave64)

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// ------------------------------------------------------------------ walker
//
// Persistent kernel. Work is a sequence of tiles (a run of walks of one point, or whole
// points; see DevItem); a wavefront takes one tile at a time with a single atomic and hands
// its walks to idle lanes (ballot + mbcnt), so lanes whose walk ends pick up a new walk at
// the next step instead of idling until the longest walk of the wave finishes. A wave only
// switches to a tile of another item (another problem) once all its lanes are idle, so the
// problem, and with it every field table and geometry pointer, stays wave-uniform. A walk
// that ends adds its estimate, its square, its distance queries and its radius proposals
// into the slot of its (tile, point) with integer atomics on exact fixed-point limbs
// (see the slot layout), so the sums do not depend on the order in which walks end.
//
// One walk (Sec. 5.1, supplemental Alg. 1, after the change of variables of Sec. 4.1
// and App. A) keeps
//   x, gamma0 = gamma(x0), Pi = product of the null-event factors (1 - sigma'(y)/sigma_bar),
//   A = running estimate.
// The weight of the recursive estimate after k balls is W_k = Pi e^{gamma(x_k) - gamma0}
// (the e^{gamma} ratios of consecutive steps telescope), so the source estimate of ball k,
// W_k |G| e^{gamma(y) - gamma(x_k)} f(y)/alpha(y), is Pi |G| e^{gamma(y) - gamma0} f(y)/alpha(y)
// and gamma is only needed at y, at the final point, and at exit points when Russian
// roulette must know W.

template <typename T>
struct WalkerArgs {
  const DevItem* items;
  int32_t n_items;
  uint32_t n_tiles;      // tiles of all items
  uint32_t* tile_counter;
  uint64_t* slots;       // accumulation slots (slot_words words each)
  int32_t slot_words;
  const LaunchParams* lp;
  uint64_t max_steps;
  int32_t variant;
  int32_t compensated;
  int32_t fp32_draws;    // FP64 walker: take the FP32 walker's uniforms (delta tracking)
  int32_t rr;
  T ww_lo;
  T ww_hi;               // > 0: expected-value splitting above this weight (delta tracking)
  T* grad;               // [grid lane][GradRecord<DIM>::kStride] or null: gradient records
  uint64_t* events;      // event-counting build only: [kEvents]
};

// Events counted by the event-counting build of the walker (algorithmic work per step).
enum Event {
  EV_STEPS = 0, EV_NODES, EV_PRIMS, EV_TRIALS, EV_TRIALS_FREE, EV_VOLUME, EV_EXIT, EV_TERMINAL,
  EV_GAMMA, EV_WALKS, EV_RR_TESTS, EV_BALL_LARGE_S, EV_CELLS, EV_LANE_ITERS, EV_ACTIVE_LANES, EV_COEF_LANES,
  kEvents
};

constexpr uint32_t kFlagCapped = 1u << 31;
constexpr uint32_t kFlagRR = 1u << 30;
constexpr uint32_t kStepMask = (1u << 30) - 1;

__device__ __forceinline__ const void* uniform_ptr(const void* p) { return (const void*)uniform_u64((uint64_t)p); }

// A walk split by the weight window resumes its pending sibling branches from this state.
constexpr int kSplitDepth = 4;
constexpr uint32_t kMaxBranches = 65535;   // the branch id fills the top half of a counter word

template <typename T, int DIM>
struct SplitEntry {
  T x[DIM];
  T Pi;
  T gx;
  int last_prim;
  uint32_t remaining;
};

// A += term, with the rounding error of the addition carried in Ac when compensated
// (TwoSum: Ac collects (A - (s - b)) + (term - b), b = s - A).
template <typename T>
__device__ __forceinline__ void add_estimate(T& A, T& Ac, T term, int compensated) {
  if (compensated) {
    const T s2 = A + term;
    const T bb = s2 - A;
    Ac += (A - (s2 - bb)) + (term - bb);
    A = s2;
  } else {
    A += term;
  }
}

// Integer add into an accumulation slot in global memory. A slot is written only by the
// wavefront that runs its tile (and read by a later kernel), so the atomic needs no scope
// beyond the work-group: it is performed in the L2 of the wave's own XCD.
struct GlobalAdd {
  __device__ __forceinline__ static void add(uint64_t* w, uint64_t v) {
    __hip_atomic_fetch_add((unsigned long long*)w, (unsigned long long)v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};

// The same into the wave's LDS copy of a slot (see SlotCache).
struct LdsAdd {
  __device__ __forceinline__ static void add(uint64_t* w, uint64_t v) {
    __hip_atomic_fetch_add((unsigned long long*)w, (unsigned long long)v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WAVEFRONT);
  }
};

// Adds u to word w of a slot: of the wave's LDS copy when `cached`, else of the global slot.
__device__ __forceinline__ void slot_word_add(uint64_t* lds, uint64_t* glob, bool cached, int w, uint64_t u) {
  if (cached) LdsAdd::add(lds + w, u);
  else GlobalAdd::add(glob + w, u);
}

// Adds v (finite; below 2^94 in magnitude, the square of an estimate below 2^47) to the
// fixed-point limbs at word `base` of a slot (limb k has weight 2^(32k - 96)).
// v = m 2^(E - 1075) with its 53-bit integer mantissa m, so v 2^96 = m 2^sh, sh = E - 979;
// bits below 2^-96 are dropped (truncation towards zero). m 2^(sh mod 32) spans at most
// 85 bits, i.e. three 32-bit chunks starting at limb sh / 32; a negative v adds the
// negated chunks.
__device__ __forceinline__ void fx_add(uint64_t* lds, uint64_t* glob, bool cached, int base, double v) {
  const uint64_t bits = (uint64_t)__double_as_longlong(v);
  const int e = (int)((bits >> 52) & 0x7FFu);
  uint64_t m = (bits & 0xFFFFFFFFFFFFFull) | (e ? (1ull << 52) : 0ull);
  int sh = (e ? e : 1) - 979;
  if (sh < 0) {
    m = sh > -64 ? m >> -sh : 0ull;
    sh = 0;
  }
  if (m == 0ull) return;
  const int k = base + (sh >> 5), b = sh & 31;
  const uint64_t lo = m << b;
  const uint64_t hi = b ? m >> (64 - b) : 0ull;
  const bool neg = (int64_t)bits < 0;
  const uint64_t c0 = lo & 0xFFFFFFFFull, c1 = lo >> 32, c2 = hi;
  if (c0) slot_word_add(lds, glob, cached, k, neg ? 0ull - c0 : c0);
  if (c1) slot_word_add(lds, glob, cached, k + 1, neg ? 0ull - c1 : c1);
  if (c2 && k + 2 < base + kFxLimbs) slot_word_add(lds, glob, cached, k + 2, neg ? 0ull - c2 : c2);
}

// What a finished walk adds to its slot: the estimate v and v^2, its distance queries and
// flags, and with gradient records (GD = dim) the components of its gradient estimate and
// their squares.
template <int GD>
__device__ __forceinline__ void emit_walk(uint64_t* lds, uint64_t* glob, bool cached, double v, uint32_t steps_flags,
                                          uint32_t step_mask, uint32_t flag_capped, uint32_t flag_rr, const double* g) {
  uint64_t flags = (steps_flags & flag_capped) ? 1ull : 0ull;
  if (steps_flags & flag_rr) flags += 1ull << kFlagShiftKilled;
  bool bad = !(fabs(v) < kFxMaxValue);
#pragma unroll
  for (int c = 0; c < GD; ++c) bad = bad || !(fabs(g[c]) < kFxMaxValue);
  if (bad) {
    flags += 1ull << kFlagShiftBad;
  } else {
    fx_add(lds, glob, cached, kSlotSum, v);
    fx_add(lds, glob, cached, kSlotSumSq, v * v);
#pragma unroll
    for (int c = 0; c < GD; ++c) {
      fx_add(lds, glob, cached, kSlotGrad + 2 * kFxLimbs * c, g[c]);
      fx_add(lds, glob, cached, kSlotGrad + 2 * kFxLimbs * c + kFxLimbs, g[c] * g[c]);
    }
  }
  slot_word_add(lds, glob, cached, kSlotSteps, steps_flags & step_mask);
  if (flags) slot_word_add(lds, glob, cached, kSlotFlags, flags);
}

// A wavefront's cache of accumulation slots in LDS: the slots of the last ENTRIES
// single-point tiles it started. A walk's slot reference is either kCachedSlot | e (entry
// e of the cache) or a global slot index. Walks whose slot is cached add into LDS (cheap
// atomics); the others (tiles of several points) add into global memory. When a new tile
// takes over an entry, the entry is added into its global slot and cleared, and the
// lanes still running walks of the old tile switch their reference to the global slot;
// the rest is added at the end of the kernel. All sums are integers, so the split
// between the two paths does not change any result. Called with every lane active.
constexpr uint32_t kCachedSlot = 0x80000000u;

template <int WORDS, int ENTRIES>
struct SlotCache {
  uint64_t* lds;             // this wave's ENTRIES x WORDS words
  uint32_t tag[ENTRIES];     // global slot held by each entry (~0u: none); wave-uniform
  uint32_t next;             // entry the next single-point tile takes; wave-uniform

  __device__ __forceinline__ void init(uint64_t* base, uint32_t lane) {
    lds = base;
#pragma unroll
    for (int e = 0; e < ENTRIES; ++e) tag[e] = ~0u;
    next = 0;
    for (int w = (int)lane; w < ENTRIES * WORDS; w += 64) lds[w] = 0;
  }
  // Adds entry e (wave-uniform) into its global slot t and clears it.
  __device__ __forceinline__ void flush(int e, uint32_t t, uint64_t* slots, int slot_words, uint32_t lane) {
    if (t == ~0u) return;
    for (int w = (int)lane; w < slot_words; w += 64) {
      const uint64_t v = lds[e * WORDS + w];
      if (v) GlobalAdd::add(slots + (size_t)t * slot_words + w, v);
      lds[e * WORDS + w] = 0;
    }
  }
  // Entry for a new single-point tile with global slot `slot`; returns the reference its
  // walks carry. `ref` is the calling lane's current reference, rewritten if it pointed
  // into the entry taken over.
  __device__ __forceinline__ uint32_t take(uint32_t slot, uint64_t* slots, int slot_words, uint32_t lane,
                                           uint32_t& ref) {
    const int e = (int)next;
    uint32_t t = ~0u;
#pragma unroll
    for (int c = 0; c < ENTRIES; ++c)
      if (c == e) t = tag[c];
    flush(e, t, slots, slot_words, lane);
    if (ref == (kCachedSlot | (uint32_t)e)) ref = t;
#pragma unroll
    for (int c = 0; c < ENTRIES; ++c)
      if (c == e) tag[c] = slot;
    next = next + 1 == (uint32_t)ENTRIES ? 0u : next + 1;
    return kCachedSlot | (uint32_t)e;
  }
  __device__ __forceinline__ void flush_all(uint64_t* slots, int slot_words, uint32_t lane) {
#pragma unroll
    for (int e = 0; e < ENTRIES; ++e) flush(e, tag[e], slots, slot_words, lane);
  }
  // Adds a finished walk into the slot it references.
  template <int GD>
  __device__ __forceinline__ void emit(uint32_t ref, uint64_t* slots, int slot_words, double v, uint32_t steps_flags,
                                       uint32_t step_mask, uint32_t flag_capped, uint32_t flag_rr, const double* g) {
    const bool cached = (ref & kCachedSlot) != 0u;
    emit_walk<GD>(lds + (ref & (uint32_t)(ENTRIES - 1)) * WORDS, slots + (size_t)(cached ? 0u : ref) * slot_words,
                  cached, v, steps_flags, step_mask, flag_capped, flag_rr, g);
  }
};

// A wavefront's queue of finished walks in LDS: estimate, distance queries with flags, and
// slot reference. Lanes whose walk ended append their result (ballot + mbcnt, one LDS
// store each); the whole wave adds the queued results into their slots, one per lane,
// when the queue cannot take an iteration's walks, before a new single-point tile takes
// over a slot-cache entry (queued references must still be valid), and at the end. The
// integer adds then run on up to 64 lanes at once instead of inside the divergent branch
// of the few lanes that ended, which would hold up the whole wave at almost every
// iteration. Called with every lane active.
template <int CAP>
struct EmitQueue {
  double* v;       // [CAP] estimates
  uint2* meta;     // [CAP] (steps | flags, slot reference)
  uint32_t n;      // queued entries; wave-uniform

  __device__ __forceinline__ void init(double* vb, uint2* mb) {
    v = vb;
    meta = mb;
    n = 0;
  }
  template <int WORDS, int ENTRIES>
  __device__ __forceinline__ void drain(SlotCache<WORDS, ENTRIES>& cache, uint64_t* slots, int slot_words,
                                        uint32_t lane) {
    if (n == 0) return;
    // entries were written by other lanes of this wave: keep the compiler from moving
    // the reads above those LDS stores (the wave's LDS operations run in order)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (lane < n) {
      const double val = v[lane];
      const uint2 m = meta[lane];
      cache.template emit<0>(m.y, slots, slot_words, val, m.x, kStepMask, kFlagCapped, kFlagRR, nullptr);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    n = 0;
  }
  // Appends the results of the lanes in `fin` (the calling lane's if `mine`), draining
  // first if they do not fit.
  template <int WORDS, int ENTRIES>
  __device__ __forceinline__ void push(uint64_t fin, bool mine, double val, uint32_t steps_flags, uint32_t ref,
                                       SlotCache<WORDS, ENTRIES>& cache, uint64_t* slots, int slot_words,
                                       uint32_t lane) {
    const uint32_t nf = (uint32_t)__popcll(fin);
    if (n + nf > (uint32_t)CAP) drain(cache, slots, slot_words, lane);
    if (mine) {
      const uint32_t r = n + lanes_below(fin);
      v[r] = val;
      meta[r] = make_uint2(steps_flags, ref);
    }
    n += nf;
  }
};

// Radius proposals (next flight: inner points) drawn by the wave's lanes for the current
// item, added to the item's counter [3] when the wave leaves the item (all lanes idle) and
// at the end; with the event-counting build also to the wave's event tally.
__device__ __forceinline__ void flush_trials(uint64_t* counters, uint32_t& ntrials, uint32_t* ev_trials) {
  uint64_t t = ntrials;
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
  if (counters && __lane_id() == 0 && t) atomicAdd((unsigned long long*)&counters[3], (unsigned long long)t);
  if (ev_trials) *ev_trials += ntrials;
  ntrials = 0;
}

// Buffers written by the walker are separate __restrict__ parameters, so loads of the
// problem tables (read-only, at wave-uniform addresses) can be served by scalar loads.
// MODE: 0 delta tracking, 1 delta tracking with the extras that cost registers (weight-window
// splitting, gradient records), 2 next flight.
template <typename T, int DIM, int GEOM, bool COUNT, int MODE>
__device__ __forceinline__ void walker_body(WalkerArgs<T> a, uint32_t* __restrict__ tile_counter,
                                            uint64_t* __restrict__ slots, uint64_t* __restrict__ events_out) {
  using SL = Slots<T, DIM>;
  constexpr bool NF = MODE == 2;
  constexpr bool EXTRA = MODE == 1;
  const uint32_t lane = __lane_id();
  constexpr int kStack = GEOM == GK_POLYGON ? kLdsStackDepthPolygon : kLdsStackDepth;
  LdsStack<T> lds_stack{nullptr, nullptr, 0, 0};
  if constexpr (GEOM == GK_POLYGON || GEOM == GK_TRIMESH) {
    __shared__ int32_t s_node[kStack * 256];
    __shared__ T s_dist[kStack * 256];
    lds_stack = LdsStack<T>{s_node + threadIdx.x, s_dist + threadIdx.x, (int)blockDim.x, kStack};
  }
  // LDS cache of accumulation slots: gradient slots are larger, so fewer entries
  constexpr int kCacheWords = EXTRA ? 64 : 16;
  constexpr int kCacheEntries = EXTRA ? 2 : 4;
  __shared__ uint64_t s_slot_cache[4 * kCacheEntries * kCacheWords];
  SlotCache<kCacheWords, kCacheEntries> cache;
  cache.init(s_slot_cache + uniform_int((int)(threadIdx.x >> 6)) * (kCacheEntries * kCacheWords), lane);
  // queue of finished walks (not with gradient records, whose results come from a
  // per-lane record; not for meshes, whose LDS stacks leave no room at five blocks per CU)
  constexpr bool kQueue = MODE != 1 && GEOM != GK_TRIMESH;
  constexpr int kQueueCap = 64;
  __shared__ double s_queue_v[kQueue ? 4 * kQueueCap : 1];
  __shared__ uint2 s_queue_m[kQueue ? 4 * kQueueCap : 1];
  EmitQueue<kQueueCap> queue;
  if constexpr (kQueue) {
    const int w = uniform_int((int)(threadIdx.x >> 6));
    queue.init(s_queue_v + w * kQueueCap, s_queue_m + w * kQueueCap);
  }
  Tally tally = {0, 0, 0, 0};
  uint32_t ev[kEvents];
  if constexpr (COUNT) {
    for (int e = 0; e < kEvents; ++e) ev[e] = 0;
  }
  const uint64_t seed = a.lp->seed;
  const uint64_t offset_add = a.lp->walk_offset_add;
  const WOS_GLOBAL DevItem* items = gptr(a.items);
  // ---- wave-uniform scheduling state: the current item, the tile being handed out
  // (walks res_next .. res_end - 1 of it: point tl_p0 + (tl_j0 + r) / walks), the next
  // claimed tile, and the item searched for it (tiles are claimed in increasing order)
  int cur_item = -1, search_item = 0;
  uint32_t res_next = 0, res_end = 0;
  uint32_t tl_p0 = 0, tl_j0 = 0, tl_slot0 = 0, tl_walks = 1, tl_single = 1;
  int64_t pend_tile = -1;
  bool queue_done = false;
  const WOS_GLOBAL DevProblem<T>* Pp = nullptr;
  // ---- lane state: phase 0 = idle, 1 = new walk whose gamma(x0) and its gradient are still
  // to be evaluated (gradient records only), 2 = walking (3: next flight inside a ball),
  // 4 = ended, its result still to be added; slot: accumulation slot of the walk
  int phase = 0;
  uint32_t slot = 0;
  T* const grad_rec = EXTRA && a.grad ? a.grad + ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * GradRecord<DIM>::kStride
                                     : nullptr;
  T x[DIM];
  T gamma0 = 0, gx = 0;
  bool gx_known = false;
  T Pi = 1, A = 0, Ac = 0;
  uint32_t nsteps = 0, ntrials = 0;
  int last_prim = -1;   // closest primitive of the previous step (bounds the next query)
  Rng rng;
  rng.set_key(seed);
  // next flight (phase 3 = inside the unrolled series of a ball): exit point z and current
  // inner point, both relative to the ball centre x; the series T and S of the ball, the
  // throughput, the ball radius and its 2D kernel constant. Pi holds prod_k T_k.
  T zr[DIM], xc[DIM];
  T nf_T = 0, nf_S = 0, nf_beta = 1, nf_R = 0, nf_c = 0;
  // delta tracking: the current ball while its radius is being drawn (pending: the last
  // proposal was rejected and the lane retries at the next iteration)
  T bR = 0, bs = 0;
  Ball<T, DIM> bb;
  bb.pb = 0;
  bb.gnorm = 0;
  bb.c2d = 0;
  bool pending = false;
  uint32_t ntry = 0;
  // weight window, high side: pending sibling branches (private memory, touched only on
  // splits), branches started by the walk so far, flags of all its branches
  // (split_state: stack depth in the low 8 bits, branches in the rest; the flags of
  // finished branches are kept in the top bits of nsteps)
  SplitEntry<T, DIM> split_stack[kSplitDepth];
  uint32_t split_state = 0;
  const bool window = a.rr || (EXTRA && a.ww_hi > (T)0);

  for (;;) {
    // ---------------------------------------------------------------- finished walks
    // A walk that ended in the last iteration adds its estimate A + Ac, its square, its
    // distance queries and flags (in nsteps) to its slot here, where little else is live.
    if constexpr (kQueue) {
      const uint64_t fin = __ballot(phase == 4);
      if (fin) {
        queue.push(fin, phase == 4, (double)A + (double)Ac, nsteps, slot, cache, slots, a.slot_words, lane);
        if (phase == 4) phase = 0;
      }
    } else if (phase == 4) {
      const double v = (double)A + (double)Ac;
      if (EXTRA && a.grad) {
        // per-walk gradient estimate (supplemental Sec. 2):
        // A0 a + (A - A0) b - A grad gamma(x0), from the lane's record
        double g[DIM];
        const T* gr = grad_rec;
        const double a0 = (double)gr[0];
#pragma unroll
        for (int c = 0; c < DIM; ++c)
          g[c] = a0 * (double)gr[1 + c] + (v - a0) * (double)gr[1 + DIM + c] - v * (double)gr[1 + 2 * DIM + c];
        cache.template emit<DIM>(slot, slots, a.slot_words, v, nsteps, kStepMask, kFlagCapped, kFlagRR, g);
      } else {
        cache.template emit<0>(slot, slots, a.slot_words, v, nsteps, kStepMask, kFlagCapped, kFlagRR, nullptr);
      }
      phase = 0;
    }
    // ---------------------------------------------------------------- refill idle lanes
    uint64_t idle = __ballot(phase == 0);
    while (idle != 0) {
      if (res_next >= res_end) {
        if (pend_tile < 0) {
          if (queue_done) break;
          // every lane is active here, so the first active lane is lane 0
          uint32_t t = 0;
          if (lane == 0) t = atomicAdd(tile_counter, 1u);
          t = __builtin_amdgcn_readfirstlane(t);
          if (t >= a.n_tiles) {
            queue_done = true;
            break;
          }
          pend_tile = (int64_t)t;
          while (pend_tile >= (int64_t)(items[search_item].tile_base + items[search_item].n_tiles))
            search_item = uniform_int(search_item + 1);
        }
        if (search_item != cur_item) {
          if (idle != ~0ull) break;  // drain the wave before switching problems
          if (cur_item >= 0) flush_trials(items[cur_item].counters, ntrials, COUNT ? &ev[EV_TRIALS] : nullptr);
          cur_item = uniform_int(search_item);
          Pp = (const WOS_GLOBAL DevProblem<T>*)uniform_ptr(items[cur_item].problem);
        }
        // the tile's walks, from the item's regular cut (DevItem)
        G<DevItem>& it = items[cur_item];
        const uint64_t tl = (uint64_t)pend_tile - it.tile_base;
        const uint32_t walks = (uint32_t)it.walks;
        if (it.tiles_per_point > 0u) {
          const uint32_t tpp = it.tiles_per_point;
          const uint32_t p0 = (uint32_t)(tl / tpp);
          const uint32_t j0 = (uint32_t)(tl - (uint64_t)p0 * tpp) * it.tile_len;
          tl_p0 = uniform_int((int)p0);
          tl_j0 = uniform_int((int)j0);
          res_end = uniform_int((int)min(it.tile_len, walks - j0));
          tl_single = 1;
        } else {
          const uint32_t p0 = (uint32_t)tl * it.points_per_tile;
          const uint32_t np = (uint32_t)min((int64_t)it.points_per_tile, it.n_points - (int64_t)p0);
          tl_p0 = uniform_int((int)p0);
          tl_j0 = 0;
          res_end = uniform_int((int)(np * walks));
          tl_single = 0;
        }
        tl_slot0 = uniform_int((int)(it.slot_base + (it.tiles_per_point > 0u ? tl : (uint64_t)tl_p0)));
        tl_walks = uniform_int((int)walks);
        if (tl_single) {
          if constexpr (kQueue) queue.drain(cache, slots, a.slot_words, lane);
          tl_slot0 = uniform_int((int)cache.take(tl_slot0, slots, a.slot_words, lane, slot));
        }
        res_next = 0;
        pend_tile = -1;
      }
      const uint32_t n_idle = __popcll(idle);
      const uint32_t avail = res_end - res_next;
      const uint32_t take = avail < n_idle ? avail : n_idle;
      const uint32_t rank = lanes_below(idle);
      if (phase == 0 && rank < take) {
        // new walk: set-up only; gamma(x0) comes from the per-point table, or for gradient
        // records is evaluated with the other lanes' step
        G<DevItem>& it = items[cur_item];
        const uint32_t r = res_next + rank;
        uint32_t p, j;
        if (tl_single) {
          p = tl_p0;
          j = tl_j0 + r;
          slot = tl_slot0;
        } else {
          const uint32_t dq = r / tl_walks;
          p = tl_p0 + dq;
          j = r - dq * tl_walks;
          slot = tl_slot0 + dq;
        }
        nsteps = 0;
        if (gptr(it.inside)[p]) {
#pragma unroll
          for (int i = 0; i < DIM; ++i) x[i] = (T)gptr(it.points)[(size_t)p * DIM + i];
          rng.init((uint32_t)(it.walk_offset + offset_add + j), p, it.problem_index);
          Pi = 1;
          A = 0;
          Ac = 0;
          last_prim = -1;
          pending = false;
          split_state = 0;
          if (EXTRA && a.grad) {
            phase = 1;   // gamma(x0) with its gradient, for the gradient record
            if constexpr (COUNT) ++ev[EV_GAMMA];
          } else {
            gamma0 = gptr((const WOS_GLOBAL T*)it.gamma0)[p];
            gx = gamma0;
            gx_known = true;
            phase = 2;
          }
          if constexpr (COUNT) ++ev[EV_WALKS];
        }
        // a point outside the domain runs no walk; the reduction marks its sums
      }
      res_next += take;
      idle = __ballot(phase == 0);
    }
    if (__ballot(phase != 0) == 0) {
      if (queue_done) break;
      continue;
    }
    // ---------------------------------------------------------------- one step
    // Every active lane evaluates the coefficients at no more than one point per iteration:
    // x0 for a new walk with gradient records, the current point for a walk that ends in the
    // epsilon shell, and the sampled point y otherwise (none while a radius proposal is
    // being retried), so the most expensive part runs in lockstep.
    if constexpr (COUNT) {
      ++ev[EV_LANE_ITERS];
      if (phase != 0) ++ev[EV_ACTIVE_LANES];
    }
    if (phase != 0) {
      G<DevProblem<T>>& P = *Pp;
      if constexpr (NF) {
        // ------------------------------------------------ next flight (Sec. 5.2, Alg. 2)
        // A ball samples its exit point z once; the recursion inside the ball is unrolled
        // into the series T (boundary) and S (source) over uniform inner points x^j, with
        // roulette on the throughput prod theta_l, theta_l = G(x^l, x^{l+1}) (sigma_bar -
        // sigma'(x^{l+1})) |B|. The source term f'(x^j)/(sigma_bar - sigma'(x^j)) times the
        // throughput is taken as f'(x^j) G |B| times the throughput before theta_{j-1}, so
        // sigma' = sigma_bar needs no division. U(x_k) ~ T U(z) + S; Pi = prod T.
        bool done = false, terminal = false, sample = false;
        uint32_t flag = 0;
        T gb = 0;
        T q[DIM], xn[DIM];
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
          q[i] = x[i];
          xn[i] = 0;
        }
        if (phase >= 2) rng.refill<SL::kNfBlocks>();
        if (phase == 3) {
          const NfBall<T, DIM> nb = nf_ball<T, DIM>(nf_R, P.sqrt_sigma_bar, nf_c);
          nf_T = m_fma(nf_poisson_area<T, DIM>(nb, xc, zr), nf_beta, nf_T);
          const T prr = fmin((T)1, nf_beta);
          if (uniform01<T, SL::kNfRoulette>(rng) <= prr) {
            nf_beta /= prr;
            sample = true;
          } else {
            add_estimate(A, Ac, Pi * nf_S, a.compensated);
            Pi *= nf_T;
#pragma unroll
            for (int i = 0; i < DIM; ++i) x[i] += zr[i];
            phase = 2;
          }
        }
        if (phase == 2 && !sample) {
          if constexpr (COUNT) ++ev[EV_STEPS];
          if (nsteps >= a.max_steps) {
            done = true;
            flag = kFlagCapped;
          } else {
            int prim;
            const T d = boundary_distance<T, DIM, GEOM, COUNT, true>(P.geom, x, &prim, &tally, lds_stack, last_prim);
            last_prim = prim;
            ++nsteps;
            if (!(d == d)) {
              done = true;
              flag = kFlagCapped;
            } else if (d < P.epsilon) {
              T xb[DIM];
              closest_point<T, DIM, GEOM>(P.geom, x, prim, xb);
              gb = boundary_value<T, DIM>(P, xb);
              terminal = true;
              if constexpr (COUNT) {
                ++ev[EV_TERMINAL];
                ++ev[EV_GAMMA];
              }
            } else {
              const bool harmonic = !(P.sigma_bar > (T)0);
              const Ball<T, DIM> b = ball_terms<T, DIM>(d, d * P.sqrt_sigma_bar, P.inv_sigma_bar, harmonic);
              nf_R = d;
              nf_c = b.c2d;
              nf_T = (T)1 - b.pb;     // P(x, z) |dB| at the centre
              nf_S = 0;
              nf_beta = 1;            // the first inner point is always taken
              T v[DIM];
              uniform_direction<T, DIM, SL::kNfExitDir>(rng, v);
#pragma unroll
              for (int i = 0; i < DIM; ++i) {
                zr[i] = d * v[i];
                xc[i] = 0;
              }
              sample = true;
            }
          }
        }
        if (sample) {
          uniform_in_ball<T, DIM, SL::kNfInner>(rng, nf_R, xn);
#pragma unroll
          for (int i = 0; i < DIM; ++i) q[i] = x[i] + xn[i];
        }
        PointCoef<T> cq;
        cq.gamma = 0;
        cq.sigma_prime = 0;
        cq.f_over_alpha = 0;
        cq.alpha = 1;
        if (phase == 1 || terminal || sample) {
          cq = point_coef<T, DIM, true>(P, q);
          if constexpr (COUNT) ++ev[EV_COEF_LANES];
        }
        if (phase == 1) {
          gamma0 = cq.gamma;
          phase = 2;
        } else if (terminal) {
          add_estimate(A, Ac, Pi * m_exp(cq.gamma - gamma0) * gb, a.compensated);
          done = true;
        } else if (sample) {
          const NfBall<T, DIM> nb = nf_ball<T, DIM>(nf_R, P.sqrt_sigma_bar, nf_c);
          const T gv = nf_green_vol<T, DIM>(nb, xc, xn);
          nf_S = m_fma(nf_beta * gv, m_exp(cq.gamma - gamma0) * cq.f_over_alpha, nf_S);
          nf_beta *= gv * (P.sigma_bar - cq.sigma_prime);
#pragma unroll
          for (int i = 0; i < DIM; ++i) xc[i] = xn[i];
          ++ntrials;
          phase = 3;
        }
        if (done) {
          nsteps = (nsteps & kStepMask) | flag;
          phase = 4;   // added to its slot at the top of the next iteration
        }
      } else {
        bool done = false, terminal = false, sampled = false;
        uint32_t flag = 0;
        T q[DIM];
  #pragma unroll
        for (int i = 0; i < DIM; ++i) q[i] = x[i];
        T gb = 0;
        if (phase == 2) {
          // the roulette slot's block only where a weight window can use it
          if (sizeof(T) == 8 && a.fp32_draws) {
            if (window) refill_fp32_draws<DIM, Slots<float, DIM>::kBlocks>(rng);
            else refill_fp32_draws<DIM, Slots<float, DIM>::kBlocksPlain>(rng);
          } else if (window) {
            rng.refill<SL::kBlocks>();
          } else {
            rng.refill<SL::kBlocksPlain>();
          }
        }
        if (phase == 2 && !pending) {
          if constexpr (COUNT) ++ev[EV_STEPS];
          if ((nsteps & kStepMask) >= a.max_steps) {
            done = true;
            flag = kFlagCapped;
          } else {
            int prim;
            const T d = boundary_distance<T, DIM, GEOM, COUNT, true>(P.geom, x, &prim, &tally, lds_stack, last_prim);
            last_prim = prim;
            ++nsteps;
            if (!(d == d)) {
              // a non-finite position cannot continue; report the walk as cut
              done = true;
              flag = kFlagCapped;
            } else if (d < P.epsilon) {
              // epsilon shell: the walk returns g(xbar) (Alg. 1) times its weight, which
              // needs gamma at the current point
              T xb[DIM];
              closest_point<T, DIM, GEOM>(P.geom, x, prim, xb);
              gb = boundary_value<T, DIM>(P, xb);
              terminal = true;
              if constexpr (COUNT) {
                ++ev[EV_TERMINAL];
                if (!gx_known) ++ev[EV_GAMMA];
              }
            } else {
              // a new ball and its normalisation; the radius is drawn below, one proposal
              // per iteration, and the direction of y once a radius is accepted (it is
              // independent of the radius, so no direction is kept across retries)
              bR = d;
              bs = d * P.sqrt_sigma_bar;
              bb = ball_terms<T, DIM>(d, bs, P.inv_sigma_bar, !(P.sigma_bar > (T)0));
              if constexpr (COUNT) {
                if (bs >= (DIM == 2 ? (T)2 : (T)1)) ++ev[EV_BALL_LARGE_S];
              }
              pending = true;
              ntry = 0;
            }
          }
        }
        if (pending) {
          ++ntrials;
          const T t = radius_trial<T, DIM, SL::kTrial, COUNT>(rng, bs, bb, !(P.sigma_bar > (T)0), &tally);
          if (t >= (T)0) {
            T bv[DIM];
            uniform_direction<T, DIM, SL::kDir>(rng, bv);
  #pragma unroll
            for (int i = 0; i < DIM; ++i) q[i] = m_fma(t * bR, bv[i], x[i]);
            sampled = true;
            pending = false;
          } else if (++ntry >= kMaxTrials) {  // only for a non-finite s: cut the walk
            done = true;
            flag = kFlagCapped;
            pending = false;
          }
        }
        const T R = bR;
        const Ball<T, DIM>& b = bb;
        const bool evaluate = phase == 1 || terminal || sampled;
        PointCoef<T> cq;
        cq.gamma = 0;
        cq.sigma_prime = 0;
        cq.f_over_alpha = 0;
        cq.alpha = 1;
        T ggx[DIM];
        if (evaluate) {
          cq = point_coef<T, DIM, true>(P, q, EXTRA && a.grad ? ggx : nullptr);
          if constexpr (COUNT) ++ev[EV_COEF_LANES];
        }
        // weight of a term at the evaluated point, Pi e^{gamma(q) - gamma(x0)} (the boundary
        // value of a walk in the shell, the source at a sampled point), formed once for both
        const T pe = Pi * m_exp(cq.gamma - gamma0);
        if (phase == 1) {
          gamma0 = cq.gamma;
          gx = gamma0;
          gx_known = true;
          phase = 2;
          if (EXTRA && a.grad) {
            // gradient record of the walk: grad gamma(x0) now, the first ball's terms
            // when it is sampled (they stay zero for a walk that starts in the shell)
            T* gr = grad_rec;
            gr[0] = 0;
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
              gr[1 + i] = 0;
              gr[1 + DIM + i] = 0;
              gr[1 + 2 * DIM + i] = ggx[i];
            }
          }
        } else if (terminal) {
          add_estimate(A, Ac, pe * gb, a.compensated);
          done = true;
        } else if (sampled) {
          const T mu = uniform01<T, SL::kMu>(rng);
          const bool volume = mu <= b.pb;
          const T src = pe * cq.f_over_alpha;
          T term = 0;
          // |G| = P_B / sigma_bar (R^2 / 2n when sigma_bar = 0) is formed here rather than
          // kept from the ball's first iteration, which saves a register across retries
          const T gnorm = P.sigma_bar > (T)0 ? b.pb * P.inv_sigma_bar : R * R * (T)(DIM == 2 ? 0.25 : 1.0 / 6.0);
          if (a.variant == 0) term = gnorm * src;
          else if (volume) term = src * P.inv_sigma_bar;
          add_estimate(A, Ac, term, a.compensated);
          if constexpr (COUNT) ++ev[volume ? EV_VOLUME : EV_EXIT];
          if (EXTRA && a.grad && (nsteps & kStepMask) == 1u && (split_state >> 8) == 0u) {
            // first ball (supplemental Sec. 2): A0 = its source term, a = grad G/G at y,
            // b = a after a volume event or grad P/P at the exit point z
            T* gr = grad_rec;
            T w[DIM], r2 = 0;
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
              w[i] = q[i] - x[i];
              r2 = m_fma(w[i], w[i], r2);
            }
            const T fg = grad_ratio_green<T, DIM>(m_sqrt(r2), R, P.sqrt_sigma_bar);
            const T fp = grad_ratio_poisson<T, DIM>(R, P.sqrt_sigma_bar);
            T vz[DIM];
            uniform_direction<T, DIM, SL::kExitDir>(rng, vz);   // the exit direction drawn below
            gr[0] = term;
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
              gr[1 + i] = fg * w[i];
              gr[1 + DIM + i] = volume ? fg * w[i] : fp * R * vz[i];
            }
          }
          if (volume) {
            // null event: weight (1 - sigma'(y)/sigma_bar) e^{gamma(y) - gamma(x)}, move to y
            Pi *= (T)1 - cq.sigma_prime * P.inv_sigma_bar;
  #pragma unroll
            for (int i = 0; i < DIM; ++i) x[i] = q[i];
            gx = cq.gamma;
            gx_known = true;
          } else {
            // boundary term: uniform point on the sphere, weight e^{gamma(z) - gamma(x)}
            T vz[DIM];
            uniform_direction<T, DIM, SL::kExitDir>(rng, vz);
  #pragma unroll
            for (int i = 0; i < DIM; ++i) x[i] = m_fma(R, vz[i], x[i]);
            gx_known = false;
            if (window) {
              gx = point_gamma<T, DIM>(P, x);
              gx_known = true;
              if constexpr (COUNT) ++ev[EV_GAMMA];
            }
          }
          if (window) {
            // static weight window (Sec. 6) on W = Pi e^{gamma(x) - gamma0}
            const T e = m_exp(gx - gamma0);
            const T W = Pi * e;
            if (a.rr && m_fabs(W) < a.ww_lo) {
              // low side: survive with probability |W|/w-
              if constexpr (COUNT) ++ev[EV_RR_TESTS];
              const T u = uniform01<T, SL::kRoulette>(rng);
              if (u * a.ww_lo <= m_fabs(W)) {
                Pi = (W < (T)0 ? -a.ww_lo : a.ww_lo) / e;
              } else {
                done = true;
                flag = kFlagRR;
              }
            } else if (EXTRA && a.ww_hi > (T)0 && m_fabs(W) > a.ww_hi && (split_state >> 8) < kMaxBranches &&
                       (split_state & 0xFFu) < (uint32_t)kSplitDepth) {
              // high side: expected-value splitting into N branches of weight W/m,
              // m = |W|/w+, N = floor(m) with probability floor(m) + 1 - m, else
              // floor(m) + 1 (E[N] = m); N - 1 siblings wait on the lane's stack. The
              // decision is taken only when the stack has room: every outcome, N = 1
              // included, takes the weight W/m, so a walk whose stack is full must skip the
              // split altogether and go on at weight W (unbiased either way)
              const T m = m_fabs(W) / a.ww_hi;
              const T fl = floor(m);
              const uint32_t N = uniform01<T, SL::kRoulette>(rng) <= fl + (T)1 - m ? (uint32_t)fl : (uint32_t)fl + 1u;
              Pi /= m;
              if (N > 1u) {
                SplitEntry<T, DIM>& se = split_stack[split_state & 0xFFu];
                ++split_state;
#pragma unroll
                for (int i = 0; i < DIM; ++i) se.x[i] = x[i];
                se.Pi = Pi;
                se.gx = gx;
                se.last_prim = last_prim;
                se.remaining = N - 1u;
              }
            }
          }
        }
        if (done) {
          nsteps |= flag;
          if (EXTRA && (split_state & 0xFFu)) {
            // the walk goes on as the next sibling branch of the latest split, from the
            // split's state, with a stream of its own
            SplitEntry<T, DIM>& se = split_stack[(split_state & 0xFFu) - 1u];
#pragma unroll
            for (int i = 0; i < DIM; ++i) x[i] = se.x[i];
            Pi = se.Pi;
            gx = se.gx;
            gx_known = true;
            last_prim = se.last_prim;
            if (--se.remaining == 0u) --split_state;
            split_state += 1u << 8;
            rng.init(rng.walk, rng.point, (rng.problem & 0xFFFFu) | ((split_state >> 8) << 16));
            pending = false;
          } else {
            phase = 4;   // added to its slot at the top of the next iteration
          }
        }
      }
    }
  }
  if (cur_item >= 0) flush_trials(items[cur_item].counters, ntrials, COUNT ? &ev[EV_TRIALS] : nullptr);
  if constexpr (kQueue) queue.drain(cache, slots, a.slot_words, lane);
  cache.flush_all(slots, a.slot_words, lane);
  if constexpr (COUNT) {
    ev[EV_NODES] = tally.nodes;
    ev[EV_PRIMS] = tally.prims;
    ev[EV_TRIALS_FREE] = tally.trials_free;
    ev[EV_CELLS] = tally.cells;
    for (int e = 0; e < kEvents; ++e) {
      uint64_t val = ev[e];
      for (int off = 32; off > 0; off >>= 1) val += __shfl_xor(val, off);
      if (lane == 0 && val) atomicAdd((unsigned long long*)&events_out[e], (unsigned long long)val);
    }
  }
}

// Kernel entry points, one per precision so that each gets its own register budget: the
// FP32 walker fits 96 VGPRs (5 waves per SIMD); the FP64 walker needs more than 256
// unless asked to fit 256 (2 waves per SIMD).
template <int DIM, int GEOM, bool COUNT, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WOS_WAVES_FP32)))
walker_kernel_fp32(WalkerArgs<float> a, uint32_t* __restrict__ tile_counter, uint64_t* __restrict__ slots,
                   uint64_t* __restrict__ events_out) {
  walker_body<float, DIM, GEOM, COUNT, MODE>(a, tile_counter, slots, events_out);
}

template <int DIM, int GEOM, bool COUNT, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WOS_WAVES_FP64)))
walker_kernel_fp64(WalkerArgs<double> a, uint32_t* __restrict__ tile_counter, uint64_t* __restrict__ slots,
                   uint64_t* __restrict__ events_out) {
  walker_body<double, DIM, GEOM, COUNT, MODE>(a, tile_counter, slots, events_out);
}

// ------------------------------------------------------------------ launch templates

template <typename T, int DIM, int GEOM, bool COUNT, int MODE>
static const void* walker_entry() {
  if constexpr (sizeof(T) == 4) return (const void*)&walker_kernel_fp32<DIM, GEOM, COUNT, MODE>;
  else return (const void*)&walker_kernel_fp64<DIM, GEOM, COUNT, MODE>;
}

template <typename T, int DIM, int GEOM, bool COUNT, int MODE>
static void launch_walker_k(dim3 g, dim3 b, hipStream_t st, const WalkerArgs<T>& a, uint32_t* counter,
                            uint64_t* slots, uint64_t* events) {
  if constexpr (sizeof(T) == 4)
    hipLaunchKernelGGL((walker_kernel_fp32<DIM, GEOM, COUNT, MODE>), g, b, 0, st, a, counter, slots, events);
  else
    hipLaunchKernelGGL((walker_kernel_fp64<DIM, GEOM, COUNT, MODE>), g, b, 0, st, a, counter, slots, events);
}

template <typename T, int DIM, int GEOM>
static hipError_t launch_walker_t(const WalkerLaunch& L, hipStream_t st) {
  WalkerArgs<T> a;
  a.items = L.items;
  a.n_items = L.n_items;
  a.n_tiles = L.n_tiles;
  a.tile_counter = L.tile_counter;
  a.slots = L.slots;
  a.slot_words = L.slot_words;
  a.lp = L.lp;
  a.max_steps = L.max_steps;
  a.variant = L.variant;
  a.compensated = L.compensated;
  a.fp32_draws = L.fp32_draws;
  a.rr = L.rr;
  a.ww_lo = (T)L.ww_lo;
  a.ww_hi = (T)L.ww_hi;
  a.grad = (T*)L.grad;
  a.events = L.events;
  const dim3 g(L.grid), b(L.block);
  uint64_t* ev = L.events;
  const int mode = walker_mode(L.variant, L.grad != nullptr, L.ww_hi > 0);
  if (mode == 2) {
    if (ev) launch_walker_k<T, DIM, GEOM, true, 2>(g, b, st, a, L.tile_counter, L.slots, ev);
    else launch_walker_k<T, DIM, GEOM, false, 2>(g, b, st, a, L.tile_counter, L.slots, ev);
  } else if (mode == 1) {
    if (ev) launch_walker_k<T, DIM, GEOM, true, 1>(g, b, st, a, L.tile_counter, L.slots, ev);
    else launch_walker_k<T, DIM, GEOM, false, 1>(g, b, st, a, L.tile_counter, L.slots, ev);
  } else {
    if (ev) launch_walker_k<T, DIM, GEOM, true, 0>(g, b, st, a, L.tile_counter, L.slots, ev);
    else launch_walker_k<T, DIM, GEOM, false, 0>(g, b, st, a, L.tile_counter, L.slots, ev);
  }
  return hipGetLastError();
}

template <typename T, int DIM, int GEOM>
static const void* walker_symbol_t(int mode) {
  return mode == 2 ? walker_entry<T, DIM, GEOM, false, 2>()
         : mode == 1 ? walker_entry<T, DIM, GEOM, false, 1>()
                     : walker_entry<T, DIM, GEOM, false, 0>();
}

// The walkers of one precision and dimension, over the geometry kinds of that dimension.
template <typename T, int DIM>
static hipError_t launch_walker_td(const WalkerLaunch& L, hipStream_t st) {
  if constexpr (DIM == 2) {
    switch (L.geom) {
      case GK_BALL: return launch_walker_t<T, 2, GK_BALL>(L, st);
      case GK_BOX: return launch_walker_t<T, 2, GK_BOX>(L, st);
      case GK_POLYGON: return launch_walker_t<T, 2, GK_POLYGON>(L, st);
      case GK_SDF: return launch_walker_t<T, 2, GK_SDF>(L, st);
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (L.geom) {
      case GK_BALL: return launch_walker_t<T, 3, GK_BALL>(L, st);
      case GK_BOX: return launch_walker_t<T, 3, GK_BOX>(L, st);
      case GK_TRIMESH: return launch_walker_t<T, 3, GK_TRIMESH>(L, st);
      case GK_SDF: return launch_walker_t<T, 3, GK_SDF>(L, st);
      default: return hipErrorInvalidValue;
    }
  }
}

template <typename T, int DIM>
static const void* walker_symbol_td(int geom, int mode) {
  if constexpr (DIM == 2)
    return geom == GK_BALL ? walker_symbol_t<T, 2, GK_BALL>(mode)
           : geom == GK_BOX ? walker_symbol_t<T, 2, GK_BOX>(mode)
           : geom == GK_SDF ? walker_symbol_t<T, 2, GK_SDF>(mode)
                            : walker_symbol_t<T, 2, GK_POLYGON>(mode);
  else
    return geom == GK_BALL ? walker_symbol_t<T, 3, GK_BALL>(mode)
           : geom == GK_BOX ? walker_symbol_t<T, 3, GK_BOX>(mode)
           : geom == GK_SDF ? walker_symbol_t<T, 3, GK_SDF>(mode)
                            : walker_symbol_t<T, 3, GK_TRIMESH>(mode);
}

}  // namespace wos
