// FP32 walkers on 2D domains (one of four translation units of wos_walker.h).
#include "wos_walker.h"

namespace wos {

hipError_t launch_walker_f32_2d(const WalkerLaunch& L, hipStream_t st) { return launch_walker_td<float, 2>(L, st); }

const void* walker_symbol_f32_2d(int geom, int mode) { return walker_symbol_td<float, 2>(geom, mode); }

}  // namespace wos
