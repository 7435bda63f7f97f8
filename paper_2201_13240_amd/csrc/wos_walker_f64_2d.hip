// FP64 walkers on 2D domains (one of four translation units of wos_walker.h).
#include "wos_walker.h"

namespace wos {

hipError_t launch_walker_f64_2d(const WalkerLaunch& L, hipStream_t st) { return launch_walker_td<double, 2>(L, st); }

const void* walker_symbol_f64_2d(int geom, int mode) { return walker_symbol_td<double, 2>(geom, mode); }

}  // namespace wos
