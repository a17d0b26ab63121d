// Kernel instances of the type-3 pipeline for float grids in 2-D, every kernel width.
#include "nufft_impl.h"

namespace fv {
namespace detail {
PipeFn pick_f32_2d(int w) { return pick_w<float, 2>(w, WList{}); }
}  // namespace detail
}  // namespace fv
