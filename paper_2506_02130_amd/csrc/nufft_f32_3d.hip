// Kernel instances of the type-3 pipeline for float grids in 3-D, every kernel width.
#include "nufft_impl.h"

namespace fv {
namespace detail {
PipeFn pick_f32_3d(int w) { return pick_w<float, 3>(w, WList{}); }
}  // namespace detail
}  // namespace fv
