// Kernel instances of the type-3 pipeline for double grids in 3-D, every kernel width.
#include "nufft_impl.h"

namespace fv {
namespace detail {
PipeFn pick_f64_3d(int w) { return pick_w<double, 3>(w, WList{}); }
}  // namespace detail
}  // namespace fv
