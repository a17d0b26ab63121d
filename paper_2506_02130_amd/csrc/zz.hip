// Direct sum in antenna-factor form V = Z diag(c) Z^H on the matrix cores
// (paper section 5.1); placeholder until the MFMA kernel lands.
#include "fv_internal.h"

namespace fv {

size_t zz_work_bytes(int, int) { return 256; }

void launch_zz(const double *, int, const double *, int, const double *, int, const double *, const double *, int,
               double *, void *, hipStream_t, StageTimer *) {
    fail(FV_EUNSUPPORTED, "matrix-core direct sum not built yet");
}

}  // namespace fv
