// Serving loop (placeholder until the scheduler lands).
#include "ctx.h"
#include "fv_internal.h"

namespace fv {
struct Server {};
}  // namespace fv

extern "C" {
fv_status fv_server_start(fv_ctx *, int) {
    fv::set_last_error("server not built yet");
    return FV_EUNSUPPORTED;
}
fv_status fv_submit(fv_ctx *, const fv_problem *, double *, uint64_t *) { return FV_EBUSY; }
fv_status fv_wait(fv_ctx *, uint64_t, double, fv_report *) { return FV_EBUSY; }
fv_status fv_server_stop(fv_ctx *) { return FV_OK; }
}
