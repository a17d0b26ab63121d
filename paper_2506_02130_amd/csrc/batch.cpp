// Batched snapshots (placeholder until the batched launcher lands).
#include "ctx.h"
#include "fv_internal.h"

extern "C" fv_status fv_simulate_batch(fv_ctx *, int, const fv_problem *, double *const *, fv_report *) {
    fv::set_last_error("batch entry point not built yet");
    return FV_EUNSUPPORTED;
}
