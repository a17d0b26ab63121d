// Polarised feed products (paper section 2.1, Jones form, one shared beam):
// the four real strength vectors of P = A C A^H formed on the device, one
// transform each through the device path, then the combination into the
// 2 x 2 products.
#include <chrono>
#include <cstring>

#include "ctx.h"
#include "fv_internal.h"

namespace fv {

void simulate_polar(fv_ctx *ctx, const fv_polar *q, double *vis, hipStream_t st, fv_report *rep) {
    auto t0 = std::chrono::steady_clock::now();
    if (!q) fail(FV_EINVAL, "null argument");
    if (q->n_ant < 1 || q->n_src < 0 || q->n_freq < 1) fail(FV_EINVAL, "bad sizes");
    if (!q->ant_enu || !q->freq_hz) fail(FV_EINVAL, "null antenna or frequency array");
    if (q->n_src > 0 && (!q->src_lmn || !q->stokes)) fail(FV_EINVAL, "null source or Stokes array");
    if (!(q->eps >= 1e-14 && q->eps <= 1e-1)) fail(FV_EINVAL, "eps out of [1e-14, 1e-1]");
    if ((q->flags & FV_METHOD_MASK) != FV_METHOD_NUFFT) fail(FV_EINVAL, "the polarised entry point runs the NUFFT");
    if ((q->flags & FV_DIM_MASK) == FV_DIM_MASK) fail(FV_EINVAL, "both 2-D and 3-D forced");
    if ((q->flags & FV_PREC_MASK) == FV_PREC_MASK) fail(FV_EINVAL, "both FP32 and FP64 forced");
    if ((q->flags & FV_PREC_MASK) == FV_PREC_FP32 && q->eps < 1e-6) fail(FV_EUNSUPPORTED, "FP32 grids need eps >= 1e-6");
    const int n_ant = q->n_ant, n_src = q->n_src, n_freq = q->n_freq;
    const long long n_pairs = (long long)n_ant * (n_ant + 1) / 2;
    const long long n_fs = (long long)n_freq * n_src, n_fp = (long long)n_freq * n_pairs;

    FV_HIP(hipSetDevice(ctx->device));
    Slot &slot = ctx->main;
    if (!slot.done) FV_HIP(hipEventCreateWithFlags(&slot.done, hipEventDisableTiming));
    FV_HIP(hipStreamWaitEvent(st, slot.done, 0));  // the previous call (any stream) is done with the workspace
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t b_prod = 8 * 4 * (size_t)n_fs, b_tmp = 16 * 4 * (size_t)n_fp;
    slot.inputs.ensure(al(b_prod + 8) + al(b_tmp) + 1024);
    slot.inputs.reset();
    double *prod = (double *)slot.inputs.take(b_prod + 8);
    double *tmp = (double *)slot.inputs.take(b_tmp);
    fv_report total;
    try {
        launch_polar_strengths(q->stokes, q->jones, n_fs, prod, st);
        run_vectors(ctx, slot, st, q->ant_enu, n_ant, q->src_lmn, n_src, q->freq_hz, n_freq, q->eps, q->flags,
                    nullptr, prod, 4, tmp, total);
        launch_polar_combine(tmp, n_fp, vis, st);
    } catch (...) {
        (void)hipEventRecord(slot.done, st);  // work already enqueued must finish before the workspace is reused
        throw;
    }
    FV_HIP(hipEventRecord(slot.done, st));
    total.src_pairs = (double)n_src * (double)n_pairs * n_freq;  // per product
    total.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = total;
}

}  // namespace fv

extern "C" fv_status fv_simulate_polar(fv_ctx *ctx, const fv_polar *q, double *vis, void *stream, fv_report *rep) {
    try {
        if (!ctx || !q || !vis) fv::fail(FV_EINVAL, "null argument");
        if ((uintptr_t)vis & 15) fv::fail(FV_EINVAL, "the output must be 16-byte aligned");
        fv::simulate_polar(ctx, q, vis, (hipStream_t)stream, rep);
        return FV_OK;
    } catch (const fv::Error &e) {
        fv::set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        fv::set_last_error("host allocation failed");
        return FV_ENOMEM;
    } catch (const std::exception &e) {
        fv::set_last_error(e.what());
        return FV_EDEVICE;
    }
}
