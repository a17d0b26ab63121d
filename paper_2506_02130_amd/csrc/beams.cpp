// Per-antenna beams (paper section 2.2.3): one transform per pattern pair
// that occurs among the antenna pairs, with the product strengths, all pairs'
// transforms batched (each stage one launch over every pattern pair and
// frequency), then one gather of every visibility from its pattern pair's
// transform.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "ctx.h"
#include "fv_internal.h"

namespace fv {

void run_vectors(fv_ctx *ctx, Slot &slot, hipStream_t st, const double *ant_dev, int n_ant, const double *src_dev,
                 int n_src, const double *freq_dev, int n_freq, double eps, unsigned flags, const double *flux,
                 const double *prod, int n_vec, double *tmp, fv_report &total) {
    const long long n_pairs = (long long)n_ant * (n_ant + 1) / 2;
    const long long n_fs = (long long)n_freq * n_src;
    // input check and planning scalars of every vector's strengths; the first
    // one also gathers the frequencies and antenna positions
    const size_t nvd = validate_doubles(n_ant, n_freq);
    const size_t nscal = 8 + (size_t)n_freq + 3 * (size_t)n_ant;
    auto fl = [&](int v) { return flux ? flux : prod + (size_t)v * n_fs; };
    auto bm = [&](int v) { return flux ? prod + (size_t)v * n_fs : nullptr; };
    double *scal = ctx->scalars(nvd * (size_t)n_vec);
    for (int v = 0; v < n_vec; ++v)
        launch_validate(src_dev, n_src, fl(v), bm(v), n_freq, ant_dev, n_ant, freq_dev, scal + (size_t)v * nvd, st);
    double *pin = (double *)ctx->plan_pin.get(sizeof(double) * (nscal + 8 * (size_t)n_vec));
    FV_HIP(hipMemcpyAsync(pin, scal, nscal * sizeof(double), hipMemcpyDeviceToHost, st));
    for (int v = 1; v < n_vec; ++v)
        FV_HIP(hipMemcpyAsync(pin + nscal + 8 * v, scal + (size_t)v * nvd, 8 * sizeof(double), hipMemcpyDeviceToHost,
                              st));
    FV_HIP(hipStreamSynchronize(st));
    const double *pfreq = pin + 8, *pant = pfreq + n_freq;
    const std::vector<double> ant(pant, pant + 3 * (size_t)n_ant), freq(pfreq, pfreq + n_freq);
    for (double a : ant)
        if (!std::isfinite(a)) fail(FV_EINVAL, "non-finite antenna position");
    for (double f : freq)
        if (!(std::isfinite(f) && f > 0)) fail(FV_EINVAL, "frequency must be finite and > 0");
    for (int v = 0; v < n_vec; ++v) {
        const double *chk = v == 0 ? pin : pin + nscal + 8 * v;
        if (n_src > 0 && (chk[6] != 0.0 || chk[7] != 0.0))
            fail(FV_EINVAL, "invalid source directions or strengths");
    }
    fv_problem meta;
    std::memset(&meta, 0, sizeof(meta));
    meta.n_ant = n_ant;
    meta.ant_enu = ant.data();
    meta.n_src = n_src;
    meta.n_freq = n_freq;
    meta.freq_hz = freq.data();
    meta.eps = eps;
    meta.flags = flags & ~FV_GRAPH;  // several transforms share the workspace: no replay
    const int dim = choose_dim(ant.data(), n_ant, eps, freq.data(), n_freq, flags);
    std::memset(&total, 0, sizeof(total));
    total.fold_axis = -1;
    // every vector is one problem of a batch: the transforms of all vectors
    // and frequencies share each stage's launch
    std::vector<fv_problem> metas(n_vec, meta);
    std::vector<DevInputs> ins(n_vec);
    for (int v = 0; v < n_vec; ++v) {
        DevInputs &in = ins[v];
        in.ant = ant_dev;
        in.freq = freq_dev;
        in.src = src_dev;
        in.flux = fl(v);
        in.beam = bm(v);
        in.vis = tmp + 2 * (size_t)v * n_freq * n_pairs;
        if (n_src > 0)
            for (int a = 0; a < dim; ++a) {  // the same directions for every vector
                in.s_c[a] = 0.5 * (pin[2 * a] + pin[2 * a + 1]);
                in.S[a] = 0.5 * (pin[2 * a + 1] - pin[2 * a]);
            }
        in.cmax = validate_partials(scal + (size_t)v * nvd, n_ant, n_freq);
        in.cmax_span = validate_span(n_fs);
    }
    StageTimer &tm = slot.timer;
    tm.reset((flags & (FV_TIMING | FV_TIMING_ACCUM)) != 0, (flags & FV_TIMING_ACCUM) != 0,
             (flags & FV_TIMING_ONE_STAGE) ? FV_TIMING_STAGE_OF(flags) : -1);
    hipStream_t keep = slot.stream;
    slot.stream = st;
    try {
        run_batch_device(ctx, slot, n_vec, metas.data(), ins.data(), total, nullptr);
    } catch (...) {
        slot.stream = keep;
        throw;
    }
    slot.stream = keep;
    fill_report(tm, total);
    total.method = FV_METHOD_NUFFT;
}

void simulate_beams(fv_ctx *ctx, const fv_beams *b, double *vis, hipStream_t st, fv_report *rep) {
    auto t0 = std::chrono::steady_clock::now();
    if (!b) fail(FV_EINVAL, "null argument");
    if (b->n_ant < 1 || b->n_src < 0 || b->n_freq < 1 || b->n_beam < 1) fail(FV_EINVAL, "bad sizes");
    if (!b->ant_enu || !b->freq_hz || !b->beam_of_ant) fail(FV_EINVAL, "null antenna, frequency or pattern array");
    if (b->n_src > 0 && (!b->src_lmn || !b->flux || !b->beams)) fail(FV_EINVAL, "null source, flux or beam array");
    if (!(b->eps >= 1e-14 && b->eps <= 1e-1)) fail(FV_EINVAL, "eps out of [1e-14, 1e-1]");
    if ((b->flags & FV_METHOD_MASK) != FV_METHOD_NUFFT) fail(FV_EINVAL, "the per-antenna beam entry point runs the NUFFT");
    if ((b->flags & FV_DIM_MASK) == FV_DIM_MASK) fail(FV_EINVAL, "both 2-D and 3-D forced");
    if ((b->flags & FV_PREC_MASK) == FV_PREC_MASK) fail(FV_EINVAL, "both FP32 and FP64 forced");
    if ((b->flags & FV_PREC_MASK) == FV_PREC_FP32 && b->eps < 1e-6) fail(FV_EUNSUPPORTED, "FP32 grids need eps >= 1e-6");
    const int n_ant = b->n_ant, n_src = b->n_src, n_freq = b->n_freq;
    for (int i = 0; i < n_ant; ++i)
        if (b->beam_of_ant[i] < 0 || b->beam_of_ant[i] >= b->n_beam) fail(FV_EINVAL, "pattern index out of range");
    const long long n_pairs = (long long)n_ant * (n_ant + 1) / 2;
    const long long n_fs = (long long)n_freq * n_src;

    // pattern pairs that occur, and the pair each visibility takes
    std::map<std::pair<int, int>, int> index;
    std::vector<int> pq, vec((size_t)n_pairs);
    for (int i = 0, k = 0; i < n_ant; ++i)
        for (int j = i; j < n_ant; ++j, ++k) {
            const int p = std::min(b->beam_of_ant[i], b->beam_of_ant[j]);
            const int q = std::max(b->beam_of_ant[i], b->beam_of_ant[j]);
            auto it = index.find({p, q});
            if (it == index.end()) {
                it = index.emplace(std::make_pair(p, q), (int)(pq.size() / 2)).first;
                pq.push_back(p);
                pq.push_back(q);
            }
            vec[(size_t)k] = it->second;
        }
    const int n_vec = (int)(pq.size() / 2);

    FV_HIP(hipSetDevice(ctx->device));
    Slot &slot = ctx->main;
    if (!slot.done) FV_HIP(hipEventCreateWithFlags(&slot.done, hipEventDisableTiming));
    FV_HIP(hipStreamWaitEvent(st, slot.done, 0));  // the previous call (any stream) is done with the workspace
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t b_prod = 8 * (size_t)n_vec * n_fs, b_tmp = 16 * (size_t)n_vec * n_freq * n_pairs;
    slot.inputs.ensure(al(8 * (size_t)n_vec + 8) + al(4 * (size_t)n_pairs) + al(b_prod + 8) + al(b_tmp) + 2048);
    slot.inputs.reset();
    int *pq_dev = (int *)slot.inputs.take(8 * (size_t)n_vec + 8);
    int *vec_dev = (int *)slot.inputs.take(4 * (size_t)n_pairs);
    double *prod = (double *)slot.inputs.take(b_prod + 8);
    double *tmp = (double *)slot.inputs.take(b_tmp);
    {
        const size_t bytes = 8 * (size_t)n_vec + 4 * (size_t)n_pairs;
        char *h = (char *)slot.inputs.host.get(bytes);
        std::memcpy(h, pq.data(), 8 * (size_t)n_vec);
        std::memcpy(h + 8 * (size_t)n_vec, vec.data(), 4 * (size_t)n_pairs);
        FV_HIP(hipMemcpyAsync(pq_dev, h, 8 * (size_t)n_vec, hipMemcpyHostToDevice, st));
        FV_HIP(hipMemcpyAsync(vec_dev, h + 8 * (size_t)n_vec, 4 * (size_t)n_pairs, hipMemcpyHostToDevice, st));
        slot.inputs.host.record(st);
    }
    if (n_src > 0) launch_beam_products(b->beams, pq_dev, n_vec, n_fs, prod, st);

    fv_report total;
    try {
        run_vectors(ctx, slot, st, b->ant_enu, n_ant, b->src_lmn, n_src, b->freq_hz, n_freq, b->eps, b->flags,
                    b->flux, prod, n_vec, tmp, total);
        launch_beam_select(tmp, vec_dev, n_pairs, n_freq, vis, st);
    } catch (...) {
        (void)hipEventRecord(slot.done, st);  // work already enqueued must finish before the workspace is reused
        throw;
    }
    FV_HIP(hipEventRecord(slot.done, st));
    total.src_pairs = (double)n_src * (double)n_pairs * n_freq;  // each visibility once
    total.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = total;
}

}  // namespace fv

extern "C" fv_status fv_simulate_beams(fv_ctx *ctx, const fv_beams *b, double *vis, void *stream, fv_report *rep) {
    try {
        if (!ctx || !b || !vis) fv::fail(FV_EINVAL, "null argument");
        if ((uintptr_t)vis & 15) fv::fail(FV_EINVAL, "the output must be 16-byte aligned");
        fv::simulate_beams(ctx, b, vis, (hipStream_t)stream, rep);
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
