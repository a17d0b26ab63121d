// Spectral basis (paper appendix A): the spectra of every source are
// projected onto K orthonormal functions of frequency, their products formed
// with the basis's structure constants, and one type-3 transform per basis
// function, planned at the top frequency, evaluates the result at every
// frequency's baselines (all frequencies are targets of the one transform);
// the interpolation reads the K grids at each target's cells with one set of
// weights and writes the basis expansion, the visibilities, directly.  K
// transforms replace n_freq of them.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.h"
#include "fv_internal.h"

namespace fv {
namespace {

// Discrete orthonormal polynomials on the frequencies: Gram-Schmidt (twice,
// for orthogonality to rounding) on 1, x, x^2, ... with
// x = (nu - nu_mid) / half-width; R's diagonal is positive by construction.
std::vector<double> spectral_basis(const double *freq, int n_freq, int K) {
    double lo = freq[0], hi = freq[0];
    for (int q = 1; q < n_freq; ++q) {
        lo = std::min(lo, freq[q]);
        hi = std::max(hi, freq[q]);
    }
    const double mid = 0.5 * (lo + hi), half = hi > lo ? 0.5 * (hi - lo) : 1.0;
    std::vector<double> M((size_t)n_freq * K);  // [q][k]
    std::vector<double> col(n_freq);
    for (int k = 0; k < K; ++k) {
        for (int q = 0; q < n_freq; ++q) col[q] = std::pow((freq[q] - mid) / half, k);
        for (int pass = 0; pass < 2; ++pass)
            for (int j = 0; j < k; ++j) {
                double dot = 0.0;
                for (int q = 0; q < n_freq; ++q) dot += M[(size_t)q * K + j] * col[q];
                for (int q = 0; q < n_freq; ++q) col[q] -= dot * M[(size_t)q * K + j];
            }
        double nrm = 0.0;
        for (int q = 0; q < n_freq; ++q) nrm += col[q] * col[q];
        nrm = std::sqrt(nrm);
        if (!(nrm > 1e-12)) fail(FV_EINVAL, "the frequencies do not support this many basis functions");
        for (int q = 0; q < n_freq; ++q) M[(size_t)q * K + k] = col[q] / nrm;
    }
    return M;
}

}  // namespace

void simulate_basis(fv_ctx *ctx, const fv_problem *p, int K, double *vis, hipStream_t st, fv_report *rep) {
    auto t0 = std::chrono::steady_clock::now();
    if (p->n_ant < 1 || p->n_src < 0 || p->n_freq < 1) fail(FV_EINVAL, "bad sizes");
    if (!p->ant_enu || !p->freq_hz || (p->n_src > 0 && (!p->src_lmn || !p->flux))) fail(FV_EINVAL, "null device array");
    if (!(p->eps >= 1e-14 && p->eps <= 1e-1)) fail(FV_EINVAL, "eps out of [1e-14, 1e-1]");
    if ((p->flags & FV_METHOD_MASK) != FV_METHOD_NUFFT) fail(FV_EINVAL, "the spectral-basis entry point runs the NUFFT");
    if ((p->flags & FV_DIM_MASK) == FV_DIM_MASK) fail(FV_EINVAL, "both 2-D and 3-D forced");
    if ((p->flags & FV_PREC_MASK) == FV_PREC_MASK) fail(FV_EINVAL, "both FP32 and FP64 forced");
    if ((p->flags & FV_PREC_MASK) == FV_PREC_FP32 && p->eps < 1e-6) fail(FV_EUNSUPPORTED, "FP32 grids need eps >= 1e-6");
    if (K < 1 || K > basis_max() || K > p->n_freq) fail(FV_EINVAL, "basis size must be in [1, min(n_freq, 16)]");
    const int n_ant = p->n_ant, n_src = p->n_src, n_freq = p->n_freq;
    const long long n_pairs = (long long)n_ant * (n_ant + 1) / 2;
    if ((double)n_pairs * n_freq >= 2147483647.0) fail(FV_EUNSUPPORTED, "too many (pair, frequency) targets");

    FV_HIP(hipSetDevice(ctx->device));
    Slot &slot = ctx->main;
    if (!slot.done) FV_HIP(hipEventCreateWithFlags(&slot.done, hipEventDisableTiming));
    FV_HIP(hipStreamWaitEvent(st, slot.done, 0));  // the previous call (any stream) is done with the workspace
    // input check and planning scalars
    const size_t nscal = 8 + (size_t)n_freq + 3 * (size_t)n_ant;
    double *scal = ctx->scalars(validate_doubles(n_ant, n_freq));
    launch_validate(p->src_lmn, n_src, p->flux, p->beam, n_freq, p->ant_enu, n_ant, p->freq_hz, scal, st);
    double *pin = (double *)ctx->plan_pin.get(nscal * sizeof(double));
    FV_HIP(hipMemcpyAsync(pin, scal, nscal * sizeof(double), hipMemcpyDeviceToHost, st));
    FV_HIP(hipStreamSynchronize(st));
    const std::vector<double> freq(pin + 8, pin + 8 + n_freq), ant(pin + 8 + n_freq, pin + nscal);
    for (double a : ant)
        if (!std::isfinite(a)) fail(FV_EINVAL, "non-finite antenna position");
    for (double f : freq)
        if (!(std::isfinite(f) && f > 0)) fail(FV_EINVAL, "frequency must be finite and > 0");
    if (n_src > 0 && (pin[6] != 0.0 || pin[7] != 0.0)) fail(FV_EINVAL, "invalid source directions or strengths");
    const int dim = choose_dim(ant.data(), n_ant, p->eps, freq.data(), n_freq, p->flags);
    double s_c[3] = {0, 0, 0}, S[3] = {0, 0, 0};
    if (n_src > 0)
        for (int a = 0; a < dim; ++a) {
            s_c[a] = 0.5 * (pin[2 * a] + pin[2 * a + 1]);
            S[a] = 0.5 * (pin[2 * a + 1] - pin[2 * a]);
        }

    // the basis and its structure constants (host, FP64)
    const std::vector<double> M = spectral_basis(freq.data(), n_freq, K);
    std::vector<double> d((size_t)K * K * K, 0.0);
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j)
            for (int k = 0; k < K; ++k) {
                double acc = 0.0;
                for (int q = 0; q < n_freq; ++q)
                    acc += M[(size_t)q * K + i] * M[(size_t)q * K + j] * M[(size_t)q * K + k];
                d[((size_t)i * K + j) * K + k] = acc;
            }

    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t bM = 8 * M.size(), bd = 8 * d.size(), bv = 8 * (size_t)K * n_src + 8;
    slot.inputs.ensure(al(bM) + al(bd) + al(bv) + 2048);
    slot.inputs.reset();
    double *M_dev = (double *)slot.inputs.take(bM);
    double *d_dev = (double *)slot.inputs.take(bd);
    double *v = (double *)slot.inputs.take(bv);
    {
        char *h = (char *)slot.inputs.host.get(bM + bd);
        std::memcpy(h, M.data(), bM);
        std::memcpy(h + bM, d.data(), bd);
        FV_HIP(hipMemcpyAsync(M_dev, h, bM, hipMemcpyHostToDevice, st));
        FV_HIP(hipMemcpyAsync(d_dev, h + bM, bd, hipMemcpyHostToDevice, st));
        slot.inputs.host.record(st);
    }

    fv_report r;
    std::memset(&r, 0, sizeof(r));
    StageTimer &tm = slot.timer;
    tm.reset((p->flags & FV_TIMING) != 0);
    hipStream_t keep = slot.stream;
    slot.stream = st;
    try {
        if (n_src == 0) {
            launch_zero_c128(vis, n_pairs * n_freq, st);
        } else {
            launch_basis_coeffs(M_dev, d_dev, n_freq, K, n_src, p->flux, p->beam, v, st);
            double numax = 0.0;
            for (double f : freq) numax = std::max(numax, f);
            std::vector<double> scales(n_freq);
            for (int q = 0; q < n_freq; ++q) scales[q] = freq[q] / numax;
            const bool fold = !(p->flags & FV_NO_FOLD);
            GeomPlan g = ctx_geometry(ctx, ant.data(), n_ant, dim, p->eps, s_c, S, fold);
            std::shared_ptr<TargetTable> tt = ctx_targets(ctx, ant.data(), p->ant_enu, g, st, &scales);
            NufftGroupKey key;
            key.dim = dim;
            key.prec = choose_prec(p->eps, p->flags);
            key.w = g.w;
            key.fold_axis = g.fold_axis;
            key.flags = p->flags & FV_AUTOTUNE;
            std::vector<SnapJob> jobs;
            for (int k = 0; k < K; ++k) {
                SnapJob j;
                j.plan = plan_snapshot(g, numax);
                j.src = p->src_lmn;
                j.n_src = n_src;
                j.flux = v + (size_t)k * n_src;
                j.beam = nullptr;
                j.out = vis;  // not written: the interpolation below writes vis directly
                j.tt = tt.get();
                jobs.push_back(j);
            }
            // one launch group (all K grids are read per target): no workspace cap
            ExecOpts opts;
            opts.autotune = (p->flags & FV_AUTOTUNE) != 0;
            opts.tunes = &ctx->tunes;
            opts.graphs = &slot.graphs;
            opts.basis_M = M_dev;
            opts.basis_vis = vis;
            opts.basis_np = n_pairs;
            r.model_bytes = nufft_execute(jobs, dim, key.prec, key.w, slot.arena, ctx->cache, st, &tm, &opts);
            r.dim = dim;
            r.prec_bits = key.prec;
            r.w = g.w;
            r.fold_axis = g.fold_axis;
            for (int a = 0; a < 3; ++a) {
                r.n1[a] = jobs[0].plan.n1[a];
                r.n2[a] = jobs[0].plan.n2[a];
            }
        }
        FV_HIP(hipGetLastError());
    } catch (...) {
        slot.stream = keep;
        (void)hipEventRecord(slot.done, st);  // work already enqueued must finish before the workspace is reused
        throw;
    }
    slot.stream = keep;
    FV_HIP(hipEventRecord(slot.done, st));
    fill_report(tm, r);
    r.method = FV_METHOD_NUFFT;
    r.src_pairs = (double)n_src * (double)n_pairs * n_freq;
    r.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = r;
}

}  // namespace fv

extern "C" fv_status fv_simulate_basis(fv_ctx *ctx, const fv_problem *p, int n_basis, double *vis, void *stream,
                                       fv_report *rep) {
    try {
        if (!ctx || !p || !vis) fv::fail(FV_EINVAL, "null argument");
        if ((uintptr_t)vis & 15) fv::fail(FV_EINVAL, "the output must be 16-byte aligned");
        fv::simulate_basis(ctx, p, n_basis, vis, (hipStream_t)stream, rep);
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
