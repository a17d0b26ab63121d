// Drift scan with the front end on the device: the sky (equatorial unit
// vectors and fluxes) stays in HBM.  Per group of times: one launch counts
// the sources above the horizon at each time (and checks the inputs), one copy
// brings the counts to the host, one launch rotates the visible sources to ENU
// and forms their strengths with the beam (paper sections 2.3 and 2.4), packed;
// one input check of every time's visible sky (two launches) gathers the
// planning scalars, one copy brings them all to the host, and the times then
// run as one batch on their visible skies (each stage one launch over every
// time and frequency of the group).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.h"
#include "fv_internal.h"

namespace fv {
namespace {

void validate_drift(const fv_drift *d) {
    if (!d) fail(FV_EINVAL, "null argument");
    if (d->n_ant < 1 || d->n_src < 0 || d->n_freq < 1 || d->n_time < 1) fail(FV_EINVAL, "bad sizes");
    if (!d->ant_enu || !d->freq_hz || !d->lst) fail(FV_EINVAL, "null antenna, frequency or time array");
    if (d->n_src > 0 && (!d->src_eq || !d->flux)) fail(FV_EINVAL, "null source or flux array");
    if (!(d->eps >= 1e-14 && d->eps <= 1e-1)) fail(FV_EINVAL, "eps out of [1e-14, 1e-1]");
    for (long long i = 0; i < 3LL * d->n_ant; ++i)
        if (!std::isfinite(d->ant_enu[i])) fail(FV_EINVAL, "non-finite antenna position");
    for (int f = 0; f < d->n_freq; ++f)
        if (!(std::isfinite(d->freq_hz[f]) && d->freq_hz[f] > 0)) fail(FV_EINVAL, "frequency must be finite and > 0");
    for (int t = 0; t < d->n_time; ++t)
        if (!std::isfinite(d->lst[t])) fail(FV_EINVAL, "non-finite sidereal time");
    if (!(std::isfinite(d->latitude) && std::fabs(d->latitude) <= M_PI / 2)) fail(FV_EINVAL, "latitude out of range");
    if (!(std::isfinite(d->beam_fwhm) && d->beam_fwhm >= 0)) fail(FV_EINVAL, "beam width must be finite and >= 0");
    if (d->beam_fwhm > 0 && !(std::isfinite(d->beam_nu_ref) && d->beam_nu_ref > 0))
        fail(FV_EINVAL, "beam reference frequency must be finite and > 0");
    if ((d->flags & FV_METHOD_MASK) != FV_METHOD_NUFFT) fail(FV_EINVAL, "the drift entry point runs the NUFFT");
    if ((d->flags & FV_DIM_MASK) == FV_DIM_MASK) fail(FV_EINVAL, "both 2-D and 3-D forced");
    if ((d->flags & FV_PREC_MASK) == FV_PREC_MASK) fail(FV_EINVAL, "both FP32 and FP64 forced");
    if ((d->flags & FV_PREC_MASK) == FV_PREC_FP32 && d->eps < 1e-6) fail(FV_EUNSUPPORTED, "FP32 grids need eps >= 1e-6");
}

// Rows E, N, U of the rotation taking equatorial unit vectors to ENU at
// sidereal time lst and latitude lat: a turn by -lst about the polar axis
// (hour angle), then the tilt of the polar axis to the local vertical.
void rotation(double lst, double lat, double *R) {
    const double cl = std::cos(lst), sl = std::sin(lst), cp = std::cos(lat), sp = std::sin(lat);
    const double m[9] = {-sl, cl, 0.0, -sp * cl, -sp * sl, cp, cp * cl, cp * sl, sp};
    std::memcpy(R, m, sizeof(m));
}

}  // namespace

void simulate_drift(fv_ctx *ctx, const fv_drift *d, double *vis, hipStream_t st, fv_report *rep) {
    auto t0 = std::chrono::steady_clock::now();
    validate_drift(d);
    FV_HIP(hipSetDevice(ctx->device));
    Slot &slot = ctx->main;
    if (!slot.done) FV_HIP(hipEventCreateWithFlags(&slot.done, hipEventDisableTiming));
    FV_HIP(hipStreamWaitEvent(st, slot.done, 0));  // the previous call (any stream) is done with the workspace
    const int n_ant = d->n_ant, n_src = d->n_src, n_freq = d->n_freq, n_time = d->n_time;
    const long long n_pairs = (long long)n_ant * (n_ant + 1) / 2;
    // per-time workspace: packed directions and strengths of the visible
    // sources, block offsets
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const int nb = frontend_blocks(n_src);
    const DriftSizing dz = drift_sizing(n_ant, n_src, n_freq, n_time, ctx->budget);
    const size_t per_time = dz.per_time, fixed = dz.fixed;
    const int group = dz.group;

    fv_problem meta;
    std::memset(&meta, 0, sizeof(meta));
    meta.n_ant = n_ant;
    meta.ant_enu = d->ant_enu;
    meta.n_src = n_src;
    meta.n_freq = n_freq;
    meta.freq_hz = d->freq_hz;
    meta.eps = d->eps;
    meta.flags = d->flags & ~FV_GRAPH;  // each time reads its own rotated directions: no replay
    const bool unit_beam = d->beam_fwhm == 0.0;
    fv_report total;
    std::memset(&total, 0, sizeof(total));
    hipStream_t keep = slot.stream;
    slot.stream = st;
    try {
        for (int t0g = 0; t0g < n_time; t0g += group) {
            const int nt = std::min(group, n_time - t0g);
            // device buffers of this group (the inputs arena is not used by run_device)
            slot.inputs.ensure(fixed + (size_t)nt * per_time + al(72 * (size_t)nt) + al(4 * (size_t)nt + 4) + 4096);
            slot.inputs.reset();
            double *ant_dev = (double *)slot.inputs.take(24 * (size_t)n_ant);
            double *freq_dev = (double *)slot.inputs.take(8 * (size_t)n_freq);
            double *kb_dev = (double *)slot.inputs.take(8 * (size_t)n_freq);
            double *rot_dev = (double *)slot.inputs.take(72 * (size_t)nt);
            int *bbad = (int *)slot.inputs.take(4 * (size_t)nb + 4);
            int *tot = (int *)slot.inputs.take(4 * (size_t)nt + 4);
            int *bcnt = (int *)slot.inputs.take(4 * (size_t)nb * nt + 4);
            const long long dir_stride = (long long)(al(24 * (size_t)n_src) / 8);
            const long long str_stride = (long long)(al(8 * (size_t)n_freq * n_src) / 8);
            double *dir = (double *)slot.inputs.take(8 * (size_t)nt * dir_stride + 8);
            double *str = (double *)slot.inputs.take(8 * (size_t)nt * str_stride + 8);
            // host tables through pinned staging: antennas, frequencies, beam factors, rotations
            const size_t tab = 3 * (size_t)n_ant + 2 * (size_t)n_freq + 9 * (size_t)nt;
            double *h = (double *)slot.inputs.host.get(tab * sizeof(double));
            std::memcpy(h, d->ant_enu, 24 * (size_t)n_ant);
            std::memcpy(h + 3 * n_ant, d->freq_hz, 8 * (size_t)n_freq);
            for (int f = 0; f < n_freq; ++f) {
                const double F = unit_beam ? 1.0 : d->beam_fwhm * d->beam_nu_ref / d->freq_hz[f];
                h[3 * n_ant + n_freq + f] = 4.0 / (F * F);
            }
            for (int t = 0; t < nt; ++t) rotation(d->lst[t0g + t], d->latitude, h + 3 * n_ant + 2 * n_freq + 9 * t);
            FV_HIP(hipMemcpyAsync(ant_dev, h, 24 * (size_t)n_ant, hipMemcpyHostToDevice, st));
            FV_HIP(hipMemcpyAsync(freq_dev, h + 3 * n_ant, 8 * (size_t)n_freq, hipMemcpyHostToDevice, st));
            FV_HIP(hipMemcpyAsync(kb_dev, h + 3 * n_ant + n_freq, 8 * (size_t)n_freq, hipMemcpyHostToDevice, st));
            FV_HIP(hipMemcpyAsync(rot_dev, h + 3 * n_ant + 2 * n_freq, 72 * (size_t)nt, hipMemcpyHostToDevice, st));
            slot.inputs.host.record(st);
            // visible counts and input checks, brought to the host in one copy
            launch_frontend_count(d->src_eq, n_src, nt, rot_dev, d->flux, n_freq, bcnt, bbad, tot, st);
            int *cnt = (int *)ctx->plan_pin.get(sizeof(int) * ((size_t)nt + 1));
            FV_HIP(hipMemcpyAsync(cnt, tot, sizeof(int) * ((size_t)nt + 1), hipMemcpyDeviceToHost, st));
            FV_HIP(hipStreamSynchronize(st));
            if (cnt[nt] != 0) fail(FV_EINVAL, "invalid source vectors or fluxes (directions must be unit vectors)");
            const std::vector<int> vis_src(cnt, cnt + nt);
            launch_frontend(d->src_eq, n_src, nt, rot_dev, d->flux, n_freq, kb_dev, unit_beam, bcnt, tot, dir,
                            dir_stride, str, str_stride, st);
            // the input check of every visible snapshot in two launches (an
            // item table per time), its results brought back in one copy
            auto al32 = [](size_t v) { return (v + 31) / 32 * 32; };  // doubles: 256-byte alignment
            std::vector<int> nblk(nt);
            std::vector<size_t> poff(nt + 1, 0);
            int max_blk = 1;
            for (int t = 0; t < nt; ++t) {
                nblk[t] = validate_blocks_batch(vis_src[t], (long long)vis_src[t] * n_freq);
                max_blk = std::max(max_blk, nblk[t]);
                poff[t + 1] = poff[t] + al32((size_t)kValStride * nblk[t]);
            }
            const size_t d_part = al32(8 * (size_t)nt), d_tab = d_part + poff[nt];
            const size_t tab_doubles = al32((sizeof(ValItem) * (size_t)nt + 7) / 8);
            double *scal = ctx->scalars(d_tab + tab_doubles);
            double *pin = (double *)ctx->plan_pin.get((d_part + tab_doubles) * sizeof(double));
            ValItem *tabh = (ValItem *)(pin + d_part);
            for (int t = 0; t < nt; ++t) {
                ValItem &v = tabh[t];
                v = ValItem{};
                v.n_src = vis_src[t];
                v.n_fs = (long long)vis_src[t] * n_freq;
                v.src = v.n_src > 0 ? dir + t * dir_stride : nullptr;
                v.flux = v.n_fs > 0 ? str + t * str_stride : nullptr;
                v.hdr = scal + 8 * (size_t)t;  // the 8 check values only (no frequencies or antennas)
                v.part = scal + d_part + poff[t];
                v.span = validate_span_n(v.n_fs, nblk[t]);
                v.nblk = nblk[t];
            }
            ValItem *tabd = (ValItem *)(scal + d_tab);
            FV_HIP(hipMemcpyAsync(tabd, tabh, sizeof(ValItem) * (size_t)nt, hipMemcpyHostToDevice, st));
            launch_validate_batch(tabd, nt, max_blk, st);
            FV_HIP(hipMemcpyAsync(pin, scal, 8 * sizeof(double) * (size_t)nt, hipMemcpyDeviceToHost, st));
            FV_HIP(hipStreamSynchronize(st));
            // every time of the group is one problem of a batch: each stage
            // one launch over all times and frequencies
            const int dim = choose_dim(d->ant_enu, n_ant, d->eps, d->freq_hz, n_freq, d->flags);
            std::vector<fv_problem> metas(nt, meta);
            std::vector<DevInputs> ins(nt);
            for (int t = 0; t < nt; ++t) {
                const double *chk = pin + 8 * t;
                const int ns = vis_src[t];
                if (ns > 0 && (chk[6] != 0.0 || chk[7] != 0.0))
                    fail(FV_EINVAL, "invalid source vectors or fluxes (directions must be unit vectors)");
                DevInputs &in = ins[t];
                in.ant = ant_dev;
                in.freq = freq_dev;
                in.src = dir + t * dir_stride;
                in.flux = str + t * str_stride;
                in.beam = nullptr;
                in.vis = vis + 2 * (size_t)(t0g + t) * n_freq * n_pairs;
                if (ns > 0)
                    for (int a = 0; a < dim; ++a) {
                        in.s_c[a] = 0.5 * (chk[2 * a] + chk[2 * a + 1]);
                        in.S[a] = 0.5 * (chk[2 * a + 1] - chk[2 * a]);
                    }
                in.cmax = scal + d_part + poff[t];
                in.cmax_span = validate_span_n((long long)ns * n_freq, nblk[t]);
                metas[t].n_src = ns;
            }
            StageTimer &tm = slot.timer;
            tm.reset((d->flags & (FV_TIMING | FV_TIMING_ACCUM)) != 0, (d->flags & FV_TIMING_ACCUM) != 0,
                     (d->flags & FV_TIMING_ONE_STAGE) ? FV_TIMING_STAGE_OF(d->flags) : -1);
            fv_report r;
            std::memset(&r, 0, sizeof(r));
            r.fold_axis = -1;
            run_batch_device(ctx, slot, nt, metas.data(), ins.data(), r, nullptr);
            fill_report(tm, r);
            r.method = FV_METHOD_NUFFT;
            accumulate_report(r, total, t0g == 0);
        }
    } catch (...) {
        slot.stream = keep;
        (void)hipEventRecord(slot.done, st);  // work already enqueued must finish before the workspace is reused
        throw;
    }
    slot.stream = keep;
    FV_HIP(hipEventRecord(slot.done, st));
    total.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = total;
}

}  // namespace fv

extern "C" fv_status fv_simulate_drift(fv_ctx *ctx, const fv_drift *d, double *vis, void *stream, fv_report *rep) {
    try {
        if (!ctx || !d || !vis) fv::fail(FV_EINVAL, "null argument");
        if ((uintptr_t)vis & 15) fv::fail(FV_EINVAL, "the output must be 16-byte aligned");
        fv::simulate_drift(ctx, d, vis, (hipStream_t)stream, rep);
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
