// Batched snapshots: every problem of the batch is uploaded once, its
// frequencies become NUFFT jobs, and all jobs of one kernel family
// (dimension, precision, kernel width) run as one launch sequence, each stage
// one launch over every snapshot of the batch (the per-(time, frequency)
// calls of the paper's simulator, section 5.4, gathered into single launches).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>

#include "ctx.h"
#include "fv_internal.h"

namespace fv {
namespace {

struct BatchInputs {
    DevInputs in;
    double *vis = nullptr;
    size_t vis_bytes = 0;
};

std::vector<BatchInputs> upload_batch(Slot &slot, int n, const fv_problem *ps) {
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        const fv_problem &p = ps[i];
        const size_t fs = sizeof(double) * (size_t)p.n_freq * p.n_src;
        const long long np = (long long)p.n_ant * (p.n_ant + 1) / 2;
        total += al(24 * (size_t)p.n_ant) + al(8 * (size_t)p.n_freq) + al(24 * (size_t)p.n_src) +
                 al(fs) * (p.beam ? 2 : 1) + al(16 * (size_t)np * p.n_freq);
    }
    slot.inputs.ensure(total + 256);
    slot.inputs.reset();
    std::vector<BatchInputs> out(n);
    hipStream_t st = slot.stream;
    for (int i = 0; i < n; ++i) {
        const fv_problem &p = ps[i];
        BatchInputs &b = out[i];
        const size_t fs = sizeof(double) * (size_t)p.n_freq * p.n_src;
        const long long np = (long long)p.n_ant * (p.n_ant + 1) / 2;
        b.in.ant = (double *)slot.inputs.take(24 * (size_t)p.n_ant);
        FV_HIP(hipMemcpyAsync((void *)b.in.ant, p.ant_enu, 24 * (size_t)p.n_ant, hipMemcpyHostToDevice, st));
        b.in.freq = (double *)slot.inputs.take(8 * (size_t)p.n_freq);
        FV_HIP(hipMemcpyAsync((void *)b.in.freq, p.freq_hz, 8 * (size_t)p.n_freq, hipMemcpyHostToDevice, st));
        if (p.n_src) {
            b.in.src = (double *)slot.inputs.take(24 * (size_t)p.n_src);
            b.in.flux = (double *)slot.inputs.take(fs);
            FV_HIP(hipMemcpyAsync((void *)b.in.src, p.src_lmn, 24 * (size_t)p.n_src, hipMemcpyHostToDevice, st));
            FV_HIP(hipMemcpyAsync((void *)b.in.flux, p.flux, fs, hipMemcpyHostToDevice, st));
            if (p.beam) {
                b.in.beam = (double *)slot.inputs.take(fs);
                FV_HIP(hipMemcpyAsync((void *)b.in.beam, p.beam, fs, hipMemcpyHostToDevice, st));
            }
        }
        b.vis_bytes = 16 * (size_t)np * p.n_freq;
        b.vis = (double *)slot.inputs.take(b.vis_bytes);
        b.in.vis = b.vis;
        const int dim = choose_dim(p.ant_enu, p.n_ant, p.eps, p.freq_hz, p.n_freq, p.flags);
        src_box(p.src_lmn, p.n_src, dim, b.in.s_c, b.in.S);
    }
    return out;
}

}  // namespace

void simulate_batch(fv_ctx *ctx, Slot &slot, int n, const fv_problem *ps, double *const *vis, fv_report *rep) {
    auto t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < n; ++i) {
        validate_host(&ps[i]);
        if (!vis[i]) fail(FV_EINVAL, "null output pointer in batch");
    }
    FV_HIP(hipSetDevice(ctx->device));
    hipStream_t st = slot.stream;
    if (slot.done) FV_HIP(hipStreamWaitEvent(st, slot.done, 0));  // a device-entry call's work
    std::vector<BatchInputs> bi = upload_batch(slot, n, ps);
    fv_report r;
    std::memset(&r, 0, sizeof(r));
    r.fold_axis = -1;
    StageTimer &tm = slot.timer;
    tm.reset(n > 0 && (ps[0].flags & FV_TIMING) != 0);
    std::map<NufftGroupKey, std::vector<SnapJob>> groups;
    std::vector<std::shared_ptr<TargetTable>> hold;
    bool first_nufft = true, arena_busy = false;
    for (int i = 0; i < n; ++i) {
        const fv_problem &p = ps[i];
        const long long np = (long long)p.n_ant * (p.n_ant + 1) / 2;
        r.src_pairs += (double)p.n_src * (double)np * (double)p.n_freq;
        const unsigned method = p.flags & FV_METHOD_MASK;
        if (p.n_src == 0) {
            launch_zero_c128(bi[i].vis, np * p.n_freq, st);
        } else if (method != FV_METHOD_NUFFT) {
            if (arena_busy) FV_HIP(hipStreamSynchronize(st));
            const int dim = choose_dim(p.ant_enu, p.n_ant, p.eps, p.freq_hz, p.n_freq, p.flags);
            run_direct(ctx, slot, p, bi[i].in, bi[i].vis, dim, choose_prec(p.eps, p.flags), &tm);
            arena_busy = method == FV_METHOD_MFMA;
        } else {
            const int dim = choose_dim(p.ant_enu, p.n_ant, p.eps, p.freq_hz, p.n_freq, p.flags);
            if (dim == 2 && !(p.flags & FV_NO_LATTICE)) {
                if (arena_busy) FV_HIP(hipStreamSynchronize(st));
                if (run_lattice(ctx, slot, p, bi[i].in, bi[i].vis, choose_prec(p.eps, p.flags), &tm, r)) {
                    arena_busy = true;
                    continue;
                }
            }
            std::vector<SnapJob> jobs;
            SnapPlan top;
            NufftGroupKey k = append_jobs(ctx, p, bi[i].in, bi[i].vis, st, jobs, hold, &top);
            auto &g = groups[k];
            g.insert(g.end(), jobs.begin(), jobs.end());
            if (first_nufft) {
                first_nufft = false;
                r.dim = k.dim;
                r.prec_bits = k.prec;
                r.w = k.w;
                r.fold_axis = k.fold_axis;
                for (int a = 0; a < 3; ++a) {
                    r.n1[a] = top.n1[a];
                    r.n2[a] = top.n2[a];
                }
            }
        }
    }
    for (auto &kv : groups) {
        if (arena_busy) FV_HIP(hipStreamSynchronize(st));  // the workspace arena is reused
        r.model_bytes += execute_jobs(ctx, slot, kv.second, kv.first, &tm);
        arena_busy = true;
    }
    FV_HIP(hipGetLastError());
    for (int i = 0; i < n; ++i)
        FV_HIP(hipMemcpyAsync(vis[i], bi[i].vis, bi[i].vis_bytes, hipMemcpyDeviceToHost, st));
    FV_HIP(hipStreamSynchronize(st));
    fill_report(tm, r);
    if (n > 0) r.method = (int)(ps[0].flags & FV_METHOD_MASK);
    r.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = r;
}

}  // namespace fv

extern "C" fv_status fv_simulate_batch(fv_ctx *ctx, int n_snap, const fv_problem *snaps, double *const *vis,
                                       fv_report *rep) {
    try {
        if (!ctx || n_snap < 0 || (n_snap > 0 && (!snaps || !vis))) fv::fail(FV_EINVAL, "null argument");
        fv::simulate_batch(ctx, ctx->main, n_snap, snaps, vis, rep);
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
