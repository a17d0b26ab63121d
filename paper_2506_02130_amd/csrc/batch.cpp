// Batched snapshots: every problem of the batch is uploaded once, its
// frequencies become NUFFT jobs, and all jobs of one kernel family
// (dimension, precision, kernel width) run as one launch sequence, each stage
// one launch over every snapshot of the batch (the per-(time, frequency)
// calls of the paper's simulator, section 5.4, gathered into single launches).
#include <algorithm>
#include <array>
#include <chrono>
#include <cstring>
#include <cmath>
#include <map>
#include <tuple>

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

void run_batch_device(fv_ctx *ctx, Slot &slot, int n, const fv_problem *ps, const DevInputs *in, fv_report &r,
                      std::vector<char> *lattice_used) {
    hipStream_t st = slot.stream;
    if (lattice_used) lattice_used->assign(n, 0);
    StageTimer &tm = slot.timer;
    std::map<NufftGroupKey, std::vector<SnapJob>> groups;
    // lattice problems by (precision, kernel width, captured): each group is
    // one launch per stage over all of its problems and frequencies
    std::map<std::tuple<int, int, bool>, std::vector<LatItem>> lat;
    std::vector<std::shared_ptr<LatticePlan>> lat_hold;
    std::vector<std::shared_ptr<TargetTable>> hold;
    bool first = true, arena_busy = false;
    for (int i = 0; i < n; ++i) {
        const fv_problem &p = ps[i];
        const long long np = (long long)p.n_ant * (p.n_ant + 1) / 2;
        r.src_pairs += (double)p.n_src * (double)np * (double)p.n_freq;
        const unsigned method = p.flags & FV_METHOD_MASK;
        if (p.n_src == 0) {
            launch_zero_c128(in[i].vis, np * p.n_freq, st);
            continue;
        }
        const int dim = choose_dim(p.ant_enu, p.n_ant, p.eps, p.freq_hz, p.n_freq, p.flags);
        const int prec = choose_prec(p.eps, p.flags);
        if (method != FV_METHOD_NUFFT) {
            if (arena_busy) FV_HIP(hipStreamSynchronize(st));  // the workspace arena is reused
            run_direct(ctx, slot, p, in[i], in[i].vis, dim, prec, &tm);
            arena_busy = method == FV_METHOD_MFMA;
            continue;
        }
        if (dim == 2 && !(p.flags & FV_NO_LATTICE)) {
            int w = 0;
            if (std::shared_ptr<LatticePlan> lp = lattice_choice(ctx, p, in[i], prec, &w)) {
                LatItem it;
                it.lp = lp.get();
                it.src = in[i].src;
                it.flux = in[i].flux;
                it.beam = in[i].beam;
                it.cmax = in[i].cmax;
                it.cmax_span = in[i].cmax_span;
                it.freq = in[i].freq;
                it.n_src = p.n_src;
                it.n_freq = p.n_freq;
                it.n_ant = p.n_ant;
                it.vis = in[i].vis;
                lat[{prec, w, (p.flags & FV_GRAPH) != 0}].push_back(it);
                lat_hold.push_back(lp);
                if (lattice_used) (*lattice_used)[i] = 1;
                if (first) {
                    first = false;
                    int nf[2];
                    lattice_grid(*lp, w, nf);
                    r.lattice = 1;
                    r.dim = 2;
                    r.prec_bits = prec;
                    r.w = w;
                    r.n1[0] = r.n2[0] = nf[0];
                    r.n1[1] = r.n2[1] = nf[1];
                }
                continue;
            }
        }
        std::vector<SnapJob> jobs;
        SnapPlan top;
        NufftGroupKey k = append_jobs(ctx, p, in[i], in[i].vis, st, jobs, hold, &top);
        auto &g = groups[k];
        g.insert(g.end(), jobs.begin(), jobs.end());
        if (first) {
            first = false;
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
    // the lattice groups take their own arena, so they follow each other and
    // the direct sums with no host wait
    if (!lat.empty()) {
        size_t need = 0;
        for (auto &kv : lat) need += lattice_batch_bytes(kv.second, std::get<0>(kv.first), std::get<1>(kv.first)) + 256;
        slot.lat.ensure(need);
        slot.lat.reset();
        for (auto &kv : lat) {
            const int prec = std::get<0>(kv.first), w = std::get<1>(kv.first);
            void *work = slot.lat.take(lattice_batch_bytes(kv.second, prec, w));
            r.model_bytes += launch_lattice_batch(kv.second, prec, w, work, slot.lat.host, st, &tm,
                                                  std::get<2>(kv.first) ? &slot.graphs : nullptr);
        }
    }
    for (auto &kv : groups) {
        if (arena_busy) FV_HIP(hipStreamSynchronize(st));  // the workspace arena is reused
        r.model_bytes += execute_jobs(ctx, slot, kv.second, kv.first, &tm);
        arena_busy = true;
    }
    FV_HIP(hipGetLastError());
}

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
    slot.timer.reset(n > 0 && (ps[0].flags & FV_TIMING) != 0);
    std::vector<DevInputs> in(n);
    for (int i = 0; i < n; ++i) in[i] = bi[i].in;
    run_batch_device(ctx, slot, n, ps, in.data(), r, nullptr);
    for (int i = 0; i < n; ++i)
        FV_HIP(hipMemcpyAsync(vis[i], bi[i].vis, bi[i].vis_bytes, hipMemcpyDeviceToHost, st));
    FV_HIP(hipStreamSynchronize(st));
    fill_report(slot.timer, r);
    if (n > 0) r.method = (int)(ps[0].flags & FV_METHOD_MASK);
    r.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = r;
}

// Problems on the device: one input-check launch per problem into one
// scratch buffer, one copy of every problem's planning scalars (check
// results, frequencies, antenna positions) through pinned staging and one
// host wait for them, then the whole batch enqueued on `st`.
void simulate_batch_dev(fv_ctx *ctx, int n, const fv_problem *ps, double *const *vis, hipStream_t st,
                        fv_report *rep) {
    auto t0 = std::chrono::steady_clock::now();
    if (n > 65535) fail(FV_EUNSUPPORTED, "more than 65535 problems in one device batch");
    for (int i = 0; i < n; ++i) {
        const fv_problem &p = ps[i];
        check_dev_args(p, vis[i]);
        if ((p.flags & FV_PREC_MASK) == FV_PREC_FP32 && p.eps < 1e-6)
            fail(FV_EUNSUPPORTED, "FP32 grids need eps >= 1e-6");
    }
    FV_HIP(hipSetDevice(ctx->device));
    Slot &slot = ctx->main;
    if (!slot.done) FV_HIP(hipEventCreateWithFlags(&slot.done, hipEventDisableTiming));
    FV_HIP(hipStreamWaitEvent(st, slot.done, 0));  // the previous call (any stream) is done with the workspaces
    // The input check of the whole batch in two launches; its partials carry
    // the largest strength of each flat range, which the lattice path reads.
    // Device scratch: [packed headers][partials of each problem][item table];
    // pinned: [packed headers][item table].
    auto al = [](size_t v) { return (v + 31) / 32 * 32; };  // in doubles: 256-byte alignment
    std::vector<size_t> hoff(n + 1, 0), poff(n + 1, 0);
    std::vector<int> nblk(n);
    int max_blk = 1;
    for (int i = 0; i < n; ++i) {
        const fv_problem &p = ps[i];
        hoff[i + 1] = hoff[i] + 8 + (size_t)p.n_freq + 3 * (size_t)p.n_ant;
        nblk[i] = validate_blocks_batch(p.n_src, (long long)p.n_src * p.n_freq);
        max_blk = std::max(max_blk, nblk[i]);
        poff[i + 1] = poff[i] + al((size_t)kValStride * nblk[i]);
    }
    const size_t d_part = al(hoff[n]), d_tab = d_part + poff[n];
    const size_t tab_doubles = al((sizeof(ValItem) * (size_t)n + 7) / 8);
    double *dev = nullptr, *pin = nullptr;
    if (!ctx->bspec.ev) FV_HIP(hipEventCreateWithFlags(&ctx->bspec.ev, hipEventDisableTiming));
    if (n > 0) {
        dev = ctx->scalars(d_tab + tab_doubles);
        pin = (double *)ctx->plan_pin.get((al(hoff[n]) + tab_doubles) * sizeof(double));
        ValItem *tab = (ValItem *)(pin + al(hoff[n]));
        for (int i = 0; i < n; ++i) {
            const fv_problem &p = ps[i];
            ValItem &v = tab[i];
            v = ValItem{};
            v.n_fs = p.n_src > 0 ? (long long)p.n_src * p.n_freq : 0;
            v.src = p.n_src > 0 ? p.src_lmn : nullptr;
            v.flux = v.n_fs ? p.flux : nullptr;
            v.beam = v.n_fs ? p.beam : nullptr;
            v.freq = p.freq_hz;
            v.ant = p.ant_enu;
            v.hdr = dev + hoff[i];
            v.part = dev + d_part + poff[i];
            v.span = validate_span_n(v.n_fs, nblk[i]);
            v.n_src = p.n_src;
            v.n_freq = p.n_freq;
            v.n_ant = p.n_ant;
            v.nblk = nblk[i];
        }
        ValItem *tab_dev = (ValItem *)(dev + d_tab);
        FV_HIP(hipMemcpyAsync(tab_dev, tab, sizeof(ValItem) * (size_t)n, hipMemcpyHostToDevice, st));
        launch_validate_batch(tab_dev, n, max_blk, st);
        FV_HIP(hipMemcpyAsync(pin, dev, hoff[n] * sizeof(double), hipMemcpyDeviceToHost, st));
        FV_HIP(hipEventRecord(ctx->bspec.ev, st));
    }
    // the device inputs of problem i with source box `box` (centre, half-width)
    auto dev_inputs = [&](int i, const double *box) {
        const fv_problem &p = ps[i];
        DevInputs d;
        d.ant = p.ant_enu;
        d.freq = p.freq_hz;
        d.src = p.src_lmn;
        d.flux = p.flux;
        d.beam = p.beam;
        d.vis = vis[i];
        for (int a = 0; a < 3; ++a) {
            d.s_c[a] = box[a];
            d.S[a] = box[3 + a];
        }
        d.cmax = dev + d_part + poff[i];
        d.cmax_span = validate_span_n((long long)p.n_src * p.n_freq, nblk[i]);
        return d;
    };
    const unsigned f0 = n > 0 ? ps[0].flags : 0u;
    auto start = [&](fv_report &r) {
        std::memset(&r, 0, sizeof(r));
        r.fold_axis = -1;
        slot.timer.reset((f0 & (FV_TIMING | FV_TIMING_ACCUM)) != 0, (f0 & FV_TIMING_ACCUM) != 0,
                         (f0 & FV_TIMING_ONE_STAGE) ? FV_TIMING_STAGE_OF(f0) : -1);
    };
    // A batch that repeats the last one's arguments (device pointers, sizes,
    // eps, flags) is enqueued right behind its input check, planned on the last
    // batch's antenna positions, frequencies and source boxes, while the host
    // waits for the check; those (and each problem's path) are verified below
    // and the batch is enqueued again, planned on this check, on a mismatch.
    auto &bs = ctx->bspec;
    bool same = bs.valid && (int)bs.args.size() == n;
    for (int i = 0; same && i < n; ++i) {
        const fv_problem &a = bs.args[i], &p = ps[i];
        same = a.n_ant == p.n_ant && a.ant_enu == p.ant_enu && a.n_src == p.n_src && a.src_lmn == p.src_lmn &&
               a.n_freq == p.n_freq && a.freq_hz == p.freq_hz && a.flux == p.flux && a.beam == p.beam &&
               a.eps == p.eps && a.flags == p.flags && bs.vis[i] == vis[i];
    }
    bs.valid = false;  // set again below once this batch's scalars are known
    fv_report r, rs;
    std::vector<char> used;
    hipStream_t keep = slot.stream;
    slot.stream = st;
    try {
        bool ran = false;
        if (same && n > 0) {
            std::vector<fv_problem> m(ps, ps + n);
            std::vector<DevInputs> din(n);
            for (int i = 0; i < n; ++i) {
                m[i].ant_enu = bs.ant[i].data();
                m[i].freq_hz = bs.freq[i].data();
                din[i] = dev_inputs(i, bs.box[i].data());
            }
            start(rs);
            run_batch_device(ctx, slot, n, m.data(), din.data(), rs, &used);
            FV_HIP(hipEventSynchronize(bs.ev));
            ran = true;
        } else if (n > 0) {
            FV_HIP(hipEventSynchronize(bs.ev));  // nothing is computed before the check has passed
        }
        std::vector<std::vector<double>> ant(n), freq(n);
        std::vector<std::array<double, 6>> box(n);
        std::vector<int> dims(n);
        std::vector<fv_problem> meta(ps, ps + n);
        std::vector<DevInputs> in(n);
        for (int i = 0; i < n; ++i) {
            const fv_problem &p = ps[i];
            dims[i] = check_dev_scalars(p, pin + hoff[i], ant[i], freq[i], box[i].data());
            meta[i].ant_enu = ant[i].data();
            meta[i].freq_hz = freq[i].data();
            in[i] = dev_inputs(i, box[i].data());
        }
        if (ran) {
            // the speculation holds when every problem has the last batch's
            // geometry and path, and a type-3 problem also its source box
            for (int i = 0; ran && i < n; ++i) {
                const fv_problem &p = ps[i];
                const bool nufft = p.n_src > 0 && (p.flags & FV_METHOD_MASK) == FV_METHOD_NUFFT;
                int w = 0;
                const bool lat = nufft && dims[i] == 2 && !(p.flags & FV_NO_LATTICE) &&
                                 lattice_choice(ctx, meta[i], in[i], choose_prec(p.eps, p.flags), &w) != nullptr;
                ran = ant[i] == bs.ant[i] && freq[i] == bs.freq[i] && dims[i] == bs.dim[i] && lat == (used[i] != 0) &&
                      (!nufft || lat || box[i] == bs.box[i]);
            }
            if (ran) r = rs;
            else FV_HIP(hipStreamSynchronize(st));  // the speculative work is done with the workspaces
        }
        if (!ran) {
            start(r);
            run_batch_device(ctx, slot, n, meta.data(), in.data(), r, &used);
        }
        bs.args.assign(ps, ps + n);
        bs.vis.assign(vis, vis + n);
        bs.ant = std::move(ant);
        bs.freq = std::move(freq);
        bs.box = std::move(box);
        bs.dim = std::move(dims);
        bs.valid = n > 0;
    } catch (...) {
        slot.stream = keep;
        (void)hipEventRecord(slot.done, st);  // work already enqueued must finish before the workspace is reused
        throw;
    }
    slot.stream = keep;
    FV_HIP(hipEventRecord(slot.done, st));
    fill_report(slot.timer, r);
    r.method = (int)(f0 & FV_METHOD_MASK);
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

extern "C" fv_status fv_simulate_batch_dev(fv_ctx *ctx, int n_snap, const fv_problem *snaps, double *const *vis,
                                           void *stream, fv_report *rep) {
    try {
        if (!ctx || n_snap < 0 || (n_snap > 0 && (!snaps || !vis))) fv::fail(FV_EINVAL, "null argument");
        fv::simulate_batch_dev(ctx, n_snap, snaps, vis, (hipStream_t)stream, rep);
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
