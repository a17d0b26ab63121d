// Context, device memory, validation and the C ABI entry points (the serving
// entry points live in server.cpp, the batch entry point in batch.cpp).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ctx.h"
#include "fv_internal.h"

namespace fv {

static thread_local std::string g_last_error;

[[noreturn]] void fail(fv_status code, const std::string &msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        (void)hipGetLastError();  // clear the sticky per-thread error where possible
        fail(FV_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
}

void set_last_error(const std::string &msg) { g_last_error = msg; }
const char *last_error_cstr() { return g_last_error.c_str(); }

void *Arena::take(size_t bytes, size_t align) {
    size_t off = (used + align - 1) / align * align;
    if (off + bytes > cap) fail(FV_ENOMEM, "workspace arena overflow");
    used = off + bytes;
    return base + off;
}

void *PinnedBuf::get(size_t bytes) {
    wait();
    if (bytes > cap) {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        const size_t want = std::max<size_t>(bytes, 4096);
        FV_HIP(hipHostMalloc(&p, want, hipHostMallocDefault));
        cap = want;
    }
    return p;
}

void PinnedBuf::record(hipStream_t s) {
    if (!ev) FV_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    FV_HIP(hipEventRecord(ev, s));
    pending = true;
}

void PinnedBuf::wait() {
    if (pending) {
        pending = false;
        FV_HIP(hipEventSynchronize(ev));
    }
}

void PinnedBuf::release() {
    if (pending && ev) (void)hipEventSynchronize(ev);
    pending = false;
    if (p) (void)hipHostFree(p);
    if (ev) (void)hipEventDestroy(ev);
    p = nullptr;
    ev = nullptr;
    cap = 0;
}

void Arena::ensure(size_t bytes) {
    if (bytes <= cap) return;
    release();
    tables.clear();
    ipsi = false;
    size_t want = std::max(bytes, cap + cap / 2);
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        e = hipMalloc(&p, bytes);
        want = bytes;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(FV_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    base = (char *)p;
    cap = want;
    used = 0;
}

void Arena::release() {
    if (base) (void)hipFree(base);
    base = nullptr;
    cap = used = 0;
}

void TargetTable::release() {
    if (tb) (void)hipFree(tb);
    if (tidx) (void)hipFree(tidx);
    if (tphi) (void)hipFree(tphi);
    tb = tphi = nullptr;
    tidx = nullptr;
}

void ensure_lds(const void *fn, size_t bytes) {
    if (bytes <= 65536) return;
    int dev = 0;
    FV_HIP(hipGetDevice(&dev));
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, size_t> set;
    std::lock_guard<std::mutex> lk(mu);
    size_t &have = set[{fn, dev}];
    if (have >= bytes) return;
    FV_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    have = bytes;
}

void StageTimer::reset(bool enable, bool accum_mode, int only_stage) {
    on = enable;
    only = only_stage;
    for (int i = 0; i < FV_NSTAGE; ++i) {
        ms[i] = bytes[i] = 0;
        launches[i] = 0;
    }
    if (!(accum_mode && accum)) {  // a new sum starts unless one is running
        marks.clear();
        used = 0;
        calls = 0;
    }
    accum = accum_mode;
    if (accum) ++calls;
    cur = -1;
}

void StageTimer::take(double *ms_out, int *launches_out, int *calls_out) {
    double sum[FV_NSTAGE] = {0};
    int cnt[FV_NSTAGE] = {0};
    if (!marks.empty()) {
        FV_HIP(hipEventSynchronize(marks.back().b));
        for (auto &m : marks) {
            float t = 0;
            FV_HIP(hipEventElapsedTime(&t, m.a, m.b));
            sum[m.stage] += t;
            cnt[m.stage] += 1;
        }
    }
    for (int i = 0; i < FV_NSTAGE; ++i) {
        if (ms_out) ms_out[i] = sum[i];
        if (launches_out) launches_out[i] = cnt[i];
    }
    if (calls_out) *calls_out = calls;
    marks.clear();
    used = 0;
    calls = 0;
    accum = false;
}

void StageTimer::begin(int stage, hipStream_t s) {
    if (!on || (only >= 0 && stage != only)) return;
    if (used + 2 > pool.size()) {
        for (int i = 0; i < 16; ++i) {
            hipEvent_t e;
            // timestamps only: no system-scope fence (the data the stages write
            // is made visible by the caller's own synchronisation)
            FV_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
            pool.push_back(e);
        }
    }
    cur = stage;
    cur_a = pool[used++];
    FV_HIP(hipEventRecord(cur_a, s));
}

void StageTimer::kernel_events(int stage, hipEvent_t *a, hipEvent_t *b) {
    *a = *b = nullptr;
    if (!on || (only >= 0 && stage != only)) return;
    if (used + 2 > pool.size()) {
        for (int i = 0; i < 16; ++i) {
            hipEvent_t e;
            FV_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
            pool.push_back(e);
        }
    }
    *a = pool[used++];
    *b = pool[used++];
    marks.push_back({stage, *a, *b});
}

void StageTimer::end(hipStream_t s) {
    if (!on || cur < 0) return;
    hipEvent_t b = pool[used++];
    FV_HIP(hipEventRecord(b, s));
    marks.push_back({cur, cur_a, b});
    cur = -1;
}

void StageTimer::collect() {
    if (!on || accum || marks.empty()) return;
    FV_HIP(hipEventSynchronize(marks.back().b));
    for (auto &m : marks) {
        float t = 0;
        FV_HIP(hipEventElapsedTime(&t, m.a, m.b));
        ms[m.stage] += t;
    }
    marks.clear();
    used = 0;
}

StageTimer::~StageTimer() {
    for (auto e : pool) (void)hipEventDestroy(e);
}

// ---------------------------------------------------------------------------
// Cache-key hash (FNV-1a style, over 8-byte words, then the tail bytes).
static uint64_t fnv1a(const void *p, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char *c = (const unsigned char *)p;
    size_t i = 0;
    for (; i + 8 <= n; i += 8) {
        uint64_t w;
        std::memcpy(&w, c + i, 8);
        h ^= w;
        h *= 1099511628211ull;
        h ^= h >> 29;
    }
    for (; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

Slot::~Slot() {
    graphs.release();
    arena.host.release();
    inputs.host.release();
    lat.host.release();
    pin.release();
    arena.release();
    inputs.release();
    lat.release();
    if (done) (void)hipEventDestroy(done);
    if (stream && own_stream) (void)hipStreamDestroy(stream);
}

}  // namespace fv

using namespace fv;

fv_ctx::~fv_ctx() {
    fv::server_free(server);
    server = nullptr;
    targets.clear();
    cache.release();
    plan_pin.release();
    if (scalar_buf) (void)hipFree(scalar_buf);
}

namespace fv {

static size_t device_free_bytes() {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return fr;
}

// Geometry plan with a cache of the pair extents per (array bytes, dim).
GeomPlan ctx_geometry(fv_ctx *ctx, const double *ant_host, int n_ant, int dim, double eps, const double *s_c,
                      const double *S, bool fold) {
    std::lock_guard<std::mutex> lk(ctx->geo_mu);
    uint64_t key = fnv1a(ant_host, sizeof(double) * 3 * (size_t)n_ant);
    key = fnv1a(&dim, sizeof(dim), key);
    key = fnv1a(&fold, sizeof(fold), key);
    key = fnv1a(S, sizeof(double) * 3, key);
    int w = kernel_width(eps);
    key = fnv1a(&w, sizeof(w), key);
    for (auto &e : ctx->geos)
        if (e.first == key) {
            GeomPlan g = e.second;
            for (int a = 0; a < 3; ++a) { g.s_c[a] = s_c[a]; g.S[a] = S[a]; }
            return g;
        }
    GeomPlan g = plan_geometry(ant_host, n_ant, dim, eps, s_c, S, fold);
    ctx->geos.push_back({key, g});
    if (ctx->geos.size() > 64) ctx->geos.erase(ctx->geos.begin());
    return g;
}

// Target table for (array, dim, fold axis, w), built on the device and cached;
// with `scales`, the table of all pairs at each of those frequency ratios.
std::shared_ptr<TargetTable> ctx_targets(fv_ctx *ctx, const double *ant_host, const double *ant_dev,
                                         const GeomPlan &g, hipStream_t st, const std::vector<double> *scales) {
    std::lock_guard<std::mutex> lk(ctx->geo_mu);
    uint64_t key = fnv1a(ant_host, sizeof(double) * 3 * (size_t)g.n_ant);
    key = fnv1a(&g.dim, sizeof(int), key);
    key = fnv1a(&g.fold_axis, sizeof(int), key);
    key = fnv1a(&g.w, sizeof(int), key);
    key = fnv1a(g.b_c, sizeof(double) * 3, key);
    key = fnv1a(g.B, sizeof(double) * 3, key);
    const int n_scale = scales ? (int)scales->size() : 1;
    if (scales) key = fnv1a(scales->data(), sizeof(double) * scales->size(), key ^ 0x9e3779b97f4a7c15ull);
    for (auto it = ctx->targets.begin(); it != ctx->targets.end(); ++it)
        if ((*it)->key == key) {
            auto t = *it;
            ctx->targets.erase(it);
            ctx->targets.push_back(t);  // most recently used at the back
            return t;
        }
    if (ctx->targets.size() >= 64) ctx->targets.pop_front();  // freed when its last user drops it
    std::shared_ptr<TargetTable> t(new TargetTable, [](TargetTable *x) {
        x->release();
        delete x;
    });
    t->key = key;
    t->dim = g.dim;
    t->w = g.w;
    t->fold_axis = g.fold_axis;
    t->n_ant = g.n_ant;
    t->n_tgt = g.n_pairs * n_scale;
    const size_t n = (size_t)std::max<long long>(t->n_tgt, 1);
    FV_HIP(hipMalloc((void **)&t->tb, n * g.dim * sizeof(double)));
    FV_HIP(hipMalloc((void **)&t->tidx, n * sizeof(int)));
    FV_HIP(hipMalloc((void **)&t->tphi, n * g.dim * sizeof(double)));
    const double *qn = ctx->cache.quad(g.w, st);
    const std::vector<int> order = target_order(ant_host, g);
    int *perm_dev = nullptr;
    // the pair order, then the frequency ratios
    FV_HIP(hipMalloc((void **)&perm_dev, order.size() * sizeof(int) + (size_t)n_scale * sizeof(double) + 16));
    double *scale_dev = (double *)((char *)perm_dev + (order.size() * sizeof(int) + 15) / 16 * 16);
    hipError_t e = hipMemcpyAsync(perm_dev, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && scales)
        e = hipMemcpyAsync(scale_dev, scales->data(), sizeof(double) * n_scale, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        try {
            if (scales)
                build_targets_multi(ant_dev, g.n_ant, g.dim, g.fold_axis, g.b_c, g.B, g.w, qn, perm_dev, scale_dev,
                                    n_scale, *t, st);
            else
                build_targets(ant_dev, g.n_ant, g.dim, g.fold_axis, g.b_c, g.B, g.w, qn, perm_dev, *t, st);
        } catch (...) {
            (void)hipStreamSynchronize(st);
            (void)hipFree(perm_dev);
            throw;
        }
        // built once per array; later users may run on other streams
        e = hipStreamSynchronize(st);
    }
    (void)hipFree(perm_dev);
    FV_HIP(e);
    ctx->targets.push_back(t);
    return t;
}

// Host-side validation of a problem whose arrays are host memory.
void validate_host(const fv_problem *p) {
    if (!p) fail(FV_EINVAL, "null problem");
    if (p->n_ant < 1 || p->n_src < 0 || p->n_freq < 1) fail(FV_EINVAL, "bad sizes");
    if (!p->ant_enu || !p->freq_hz) fail(FV_EINVAL, "null antenna or frequency array");
    if (p->n_src > 0 && (!p->src_lmn || !p->flux)) fail(FV_EINVAL, "null source or flux array");
    if (!(p->eps >= 1e-14 && p->eps <= 1e-1)) fail(FV_EINVAL, "eps out of [1e-14, 1e-1]");
    for (long long i = 0; i < 3LL * p->n_ant; ++i)
        if (!std::isfinite(p->ant_enu[i])) fail(FV_EINVAL, "non-finite antenna position");
    for (int f = 0; f < p->n_freq; ++f)
        if (!(std::isfinite(p->freq_hz[f]) && p->freq_hz[f] > 0)) fail(FV_EINVAL, "frequency must be finite and > 0");
    for (int j = 0; j < p->n_src; ++j) {
        const double *s = p->src_lmn + 3 * (size_t)j;
        if (!(std::isfinite(s[0]) && std::isfinite(s[1]) && std::isfinite(s[2])))
            fail(FV_EINVAL, "non-finite source direction");
        double r = std::sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
        if (std::fabs(r - 1.0) > 1e-9) fail(FV_EINVAL, "source direction is not a unit vector");
    }
    const long long nfs = (long long)p->n_freq * p->n_src;
    for (long long i = 0; i < nfs; ++i)
        if (!std::isfinite(p->flux[i])) fail(FV_EINVAL, "non-finite flux");
    if (p->beam)
        for (long long i = 0; i < nfs; ++i)
            if (!std::isfinite(p->beam[i])) fail(FV_EINVAL, "non-finite beam");
    unsigned m = p->flags & FV_METHOD_MASK;
    if (m != FV_METHOD_NUFFT && m != FV_METHOD_DIRECT && m != FV_METHOD_MFMA) fail(FV_EINVAL, "unknown method");
    if ((p->flags & FV_DIM_MASK) == FV_DIM_MASK) fail(FV_EINVAL, "both 2-D and 3-D forced");
    if ((p->flags & FV_PREC_MASK) == FV_PREC_MASK) fail(FV_EINVAL, "both FP32 and FP64 forced");
    if ((p->flags & FV_PREC_MASK) == FV_PREC_FP32 && p->eps < 1e-6) fail(FV_EUNSUPPORTED, "FP32 grids need eps >= 1e-6");
}

std::shared_ptr<LatticePlan> ctx_lattice(fv_ctx *ctx, const double *ant_host, int n_ant, double tol, int w) {
    std::lock_guard<std::mutex> lk(ctx->geo_mu);
    uint64_t key = fnv1a(ant_host, sizeof(double) * 3 * (size_t)n_ant);
    key = fnv1a(&tol, sizeof(tol), key);
    key = fnv1a(&w, sizeof(w), key);
    for (auto &e : ctx->lattices)
        if (e.first == key) return e.second;
    std::shared_ptr<LatticePlan> lp(new LatticePlan);
    if (!find_lattice(ant_host, n_ant, tol, lp.get()))
        lp.reset();
    else if (lattice_fits(*lp, 64, w))
        lattice_tables(*lp, w);
    ctx->lattices.push_back({key, lp});
    if (ctx->lattices.size() > 64) ctx->lattices.erase(ctx->lattices.begin());
    return lp;
}

std::shared_ptr<LatticePlan> lattice_choice(fv_ctx *ctx, const fv_problem &p, const DevInputs &in, int prec, int *w_out) {
    double numax = 0.0;
    for (int f = 0; f < p.n_freq; ++f) numax = std::max(numax, p.freq_hz[f]);
    const double tol = p.eps * kCLight / (20.0 * M_PI * numax);
    const int w = kernel_width_type1(p.eps);
    std::shared_ptr<LatticePlan> lp = ctx_lattice(ctx, p.ant_enu, p.n_ant, tol, w);
    if (!lp || !lattice_fits(*lp, prec, w)) return nullptr;
    int nf[2];
    lattice_grid(*lp, w, nf);
    GeomPlan g = ctx_geometry(ctx, p.ant_enu, p.n_ant, 2, p.eps, in.s_c, in.S, !(p.flags & FV_NO_FOLD));
    const SnapPlan top = plan_snapshot(g, numax);
    if ((double)nf[0] * nf[1] > (double)top.n1[0] * top.n1[1]) return nullptr;
    *w_out = w;
    return lp;
}

bool run_lattice(fv_ctx *ctx, Slot &slot, const fv_problem &p, const DevInputs &in, double *vis_dev, int prec,
                 StageTimer *tm, fv_report &r) {
    int w = 0;
    std::shared_ptr<LatticePlan> lp = lattice_choice(ctx, p, in, prec, &w);
    if (!lp) return false;
    int nf[2];
    lattice_grid(*lp, w, nf);
    const size_t need = lattice_work_bytes(*lp, p.n_src, p.n_freq, p.n_ant, prec, w);
    slot.arena.ensure(need);
    slot.arena.reset();
    void *work = slot.arena.take(need);
    r.model_bytes += launch_lattice(*lp, in.src, p.n_src, in.freq, p.n_freq, in.flux, in.beam, in.cmax,
                                    in.cmax_span, p.n_ant, prec, w, vis_dev, work, slot.stream, tm);
    r.lattice = 1;
    r.w = w;
    r.n1[0] = nf[0];
    r.n1[1] = nf[1];
    r.n2[0] = nf[0];
    r.n2[1] = nf[1];
    return true;
}

// NUFFT jobs (one per frequency) of one problem whose inputs are on the
// device; keeps the target table alive through `hold`.
NufftGroupKey append_jobs(fv_ctx *ctx, const fv_problem &p, const DevInputs &in, double *vis_dev, hipStream_t st,
                          std::vector<SnapJob> &jobs, std::vector<std::shared_ptr<TargetTable>> &hold,
                          SnapPlan *top) {
    const int n_freq = p.n_freq, n_src = p.n_src;
    const long long n_pairs = (long long)p.n_ant * (p.n_ant + 1) / 2;
    NufftGroupKey k;
    k.dim = choose_dim(p.ant_enu, p.n_ant, p.eps, p.freq_hz, n_freq, p.flags);
    k.flags = p.flags & (FV_AUTOTUNE | FV_GRAPH | FV_DETERMINISTIC);
    k.prec = choose_prec(p.eps, p.flags);
    const bool fold = !(p.flags & FV_NO_FOLD);
    GeomPlan g = ctx_geometry(ctx, p.ant_enu, p.n_ant, k.dim, p.eps, in.s_c, in.S, fold);
    k.w = g.w;
    k.fold_axis = g.fold_axis;
    std::shared_ptr<TargetTable> tt = ctx_targets(ctx, p.ant_enu, in.ant, g, st);
    hold.push_back(tt);
    int best_f = 0;
    for (int f = 0; f < n_freq; ++f) {
        SnapJob j;
        j.plan = plan_snapshot(g, p.freq_hz[f]);
        j.src = in.src;
        j.n_src = n_src;
        j.flux = in.flux + (size_t)f * n_src;
        j.beam = in.beam ? in.beam + (size_t)f * n_src : nullptr;
        j.out = vis_dev + 2 * (size_t)f * n_pairs;
        j.tt = tt.get();
        jobs.push_back(j);
        if (p.freq_hz[f] > p.freq_hz[best_f]) best_f = f;
    }
    if (top) *top = jobs[jobs.size() - n_freq + best_f].plan;
    return k;
}

// Runs jobs of one (dim, precision, w) in groups whose workspace fits the
// context's chunk size; returns the algorithmic bytes of the grid stages.
double execute_jobs(fv_ctx *ctx, Slot &slot, const std::vector<SnapJob> &jobs, const NufftGroupKey &k,
                    StageTimer *tm) {
    hipStream_t st = slot.stream;
    ExecOpts opts;
    opts.autotune = (k.flags & FV_AUTOTUNE) != 0;
    opts.graph = (k.flags & FV_GRAPH) != 0;
    opts.det = (k.flags & FV_DETERMINISTIC) != 0;
    opts.tunes = &ctx->tunes;
    opts.graphs = &slot.graphs;
    const size_t cap = std::max<size_t>(ctx->chunk_bytes, 1 << 20);
    // one launch group when everything fits (the usual case); else groups of
    // frequencies sized job by job
    opts.cap = cap;
    bool too_big = false;
    const double b1 = nufft_execute(jobs, k.dim, k.prec, k.w, slot.arena, ctx->cache, st, tm, &opts, &too_big);
    if (!too_big) return b1;
    opts.cap = 0;
    std::vector<size_t> each(jobs.size());
    for (size_t i = 0; i < jobs.size(); ++i)
        each[i] = nufft_workspace_bytes(std::vector<SnapJob>{jobs[i]}, k.dim, k.prec, k.w, opts.det);
    double bytes = 0.0;
    size_t i0 = 0;
    while (i0 < jobs.size()) {
        size_t i1 = i0 + 1, tot = each[i0];
        while (i1 < jobs.size() && tot + each[i1] <= cap) tot += each[i1++];
        std::vector<SnapJob> part(jobs.begin() + i0, jobs.begin() + i1);
        if (i0 > 0) FV_HIP(hipStreamSynchronize(st));  // the arena is reused
        bytes += nufft_execute(part, k.dim, k.prec, k.w, slot.arena, ctx->cache, st, tm, &opts);
        i0 = i1;
    }
    return bytes;
}

// Direct-sum methods of one problem.
void run_direct(fv_ctx *ctx, Slot &slot, const fv_problem &p, const DevInputs &in, double *vis_dev, int dim,
                int prec, StageTimer *tm) {
    const unsigned method = p.flags & FV_METHOD_MASK;
    hipStream_t st = slot.stream;
    if (method == FV_METHOD_DIRECT) {
        launch_direct(in.ant, p.n_ant, in.src, p.n_src, p.freq_hz, p.n_freq, in.flux, in.beam, dim, prec, vis_dev,
                      st, tm);
    } else {
        const size_t cap = std::max<size_t>(ctx->chunk_bytes, 1 << 20);
        const size_t need = zz_work_bytes(p.n_ant, p.n_src, prec, cap);
        slot.arena.ensure(need);
        slot.arena.reset();
        void *work = slot.arena.take(need);
        launch_zz(in.ant, p.n_ant, in.src, p.n_src, p.freq_hz, p.n_freq, in.flux, in.beam, dim, prec, vis_dev, work,
                  cap, st, tm);
    }
}

void accumulate_report(const fv_report &a, fv_report &r, bool first) {
    if (first) {
        const double keep_pairs = r.src_pairs;
        r = a;
        r.src_pairs = keep_pairs + a.src_pairs;
        return;
    }
    r.src_pairs += a.src_pairs;
    r.model_bytes += a.model_bytes;
    for (int i = 0; i < FV_NSTAGE; ++i) {
        r.t_stage_ms[i] += a.t_stage_ms[i];
        r.stage_bytes[i] += a.stage_bytes[i];
        r.stage_launches[i] += a.stage_launches[i];
    }
    r.lattice = std::max(r.lattice, a.lattice);
}

void fill_report(StageTimer &tm, fv_report &r) {
    tm.collect();
    for (int i = 0; i < FV_NSTAGE; ++i) {
        r.t_stage_ms[i] = tm.ms[i];
        r.stage_bytes[i] = tm.bytes[i];
        r.stage_launches[i] = tm.launches[i];
    }
}

int check_dev_scalars(const fv_problem &p, const double *hdr, std::vector<double> &ant, std::vector<double> &freq,
                      double box[6]) {
    const double *pf = hdr + 8, *pa = pf + p.n_freq;
    freq.assign(pf, pf + p.n_freq);
    ant.assign(pa, pa + 3 * (size_t)p.n_ant);
    for (double a : ant)
        if (!std::isfinite(a)) fail(FV_EINVAL, "non-finite antenna position");
    for (double f : freq)
        if (!(std::isfinite(f) && f > 0)) fail(FV_EINVAL, "frequency must be finite and > 0");
    if (p.n_src > 0 && (hdr[6] != 0.0 || hdr[7] != 0.0)) fail(FV_EINVAL, "invalid source directions or strengths");
    if ((p.flags & FV_PREC_MASK) == FV_PREC_FP32 && p.eps < 1e-6) fail(FV_EUNSUPPORTED, "FP32 grids need eps >= 1e-6");
    const int dim = choose_dim(ant.data(), p.n_ant, p.eps, freq.data(), p.n_freq, p.flags);
    for (int a = 0; a < 6; ++a) box[a] = 0.0;
    if (p.n_src > 0)
        for (int a = 0; a < dim; ++a) {
            box[a] = 0.5 * (hdr[2 * a] + hdr[2 * a + 1]);
            box[3 + a] = 0.5 * (hdr[2 * a + 1] - hdr[2 * a]);
        }
    return dim;
}

void check_dev_args(const fv_problem &p, const double *vis) {
    if (!vis) fail(FV_EINVAL, "null output pointer");
    if ((uintptr_t)vis & 15) fail(FV_EINVAL, "the output must be 16-byte aligned");
    if (p.n_ant < 1 || p.n_src < 0 || p.n_freq < 1) fail(FV_EINVAL, "bad sizes");
    if (!p.ant_enu || !p.freq_hz || (p.n_src > 0 && (!p.src_lmn || !p.flux))) fail(FV_EINVAL, "null device array");
    if (!(p.eps >= 1e-14 && p.eps <= 1e-1)) fail(FV_EINVAL, "eps out of [1e-14, 1e-1]");
}

void simulate_dev_sync(fv_ctx *ctx, Slot &slot, const fv_problem &p, double *vis, fv_report *rep) {
    auto t0 = std::chrono::steady_clock::now();
    check_dev_args(p, vis);
    FV_HIP(hipSetDevice(ctx->device));
    hipStream_t st = slot.stream;
    const size_t nval = validate_doubles(p.n_ant, p.n_freq), nhdr = 8 + (size_t)p.n_freq + 3 * (size_t)p.n_ant;
    slot.inputs.ensure(nval * sizeof(double) + 256);
    slot.inputs.reset();
    double *dev = (double *)slot.inputs.take(nval * sizeof(double));
    double *pin = (double *)slot.pin.get(nhdr * sizeof(double));
    launch_validate(p.src_lmn, p.n_src, p.flux, p.beam, p.n_freq, p.ant_enu, p.n_ant, p.freq_hz, dev, st);
    FV_HIP(hipMemcpyAsync(pin, dev, nhdr * sizeof(double), hipMemcpyDeviceToHost, st));
    FV_HIP(hipStreamSynchronize(st));
    std::vector<double> ant, freq;
    double box[6];
    check_dev_scalars(p, pin, ant, freq, box);
    fv_problem meta = p;
    meta.ant_enu = ant.data();
    meta.freq_hz = freq.data();
    DevInputs in;
    in.ant = p.ant_enu;
    in.freq = p.freq_hz;
    in.src = p.src_lmn;
    in.flux = p.flux;
    in.beam = p.beam;
    in.vis = vis;
    for (int a = 0; a < 3; ++a) {
        in.s_c[a] = box[a];
        in.S[a] = box[3 + a];
    }
    in.cmax = validate_partials(dev, p.n_ant, p.n_freq);
    in.cmax_span = validate_span((long long)p.n_src * p.n_freq);
    fv_report r;
    run_device(ctx, slot, meta, in, vis, &r);
    FV_HIP(hipStreamSynchronize(st));
    r.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = r;
}

// Everything the device path needs once the inputs are on the device and the
// planning scalars (antenna positions, frequencies, source box) on the host.
void run_device(fv_ctx *ctx, Slot &slot, const fv_problem &host_meta, const DevInputs &in, double *vis_dev,
                fv_report *rep) {
    const fv_problem *p = &host_meta;
    const int n_ant = p->n_ant, n_freq = p->n_freq, n_src = p->n_src;
    const long long n_pairs = (long long)n_ant * (n_ant + 1) / 2;
    hipStream_t st = slot.stream;
    const unsigned method = p->flags & FV_METHOD_MASK;
    const int dim = choose_dim(p->ant_enu, n_ant, p->eps, p->freq_hz, n_freq, p->flags);
    const int prec = choose_prec(p->eps, p->flags);
    fv_report r;
    std::memset(&r, 0, sizeof(r));
    StageTimer &tm = slot.timer;
    tm.reset((p->flags & (FV_TIMING | FV_TIMING_ACCUM)) != 0, (p->flags & FV_TIMING_ACCUM) != 0,
             (p->flags & FV_TIMING_ONE_STAGE) ? FV_TIMING_STAGE_OF(p->flags) : -1);
    r.dim = dim;
    r.prec_bits = prec;
    r.method = (int)method;
    r.fold_axis = -1;
    r.src_pairs = (double)n_src * (double)n_pairs * (double)n_freq;
    if (n_src == 0) {
        launch_zero_c128(vis_dev, n_pairs * n_freq, st);
    } else if (method != FV_METHOD_NUFFT) {
        run_direct(ctx, slot, *p, in, vis_dev, dim, prec, &tm);
    } else if (dim == 2 && !(p->flags & FV_NO_LATTICE) && run_lattice(ctx, slot, *p, in, vis_dev, prec, &tm, r)) {
        // type-1 path done
    } else {
        std::vector<SnapJob> jobs;
        std::vector<std::shared_ptr<TargetTable>> hold;
        SnapPlan top;
        NufftGroupKey k = append_jobs(ctx, *p, in, vis_dev, st, jobs, hold, &top);
        r.model_bytes = execute_jobs(ctx, slot, jobs, k, &tm);
        r.prec_bits = k.prec;
        r.w = k.w;
        r.fold_axis = k.fold_axis;
        for (int a = 0; a < 3; ++a) {
            r.n1[a] = top.n1[a];
            r.n2[a] = top.n2[a];
        }
    }
    FV_HIP(hipGetLastError());
    fill_report(tm, r);
    if (rep) *rep = r;
}

DevInputs upload(Slot &slot, const fv_problem *p, double *s_c, double *S) {
    const int n_ant = p->n_ant, n_src = p->n_src, n_freq = p->n_freq;
    const size_t b_ant = sizeof(double) * 3 * n_ant, b_src = sizeof(double) * 3 * (size_t)n_src;
    const size_t b_fs = sizeof(double) * (size_t)n_freq * n_src;
    const long long n_pairs = (long long)n_ant * (n_ant + 1) / 2;
    const size_t b_vis = sizeof(double) * 2 * (size_t)n_pairs * n_freq;
    const size_t b_freq = sizeof(double) * (size_t)n_freq;
    slot.inputs.ensure(b_ant + b_freq + b_src + 2 * b_fs + b_vis + 8 * 256);
    slot.inputs.reset();
    DevInputs in;
    in.ant = (double *)slot.inputs.take(b_ant);
    in.freq = (double *)slot.inputs.take(b_freq);
    in.src = n_src ? (double *)slot.inputs.take(b_src) : nullptr;
    in.flux = n_src ? (double *)slot.inputs.take(b_fs) : nullptr;
    in.beam = (n_src && p->beam) ? (double *)slot.inputs.take(b_fs) : nullptr;
    in.vis = (double *)slot.inputs.take(b_vis);
    hipStream_t st = slot.stream;
    FV_HIP(hipMemcpyAsync((void *)in.ant, p->ant_enu, b_ant, hipMemcpyHostToDevice, st));
    FV_HIP(hipMemcpyAsync((void *)in.freq, p->freq_hz, b_freq, hipMemcpyHostToDevice, st));
    if (n_src) {
        FV_HIP(hipMemcpyAsync((void *)in.src, p->src_lmn, b_src, hipMemcpyHostToDevice, st));
        FV_HIP(hipMemcpyAsync((void *)in.flux, p->flux, b_fs, hipMemcpyHostToDevice, st));
        if (p->beam) FV_HIP(hipMemcpyAsync((void *)in.beam, p->beam, b_fs, hipMemcpyHostToDevice, st));
    }
    const int dim = choose_dim(p->ant_enu, n_ant, p->eps, p->freq_hz, n_freq, p->flags);
    src_box(p->src_lmn, n_src, dim, s_c, S);
    for (int a = 0; a < 3; ++a) {
        in.s_c[a] = s_c[a];
        in.S[a] = S[a];
    }
    return in;
}

void simulate_host(fv_ctx *ctx, Slot &slot, const fv_problem *p, double *vis, fv_report *rep) {
    auto t0 = std::chrono::steady_clock::now();
    validate_host(p);
    FV_HIP(hipSetDevice(ctx->device));
    if (slot.done) FV_HIP(hipStreamWaitEvent(slot.stream, slot.done, 0));  // a device-entry call's work
    double s_c[3], S[3];
    DevInputs in = upload(slot, p, s_c, S);
    fv_report r;
    run_device(ctx, slot, *p, in, in.vis, &r);
    const long long n_pairs = (long long)p->n_ant * (p->n_ant + 1) / 2;
    FV_HIP(hipMemcpyAsync(vis, in.vis, sizeof(double) * 2 * (size_t)n_pairs * p->n_freq, hipMemcpyDeviceToHost,
                          slot.stream));
    FV_HIP(hipStreamSynchronize(slot.stream));
    r.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = r;
}

}  // namespace fv

// ===========================================================================
// C ABI
// ===========================================================================
#define FV_GUARD_BEGIN try {
#define FV_GUARD_END                                   \
    }                                                  \
    catch (const fv::Error &e) {                       \
        fv::set_last_error(e.msg);                     \
        return e.code;                                 \
    }                                                  \
    catch (const std::bad_alloc &) {                   \
        fv::set_last_error("host allocation failed");  \
        return FV_ENOMEM;                              \
    }                                                  \
    catch (const std::exception &e) {                  \
        fv::set_last_error(e.what());                  \
        return FV_EDEVICE;                             \
    }                                                  \
    catch (...) {                                      \
        fv::set_last_error("unknown failure");         \
        return FV_EDEVICE;                             \
    }

extern "C" {

fv_status fv_create(int device, size_t hbm_budget_bytes, fv_ctx **out) {
    FV_GUARD_BEGIN
    if (!out) fv::fail(FV_EINVAL, "null output pointer");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) {
        (void)hipGetLastError();
        fv::fail(FV_EDEVICE, "no HIP device");
    }
    if (device < 0 || device >= n) fv::fail(FV_EINVAL, "device index out of range");
    FV_HIP(hipSetDevice(device));
    fv_ctx *c = new fv_ctx();
    c->device = device;
    size_t fr = fv::device_free_bytes();
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * fr);
    c->chunk_bytes = std::max<size_t>(c->budget / 4, std::min<size_t>(c->budget, 256u << 20));
    hipError_t e = hipStreamCreateWithFlags(&c->main.stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete c;
        FV_HIP(e);
    }
    c->main.own_stream = true;
    *out = c;
    return FV_OK;
    FV_GUARD_END
}

void fv_destroy(fv_ctx *ctx) {
    if (!ctx) return;
    try {
        fv_server_stop(ctx);
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        if (ctx->spec.ev) (void)hipEventDestroy(ctx->spec.ev);
        if (ctx->bspec.ev) (void)hipEventDestroy(ctx->bspec.ev);
        if (ctx->side_fork) (void)hipEventDestroy(ctx->side_fork);
        if (ctx->side) (void)hipStreamDestroy(ctx->side);
    } catch (...) {
    }
    delete ctx;
}

const char *fv_last_error(void) { return fv::last_error_cstr(); }

fv_status fv_simulate(fv_ctx *ctx, const fv_problem *p, double *vis, fv_report *rep) {
    FV_GUARD_BEGIN
    if (!ctx || !vis) fv::fail(FV_EINVAL, "null context or output");
    fv::simulate_host(ctx, ctx->main, p, vis, rep);
    return FV_OK;
    FV_GUARD_END
}

fv_status fv_simulate_dev(fv_ctx *ctx, const fv_problem *p, double *vis, void *stream, fv_report *rep) {
    FV_GUARD_BEGIN
    auto t0 = std::chrono::steady_clock::now();
    if (!ctx || !p || !vis) fv::fail(FV_EINVAL, "null argument");
    fv::check_dev_args(*p, vis);
    FV_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    // input check and planning scalars in one pass, one copy through pinned
    // staging: [check 8][freq][ant]
    const size_t n_ant3 = 3 * (size_t)p->n_ant;
    const size_t nscal = 8 + (size_t)p->n_freq + n_ant3;
    fv::Slot &slot = ctx->main;
    if (!slot.done) FV_HIP(hipEventCreateWithFlags(&slot.done, hipEventDisableTiming));
    FV_HIP(hipStreamWaitEvent(st, slot.done, 0));  // the previous call (any stream) is done with the workspace
    double *pin = (double *)ctx->plan_pin.get(nscal * sizeof(double));
    double *dev = ctx->scalars(fv::validate_doubles(p->n_ant, p->n_freq));
    auto &sp = ctx->spec;
    const void *ptrs[5] = {p->ant_enu, p->freq_hz, p->src_lmn, p->flux, p->beam};
    const bool speculate = sp.valid && std::memcmp(sp.ptr, ptrs, sizeof(ptrs)) == 0 && sp.n_ant == p->n_ant &&
                           sp.n_freq == p->n_freq && sp.n_src == p->n_src && sp.eps == p->eps && sp.flags == p->flags;
    sp.valid = false;  // set again below once this call's scalars are known
    if (!sp.ev) FV_HIP(hipEventCreateWithFlags(&sp.ev, hipEventDisableTiming));
    // A repeated call whose last path was type 3 runs its input check on the
    // context's side stream, beside the speculative transform: type 3 reads
    // nothing the check writes.  The caller's stream joins the check before
    // anything that may read it (a path change after the check) and before
    // the call ends.
    const bool side = speculate && !sp.lattice;
    hipStream_t vs = st;
    if (side) {
        if (!ctx->side) FV_HIP(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
        if (!ctx->side_fork) FV_HIP(hipEventCreateWithFlags(&ctx->side_fork, hipEventDisableTiming));
        FV_HIP(hipEventRecord(ctx->side_fork, st));  // after the wait for the previous call
        FV_HIP(hipStreamWaitEvent(ctx->side, ctx->side_fork, 0));
        vs = ctx->side;
    }
    fv::launch_validate(p->src_lmn, p->n_src, p->flux, p->beam, p->n_freq, p->ant_enu, p->n_ant, p->freq_hz, dev,
                        vs);
    FV_HIP(hipMemcpyAsync(pin, dev, nscal * sizeof(double), hipMemcpyDeviceToHost, vs));
    if (speculate) FV_HIP(hipEventRecord(sp.ev, vs));  // the check's copy
    // the device inputs; the source box is filled from the host-side check
    auto dev_inputs = [&](const double *box) {
        fv::DevInputs in;
        in.ant = p->ant_enu;
        in.freq = p->freq_hz;
        in.src = p->src_lmn;
        in.flux = p->flux;
        in.beam = p->beam;
        in.vis = vis;
        for (int a = 0; a < 3; ++a) {
            in.s_c[a] = box[a];
            in.S[a] = box[3 + a];
        }
        in.cmax = fv::validate_partials(dev, p->n_ant, p->n_freq);
        in.cmax_span = fv::validate_span((long long)p->n_src * p->n_freq);
        return in;
    };
    hipStream_t keep = slot.stream;
    slot.stream = st;
    try {
        fv_report rs;
        bool ran = false;
        if (speculate) {
            fv_problem meta = *p;
            meta.ant_enu = sp.ant.data();
            meta.freq_hz = sp.freq.data();
            double box[6];
            std::memcpy(box, sp.s_c, sizeof(sp.s_c));
            std::memcpy(box + 3, sp.S, sizeof(sp.S));
            fv::run_device(ctx, slot, meta, dev_inputs(box), vis, &rs);  // the last call's path and plan
            if (side) FV_HIP(hipStreamWaitEvent(st, sp.ev, 0));  // the join
            FV_HIP(hipEventSynchronize(sp.ev));
            ran = true;
        } else {
            FV_HIP(hipStreamSynchronize(st));
        }
        std::vector<double> ant, freq;
        double box[6];
        const int dim = fv::check_dev_scalars(*p, pin, ant, freq, box);
        fv_problem meta = *p;
        meta.ant_enu = ant.data();
        meta.freq_hz = freq.data();
        const fv::DevInputs in = dev_inputs(box);
        if (ran) {
            // the speculation holds when the geometry is the last call's and its
            // path is still the choice for this call's source box; a type-3 plan
            // also follows the source box itself
            int w = 0;
            const bool lat = dim == 2 && !(p->flags & FV_NO_LATTICE) &&
                             fv::lattice_choice(ctx, meta, in, fv::choose_prec(p->eps, p->flags), &w) != nullptr;
            ran = ant == sp.ant && freq == sp.freq && dim == sp.dim && lat == sp.lattice &&
                  (sp.lattice || (std::memcmp(box, sp.s_c, sizeof(sp.s_c)) == 0 &&
                                  std::memcmp(box + 3, sp.S, sizeof(sp.S)) == 0));
            if (ran && rep) *rep = rs;
        }
        if (!ran) fv::run_device(ctx, slot, meta, in, vis, rep ? rep : &rs);
        const fv_report &used = rep ? *rep : rs;
        if (p->n_src > 0 && (p->flags & FV_METHOD_MASK) == FV_METHOD_NUFFT && !(p->flags & FV_GRAPH)) {
            std::memcpy(sp.ptr, ptrs, sizeof(ptrs));
            sp.n_ant = p->n_ant;
            sp.n_freq = p->n_freq;
            sp.n_src = p->n_src;
            sp.eps = p->eps;
            sp.flags = p->flags;
            sp.ant = ant;
            sp.freq = freq;
            std::memcpy(sp.s_c, box, sizeof(sp.s_c));
            std::memcpy(sp.S, box + 3, sizeof(sp.S));
            sp.lattice = used.lattice != 0;
            sp.dim = used.dim;
            sp.valid = true;
        }
    } catch (...) {
        slot.stream = keep;
        if (side) (void)hipStreamWaitEvent(st, sp.ev, 0);  // the side stream's check joins first
        (void)hipEventRecord(slot.done, st);  // work already enqueued must finish before the workspace is reused
        throw;
    }
    slot.stream = keep;
    FV_HIP(hipEventRecord(slot.done, st));
    if (rep) rep->t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return FV_OK;
    FV_GUARD_END
}

fv_status fv_stage_times(fv_ctx *ctx, double *ms, int *launches, int *n_calls) {
    FV_GUARD_BEGIN
    if (!ctx) fv::fail(FV_EINVAL, "null context");
    FV_HIP(hipSetDevice(ctx->device));
    ctx->main.timer.take(ms, launches, n_calls);
    return FV_OK;
    FV_GUARD_END
}

fv_status fv_set_tune_cache(fv_ctx *ctx, const char *path) {
    FV_GUARD_BEGIN
    if (!ctx) fv::fail(FV_EINVAL, "null context");
    ctx->tunes.load(path ? std::string(path) : std::string());
    return FV_OK;
    FV_GUARD_END
}

fv_status fv_debug_stages(fv_ctx *ctx, const fv_problem *p, int f, double *plan_out, double *spread, size_t spread_cap,
                          double *fftout, size_t fftout_cap) {
    FV_GUARD_BEGIN
    if (!ctx || !p || !plan_out) fv::fail(FV_EINVAL, "null argument");
    fv::validate_host(p);
    if (f < 0 || f >= p->n_freq) fv::fail(FV_EINVAL, "frequency index out of range");
    if ((p->flags & FV_METHOD_MASK) != FV_METHOD_NUFFT) fv::fail(FV_EINVAL, "stages exist for the NUFFT only");
    if (p->n_src == 0) fv::fail(FV_EINVAL, "stages need at least one source");
    FV_HIP(hipSetDevice(ctx->device));
    fv::Slot &slot = ctx->main;
    double s_c[3], S[3];
    fv::DevInputs in = fv::upload(slot, p, s_c, S);
    const int dim = fv::choose_dim(p->ant_enu, p->n_ant, p->eps, p->freq_hz, p->n_freq, p->flags);
    const int prec = fv::choose_prec(p->eps, p->flags);
    const bool fold = !(p->flags & FV_NO_FOLD);
    fv::GeomPlan g = fv::ctx_geometry(ctx, p->ant_enu, p->n_ant, dim, p->eps, s_c, S, fold);
    std::shared_ptr<fv::TargetTable> tt = fv::ctx_targets(ctx, p->ant_enu, in.ant, g, slot.stream);
    fv::SnapJob j;
    j.plan = fv::plan_snapshot(g, p->freq_hz[f]);
    j.src = in.src;
    j.n_src = p->n_src;
    j.flux = in.flux + (size_t)f * p->n_src;
    j.beam = in.beam ? in.beam + (size_t)f * p->n_src : nullptr;
    j.out = in.vis;
    j.tt = tt.get();
    const fv::SnapPlan &sp = j.plan;
    double *po = plan_out;
    po[0] = dim;
    po[1] = g.w;
    po[2] = g.fold_axis;
    for (int a = 0; a < 3; ++a) {
        po[3 + a] = sp.n1[a];
        po[6 + a] = sp.n2[a];
        po[9 + a] = sp.M[a];
        po[12 + a] = sp.P[a];
        po[15 + a] = g.s_c[a];
        po[18 + a] = g.S[a];
        po[21 + a] = g.b_c[a];
        po[24 + a] = g.B[a];
    }
    po[27] = prec;
    po[28] = sp.X[0];
    po[29] = sp.X[1];
    po[30] = sp.X[2];
    const size_t n1c = (size_t)sp.cells1(), nMc = (size_t)sp.cellsM();
    if ((spread && spread_cap < n1c) || (fftout && fftout_cap < nMc)) fv::fail(FV_EINVAL, "output buffers too small");
    fv::nufft_debug(j, dim, prec, g.w, slot.arena, ctx->cache, spread, fftout, slot.stream);
    return FV_OK;
    FV_GUARD_END
}

}  // extern "C"
