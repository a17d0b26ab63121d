// Host orchestration of the type-3 pipeline; the kernels are in nufft_impl.h
// and their instances in nufft_{f32,f64}_{2d,3d}.hip.
#include "nufft_impl.h"

namespace fv {
using namespace detail;
namespace {

PipeFn pick(int dim, int prec_bits, int w) {
    if (prec_bits == 32) return dim == 2 ? pick_f32_2d(w) : pick_f32_3d(w);
    return dim == 2 ? pick_f64_2d(w) : pick_f64_3d(w);
}

}  // namespace


namespace {
struct Prepared {
    Layout L;
    PipeFn fn = nullptr;
    Bufs B;
};

// Uploads the tables of a layout already built for `jobs`.
Prepared prepare_layout(Layout &&layout, const std::vector<SnapJob> &jobs, int dim, int prec_bits, int w,
                        Arena &arena, DevCache &cache, hipStream_t st) {
    if (w < kMinW || w > kMaxW) fail(FV_EUNSUPPORTED, "kernel width out of range");
    Prepared P;
    P.fn = pick(dim, prec_bits, w);
    if (!P.fn) fail(FV_EUNSUPPORTED, "no kernel instance for this width");
    P.L = std::move(layout);
    Layout &L = P.L;
    const double *qn = cache.quad(w, st);
    for (size_t i = 0; i < jobs.size(); ++i) {
        SnapDev &d = L.snaps[i];
        d.qn = qn;
        for (int a = 0; a < dim; ++a) {
            d.tw[a] = cache.twiddle(d.n2[a], prec_bits, st);
            d.drev[a] = cache.digit_reversal(d.n1[a], st);
        }
    }
    const int n = (int)jobs.size();
    const size_t need = layout_bytes(L, dim, prec_bits, n);
    // what the last launch uploaded here (empty if the arena was used or
    // reallocated since)
    std::vector<char> prev;
    prev.swap(arena.tables);
    const bool prev_ipsi = arena.ipsi;
    arena.ipsi = false;  // set again once a launch with these tables is enqueued
    const size_t cap0 = arena.cap;
    arena.ensure(need);
    if (arena.cap != cap0) prev.clear();  // reallocated: contents lost
    arena.reset();
    SnapDev *snaps_dev = (SnapDev *)arena.take(n * sizeof(SnapDev));
    P.B.snaps = snaps_dev;
    P.B.bins = (int *)arena.take(std::max<long long>(L.total_bins, 1) * 4);
    P.B.rank = (int *)arena.take(std::max<long long>(L.total_src, 1) * 4);
    P.B.recs = arena.take(std::max<long long>(L.total_src, 1) * rec_bytes(dim, prec_bits));
    P.B.ipsi = arena.take(std::max<long long>(L.total_ipsi, 1) * (prec_bits == 32 ? 4 : 8));
    P.B.grid = arena.take(std::max<long long>(L.total_grid, 1) * (prec_bits == 32 ? 8 : 16));
    const size_t ng = L.orders.size();
    if (ng) {
        P.B.perm = (int *)arena.take(L.order_src * 4);
        P.B.order_counts = (int *)arena.take(L.order_counts * 4);
        P.B.src_ord = (double *)arena.take(L.order_src * 24);
        P.B.orders = (OrderGroup *)arena.take(ng * sizeof(OrderGroup));
    }
    if (L.det) {
        P.B.recs_tmp = arena.take(std::max<long long>(L.total_src, 1) * rec_bytes(dim, prec_bits));
        P.B.srcid = (int *)arena.take(std::max<long long>(L.total_src, 1) * 4);
    }
    // the tables go up from pinned staging; the staging is reused only after
    // this copy has completed (PinnedBuf::get waits for it).  The same bytes
    // at the same places as the last upload to this arena are already there
    // (same layout, so the same offsets; nothing else has used the arena).
    const size_t tb = n * sizeof(SnapDev), ob = ng * sizeof(OrderGroup);
    const void *where[3] = {arena.base, snaps_dev, P.B.orders};
    std::vector<char> bytes(tb + ob + sizeof(where));
    std::memcpy(bytes.data(), L.snaps.data(), tb);
    if (ng) std::memcpy(bytes.data() + tb, L.orders.data(), ob);
    std::memcpy(bytes.data() + tb + ob, where, sizeof(where));
    P.B.ipsi_ready = prev_ipsi && bytes == prev;
    if (bytes != prev) {
        char *stage = (char *)arena.host.get(tb + ob);
        std::memcpy(stage, bytes.data(), tb + ob);
        FV_HIP(hipMemcpyAsync(snaps_dev, stage, tb, hipMemcpyHostToDevice, st));
        if (ng) FV_HIP(hipMemcpyAsync(P.B.orders, stage + tb, ob, hipMemcpyHostToDevice, st));
        arena.host.record(st);
    }
    arena.tables.swap(bytes);
    return P;
}

Prepared prepare(const std::vector<SnapJob> &jobs, int dim, int prec_bits, int w, Arena &arena, DevCache &cache,
                 hipStream_t st, const Tuning &tune, bool det = false) {
    return prepare_layout(make_layout(jobs, dim, prec_bits, w, tune, det), jobs, dim, prec_bits, w, arena, cache,
                          st);
}

void fetch_c128(const void *dev, long long n, int prec_bits, double *host, hipStream_t st) {
    if (prec_bits == 64) {
        FV_HIP(hipMemcpyAsync(host, dev, (size_t)n * 16, hipMemcpyDeviceToHost, st));
        FV_HIP(hipStreamSynchronize(st));
        return;
    }
    std::vector<float> tmp(2 * (size_t)n);
    FV_HIP(hipMemcpyAsync(tmp.data(), dev, (size_t)n * 8, hipMemcpyDeviceToHost, st));
    FV_HIP(hipStreamSynchronize(st));
    for (size_t i = 0; i < tmp.size(); ++i) host[i] = tmp[i];
}
}  // namespace

// Class of a launch group for the autotuner: dimension, precision and the
// power-of-two buckets of the largest line length per axis and of the
// snapshot count.
std::string tune_key(const std::vector<SnapJob> &jobs, int dim, int prec_bits) {
    auto bucket = [](long long v) {
        long long b = 1;
        while (b < v) b <<= 1;
        return b;
    };
    int n1max[3] = {1, 1, 1};
    for (auto &j : jobs)
        for (int a = 0; a < dim; ++a) n1max[a] = std::max(n1max[a], j.plan.n1[a]);
    std::string k = "d" + std::to_string(dim) + "_p" + std::to_string(prec_bits) + "_n";
    for (int a = 0; a < dim; ++a) k += (a ? "x" : "") + std::to_string(bucket(n1max[a]));
    return k + "_s" + std::to_string(bucket((long long)jobs.size()));
}

namespace {
// Times the FFT passes (stage 2 only, on whatever the grid holds) for each
// candidate launch shape and returns the fastest.
Tuning autotune(const std::vector<SnapJob> &jobs, int dim, int prec_bits, int w, Arena &arena, DevCache &cache,
                hipStream_t st) {
    hipEvent_t a, b;
    FV_HIP(hipEventCreate(&a));
    FV_HIP(hipEventCreate(&b));
    Tuning best = Tuning::defaults();
    best.fft_ms = 1e30;
    try {
        for (int split : {0, 1})
        for (int rows : {1, 2})
            for (int lines : {1, 2, 4})
                for (int tpb1 : {256, 512})
                    for (int tpbm : {128, 256, 512}) {
                        Tuning t;
                        t.split = split;
                        t.rows = rows;
                        t.lines = lines;
                        t.tpb1 = tpb1;
                        t.tpbm = tpbm;
                        Prepared P = prepare(jobs, dim, prec_bits, w, arena, cache, st, t);
                        P.fn(P.L, P.B, (int)jobs.size(), st, 2, nullptr);  // warm
                        float ms = 1e30f;
                        for (int r = 0; r < 2; ++r) {
                            FV_HIP(hipEventRecord(a, st));
                            P.fn(P.L, P.B, (int)jobs.size(), st, 2, nullptr);
                            FV_HIP(hipEventRecord(b, st));
                            FV_HIP(hipEventSynchronize(b));
                            float x = 0;
                            FV_HIP(hipEventElapsedTime(&x, a, b));
                            ms = std::min(ms, x);
                        }
                        if (ms < best.fft_ms) {
                            best = t;
                            best.fft_ms = ms;
                        }
                    }
    } catch (...) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        throw;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return best;
}

uint64_t mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    return h;
}

// Everything a captured launch sequence bakes in: kernel arguments (buffer
// addresses, sizes) and launch dimensions.  The per-snapshot table itself is
// device memory, uploaded before every replay.
uint64_t graph_key(const Prepared &P, int n, int dim, int prec_bits, int w) {
    const Layout &L = P.L;
    uint64_t h = 1469598103934665603ull;
    for (long long v : {(long long)n, (long long)dim, (long long)prec_bits, (long long)w, L.max_wg[0], L.max_wg[1],
                        L.max_wg[2], L.max_tiles, L.max_src, L.max_tgt, L.max_ipsi, L.total_bins,
                        (long long)L.orders.size(), L.max_order_src, L.order_counts, (long long)L.tpb[0],
                        (long long)L.tpb[1], (long long)L.tpb[2], (long long)L.fft_lds[0], (long long)L.fft_lds[1],
                        (long long)L.fft_lds[2], (long long)L.det, (long long)L.reg[0], (long long)L.reg[1],
                        (long long)L.reg[2], L.reg_wg[0], L.reg_wg[1], L.reg_wg[2], (long long)L.reg_lds[0],
                        (long long)L.reg_lds[1], (long long)L.reg_lds[2]})
        h = mix(h, (uint64_t)v);
    for (const void *p : {(const void *)P.B.snaps, (const void *)P.B.bins, (const void *)P.B.rank,
                          (const void *)P.B.recs, (const void *)P.B.ipsi, (const void *)P.B.grid,
                          (const void *)P.B.perm, (const void *)P.B.order_counts, (const void *)P.B.src_ord,
                          (const void *)P.B.orders, (const void *)P.B.recs_tmp, (const void *)P.B.srcid,
                          (const void *)P.B.basis_M, (const void *)P.B.basis_vis})
        h = mix(h, (uint64_t)(uintptr_t)p);
    h = mix(h, (uint64_t)P.B.basis_np);
    return h;
}
}  // namespace

double nufft_execute(const std::vector<SnapJob> &jobs, int dim, int prec_bits, int w, Arena &arena, DevCache &cache,
                     hipStream_t st, StageTimer *timer, const ExecOpts *opts, bool *too_big) {
    if (too_big) *too_big = false;
    if (jobs.empty()) return 0.0;
    // the workspace size does not depend on the launch shape
    Tuning tune = Tuning::defaults();
    const bool det = opts && opts->det;
    Layout layout = make_layout(jobs, dim, prec_bits, w, tune, det);
    if (opts && opts->cap && too_big && layout_bytes(layout, dim, prec_bits, (int)jobs.size()) > opts->cap) {
        *too_big = true;
        return 0.0;
    }
    if (opts && opts->tunes) {
        const std::string key = tune_key(jobs, dim, prec_bits);
        bool have = opts->tunes->find(key, &tune);
        if (!have && opts->autotune) {
            tune = autotune(jobs, dim, prec_bits, w, arena, cache, st);
            opts->tunes->put(key, tune);
            have = true;
        }
        if (have) layout = make_layout(jobs, dim, prec_bits, w, tune, det);
    }
    Prepared P = prepare_layout(std::move(layout), jobs, dim, prec_bits, w, arena, cache, st);
    if (opts && opts->basis_vis) {
        P.B.basis_M = opts->basis_M;
        P.B.basis_vis = opts->basis_vis;
        P.B.basis_np = opts->basis_np;
    }
    const int n = (int)jobs.size();
    // graphs need a capturable (non-null) stream; per-stage timing stays eager
    const bool graph = opts && opts->graph && opts->graphs && st != nullptr && !(timer && timer->on);
    if (!graph) {
        P.fn(P.L, P.B, n, st, 7, timer);
        arena.ipsi = true;
        return P.L.model_bytes;
    }
    P.B.ipsi_ready = false;  // a captured sequence always computes them
    const uint64_t key = graph_key(P, n, dim, prec_bits, w);
    hipGraphExec_t ex = opts->graphs->find(key);
    if (!ex) {
        hipGraph_t g = nullptr;
        FV_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        try {
            P.fn(P.L, P.B, n, st, 7, nullptr);
        } catch (...) {
            (void)hipStreamEndCapture(st, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        FV_HIP(hipStreamEndCapture(st, &g));
        hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        FV_HIP(e);
        opts->graphs->put(key, ex);
    }
    FV_HIP(hipGraphLaunch(ex, st));
    arena.ipsi = true;
    return P.L.model_bytes;
}

void nufft_debug(const SnapJob &job, int dim, int prec_bits, int w, Arena &arena, DevCache &cache, double *spread,
                 double *fftout, hipStream_t st) {
    std::vector<SnapJob> jobs{job};
    Prepared P = prepare(jobs, dim, prec_bits, w, arena, cache, st, Tuning::defaults());
    const SnapDev &d = P.L.snaps[0];
    const size_t csz = prec_bits == 32 ? 8 : 16;
    P.fn(P.L, P.B, 1, st, 1, nullptr);
    if (spread) fetch_c128((char *)P.B.grid + d.bufA * csz, job.plan.cells1(), prec_bits, spread, st);
    P.fn(P.L, P.B, 1, st, 2, nullptr);
    const long long fin = dim == 2 ? d.bufA : d.bufB;
    if (fftout) fetch_c128((char *)P.B.grid + fin * csz, job.plan.cellsM(), prec_bits, fftout, st);
    P.fn(P.L, P.B, 1, st, 4, nullptr);
    FV_HIP(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------------------
namespace {

// Target table over several frequencies of one planned snapshot: target
// q n_pairs + t is pair perm[t]'s folded baseline scaled by scale[q] (the
// frequency over the planned one); the output index is q n_pairs + pair.
__global__ __launch_bounds__(256) void k_targets_multi(const double *ant, int n_ant, long long n_pairs, int n_scale,
                                                       const double *scale, int dim, int fold_axis, double3 b_c,
                                                       double3 B, double xi0, const double *qn, const int *perm,
                                                       double *tb, int *tidx, double *tphi) {
    const long long n_tgt = n_pairs * n_scale;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_tgt) return;
    const int q = (int)(t / n_pairs);
    const long long tp = t - (long long)q * n_pairs;
    const long long p = perm ? (long long)perm[tp] : tp;
    int i, j;
    pair_decode(p, n_ant, &i, &j);
    double b[3];
    for (int a = 0; a < 3; ++a) b[a] = ant[3 * (size_t)i + a] - ant[3 * (size_t)j + a];
    bool flip = false;
    if (fold_axis >= 0) {
        int order[3] = {fold_axis, 0, 0};
        int k = 1;
        for (int a = 0; a < dim; ++a)
            if (a != fold_axis) order[k++] = a;
        for (int r = 0; r < dim; ++r) {
            const double v = b[order[r]];
            if (v < 0) { flip = true; break; }
            if (v > 0) break;
        }
    }
    const double sc = scale[q];
    const double bc[3] = {b_c.x, b_c.y, b_c.z}, Bh[3] = {B.x, B.y, B.z};
    for (int a = 0; a < dim; ++a) {
        const double f = (flip ? -b[a] : b[a]) * sc;
        tb[(long long)a * n_tgt + t] = f;
        const double xi = Bh[a] > 0 ? xi0 * (f - bc[a]) / Bh[a] : 0.0;
        tphi[(long long)a * n_tgt + t] = phihat_quad(xi, qn);
    }
    tidx[t] = (int)((long long)q * n_pairs + p) | (flip ? (int)0x80000000 : 0);
}

}  // namespace

void build_targets_multi(const double *ant_dev, int n_ant, int dim, int fold_axis, const double *b_c, const double *B,
                         int w, const double *qn_dev, const int *perm_dev, const double *scale_dev, int n_scale,
                         TargetTable &tt, hipStream_t st) {
    const long long n = (long long)n_ant * (n_ant + 1) / 2 * n_scale;
    const double xi0 = w * M_PI / (2.0 * kSigma);
    hipLaunchKernelGGL(k_targets_multi, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ant_dev, n_ant,
                       (long long)n_ant * (n_ant + 1) / 2, n_scale, scale_dev, dim, fold_axis,
                       make_double3(b_c[0], b_c[1], b_c[2]), make_double3(B[0], B[1], B[2]), xi0, qn_dev, perm_dev,
                       tt.tb, tt.tidx, tt.tphi);
    FV_HIP(hipGetLastError());
}

void build_targets(const double *ant_dev, int n_ant, int dim, int fold_axis, const double *b_c, const double *B, int w,
                   const double *qn_dev, const int *perm_dev, TargetTable &tt, hipStream_t st) {
    const long long n = (long long)n_ant * (n_ant + 1) / 2;
    const double xi0 = w * M_PI / (2.0 * kSigma);
    hipLaunchKernelGGL(k_targets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ant_dev, n_ant, n, dim,
                       fold_axis, make_double3(b_c[0], b_c[1], b_c[2]), make_double3(B[0], B[1], B[2]), xi0, qn_dev,
                       perm_dev, tt.tb, tt.tidx, tt.tphi);
    FV_HIP(hipGetLastError());
}

// Each table is built once, on the stream of the first call that needs it;
// the build is waited for before the table is published, since later users
// may run on other streams.
const void *DevCache::twiddle(int n, int prec_bits, hipStream_t st) {
    std::lock_guard<std::mutex> lk(mu);
    auto key = std::make_pair(n, prec_bits);
    auto it = twiddles.find(key);
    if (it != twiddles.end()) return it->second;
    void *p = nullptr;
    const size_t csz = prec_bits == 32 ? 8 : 16;
    FV_HIP(hipMalloc(&p, (size_t)n * csz));
    if (prec_bits == 32)
        hipLaunchKernelGGL(k_twiddle<float>, dim3((n + 255) / 256), dim3(256), 0, st, n, (float2 *)p);
    else
        hipLaunchKernelGGL(k_twiddle<double>, dim3((n + 255) / 256), dim3(256), 0, st, n, (double2 *)p);
    FV_HIP(hipGetLastError());
    FV_HIP(hipStreamSynchronize(st));
    twiddles[key] = p;
    return p;
}

const int *DevCache::digit_reversal(int n, hipStream_t st) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = drevs.find(n);
    if (it != drevs.end()) return it->second;
    int *p = nullptr;
    FV_HIP(hipMalloc(&p, (size_t)n * sizeof(int)));
    hipLaunchKernelGGL(k_digrev, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, p);
    FV_HIP(hipGetLastError());
    FV_HIP(hipStreamSynchronize(st));
    drevs[n] = p;
    return p;
}

const double *DevCache::quad(int w, hipStream_t st) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = qnodes.find(w);
    if (it != qnodes.end()) return it->second;
    double host[2 * kQuadHalf];
    quad_table(w, host);
    double *p = nullptr;
    FV_HIP(hipMalloc(&p, sizeof(host)));
    FV_HIP(hipMemcpyAsync(p, host, sizeof(host), hipMemcpyHostToDevice, st));
    FV_HIP(hipStreamSynchronize(st));
    qnodes[w] = p;
    return p;
}

void DevCache::release() {
    std::lock_guard<std::mutex> lk(mu);
    for (auto &kv : twiddles) (void)hipFree(kv.second);
    for (auto &kv : drevs) (void)hipFree(kv.second);
    drevs.clear();
    for (auto &kv : qnodes) (void)hipFree(kv.second);
    twiddles.clear();
    qnodes.clear();
}

}  // namespace fv
