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

size_t nufft_workspace_bytes(const std::vector<SnapJob> &jobs, int dim, int prec_bits, int w) {
    Layout L = make_layout(jobs, dim, prec_bits, w);
    return layout_bytes(L, dim, prec_bits, (int)jobs.size());
}

namespace {
struct Prepared {
    Layout L;
    PipeFn fn = nullptr;
    Bufs B;
};

Prepared prepare(const std::vector<SnapJob> &jobs, int dim, int prec_bits, int w, Arena &arena, DevCache &cache,
                 hipStream_t st) {
    if (w < kMinW || w > kMaxW) fail(FV_EUNSUPPORTED, "kernel width out of range");
    Prepared P;
    P.fn = pick(dim, prec_bits, w);
    if (!P.fn) fail(FV_EUNSUPPORTED, "no kernel instance for this width");
    P.L = make_layout(jobs, dim, prec_bits, w);
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
    arena.ensure(need);
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
    // the tables go up from pinned staging; the staging is reused only after
    // this copy has completed (PinnedBuf::get waits for it)
    const size_t tb = n * sizeof(SnapDev), ob = ng * sizeof(OrderGroup);
    char *stage = (char *)arena.host.get(tb + ob);
    std::memcpy(stage, L.snaps.data(), tb);
    if (ng) std::memcpy(stage + tb, L.orders.data(), ob);
    FV_HIP(hipMemcpyAsync(snaps_dev, stage, tb, hipMemcpyHostToDevice, st));
    if (ng) FV_HIP(hipMemcpyAsync(P.B.orders, stage + tb, ob, hipMemcpyHostToDevice, st));
    arena.host.record(st);
    return P;
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

double nufft_execute(const std::vector<SnapJob> &jobs, int dim, int prec_bits, int w, Arena &arena, DevCache &cache,
                     hipStream_t st, StageTimer *timer) {
    if (jobs.empty()) return 0.0;
    Prepared P = prepare(jobs, dim, prec_bits, w, arena, cache, st);
    P.fn(P.L, P.B, (int)jobs.size(), st, 7, timer);
    return P.L.model_bytes;
}

void nufft_debug(const SnapJob &job, int dim, int prec_bits, int w, Arena &arena, DevCache &cache, double *spread,
                 double *fftout, hipStream_t st) {
    std::vector<SnapJob> jobs{job};
    Prepared P = prepare(jobs, dim, prec_bits, w, arena, cache, st);
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
void build_targets(const double *ant_dev, int n_ant, int dim, int fold_axis, const double *b_c, const double *B, int w,
                   const double *qn_dev, TargetTable &tt, hipStream_t st) {
    const long long n = (long long)n_ant * (n_ant + 1) / 2;
    const double xi0 = w * M_PI / (2.0 * kSigma);
    hipLaunchKernelGGL(k_targets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ant_dev, n_ant, n, dim,
                       fold_axis, make_double3(b_c[0], b_c[1], b_c[2]), make_double3(B[0], B[1], B[2]), xi0, qn_dev,
                       tt.tb, tt.tidx, tt.tphi);
    FV_HIP(hipGetLastError());
}

const void *DevCache::twiddle(int n, int prec_bits, hipStream_t st) {
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
    twiddles[key] = p;
    return p;
}

const int *DevCache::digit_reversal(int n, hipStream_t st) {
    auto it = drevs.find(n);
    if (it != drevs.end()) return it->second;
    int *p = nullptr;
    FV_HIP(hipMalloc(&p, (size_t)n * sizeof(int)));
    hipLaunchKernelGGL(k_digrev, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, p);
    FV_HIP(hipGetLastError());
    drevs[n] = p;
    return p;
}

const double *DevCache::quad(int w, hipStream_t st) {
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
    for (auto &kv : twiddles) (void)hipFree(kv.second);
    for (auto &kv : drevs) (void)hipFree(kv.second);
    drevs.clear();
    for (auto &kv : qnodes) (void)hipFree(kv.second);
    twiddles.clear();
    qnodes.clear();
}

}  // namespace fv
