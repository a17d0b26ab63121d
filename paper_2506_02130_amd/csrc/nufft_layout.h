// Host side of the type-3 pipeline's workspace: the per-snapshot table
// (SnapDev) and the sizes and offsets of every device buffer of a launch
// group.  Host code only (no kernels), so that the sizing can be checked on
// a machine without a GPU.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

#include "fv_internal.h"

namespace fv {

template <typename R, int D>
struct Rec {
    int l0[D];
    R off[D];
    R cr, ci;
};

template <int D>
struct TileShape;
// Spread tiles: a workgroup covers X x Y x Z cells.  In 3-D each of its 4
// wavefronts owns an 8-column slice and walks it in 8 x 8 (x TZ) sub-tiles, one
// cell (x TZ slices) per lane; in 2-D its one wavefront owns one matrix-core
// tile.
template <>
struct TileShape<2> {
    static constexpr int X = 16, Y = 16, Z = 1;  // 1 matrix-core tile of 16 x 16
};
template <>
struct TileShape<3> {
    static constexpr int X = 32, Y = 8, Z = 8;
};

__host__ __device__ inline int sub_bin_edge(int a) { return a < 2 ? kSubBin : kSubBinZ; }

// Shared spatial order of a source list read by several snapshots: counting
// sort by the sub-bins of one snapshot of the list (its finest grid).
// Workgroup row y handles list y; perm[base + position] = source index and
// src_ord holds the directions in that order.
struct OrderGroup {
    int snap;              // snapshot whose sub-bins define the order
    int n_src;
    long long base;        // offset in perm / rank scratch (and D x in src_ord: D coordinates per source)
    long long cnt_base;    // offset of the list's nb + 1 counts
    long long nb;          // sub-bins of that snapshot
};

// LDS stride of a line of the general FFT kernel: one pad complex every 16.
__host__ __device__ inline int cline_pad(int L) { return L + (L >> 4) + 1; }

// Entries of the two twiddle tables of an N-point line.
__host__ __device__ inline int fft_tw_entries(int N) { return (N >> 6) + 1 + 64; }

namespace detail {

struct Layout {
    std::vector<SnapDev> snaps;
    long long total_tiles = 0, total_src = 0, total_bins = 0, total_ipsi = 0, total_grid = 0;
    long long max_src = 0, max_tgt = 0, max_ipsi = 0, max_tiles = 0;
    bool any_degenerate = false;  // some snapshot has a clamped axis (interpolation's quadrature variant)
    long long wg_total[3] = {0, 0, 0};
    long long max_wg[3] = {0, 0, 0};
    int tpb[3] = {256, 256, 256};
    size_t fft_lds[3] = {0, 0, 0};
    double model_bytes = 0;
    double sbytes[FV_NSTAGE] = {0, 0, 0, 0, 0, 0, 0, 0};  // algorithmic bytes per stage
    // shared spatial orders, one per source list read by several snapshots
    std::vector<OrderGroup> orders;
    long long order_src = 0, order_counts = 0, max_order_src = 0;
    bool det = false;  // deterministic record order (stable ranks inside each sub-bin)
    // planned FFT passes (FP32, every snapshot's line length has a plan)
    bool reg[3] = {false, false, false};
    long long reg_wg[3] = {0, 0, 0};
    size_t reg_lds[3] = {0, 0, 0};
};


inline int env_int(const char *name, int dflt) {
    const char *e = std::getenv(name);
    return e ? std::atoi(e) : dflt;
}

inline size_t rec_bytes(int dim, int prec_bits) {
    if (prec_bits == 32) return dim == 2 ? sizeof(Rec<float, 2>) : sizeof(Rec<float, 3>);
    return dim == 2 ? sizeof(Rec<double, 2>) : sizeof(Rec<double, 3>);
}

inline Layout make_layout(const std::vector<SnapJob> &jobs, int dim, int prec_bits, int w, const Tuning &tune,
                          bool det = false) {
    Layout L;
    L.det = det;
    const size_t csz = prec_bits == 32 ? 8 : 16;
    const int T[3] = {dim == 2 ? TileShape<2>::X : TileShape<3>::X, dim == 2 ? TileShape<2>::Y : TileShape<3>::Y,
                      dim == 2 ? 1 : TileShape<3>::Z};
    // FFT threads per pass from the largest line length (n1 points per line)
    for (int a = 0; a < dim; ++a) {
        int lmax = 0, nmax = 0;
        for (auto &j : jobs) {
            lmax = std::max(lmax, j.plan.n1[a]);
            nmax = std::max(nmax, j.plan.n2[a]);
        }
        L.tpb[a] = tune.tpb(lmax, a > 0);
        if ((size_t)(2 * cline_pad(lmax) + fft_tw_entries(nmax)) * csz > 160u * 1024)
            fail(FV_EUNSUPPORTED, "FFT line of " + std::to_string(nmax) + " points exceeds the LDS transform");
    }
    for (auto &j : jobs) {
        const SnapPlan &p = j.plan;
        SnapDev d;
        std::memset(&d, 0, sizeof(d));
        d.order_base = -1;
        long long nb = 1, ncell = 1, nipsi = 0;
        for (int a = 0; a < 3; ++a) {
            d.n1[a] = p.n1[a];
            d.n2[a] = p.n2[a];
            d.M[a] = p.M[a];
            d.P[a] = p.P[a];
            d.ntile[a] = a < dim ? (p.n1[a] + T[a] - 1) / T[a] : 1;
            d.nsb[a] = a < dim ? (p.n1[a] - w) / sub_bin_edge(a) + 1 : 1;
            nb *= d.nsb[a];
            if (a < dim) {
                ncell *= d.ntile[a];
                nipsi += p.n1[a];
            }
        }
        d.dim = dim;
        d.w = w;
        d.n_src = j.n_src;
        d.n_tgt = (int)j.tt->n_tgt;
        d.degenerate = p.degenerate;
        d.tile_base = L.total_tiles;
        L.total_tiles += ncell;
        L.max_tiles = std::max(L.max_tiles, ncell);
        d.src_base = L.total_src;
        L.total_src += j.n_src;
        d.bin_base = L.total_bins;
        L.total_bins += (nb + 1 + 3) / 4 * 4;  // 16-byte aligned per snapshot (vector scan loads)
        d.ipsi_base = L.total_ipsi;
        L.total_ipsi += nipsi;
        // grid regions (elements)
        long long A, B;
        const long long n1x = p.n1[0], n1y = p.n1[1], n1z = p.n1[2], Mx = p.M[0], My = p.M[1], Mz = p.M[2];
        if (dim == 2) {
            A = std::max(n1x * n1y, Mx * My);
            B = Mx * n1y;
        } else {
            A = std::max(n1x * n1y * n1z, Mx * My * n1z);
            B = std::max(Mx * n1y * n1z, Mx * My * Mz);
        }
        auto al = [](long long v) { return (v + 63) / 64 * 64; };
        d.bufA = L.total_grid;
        L.total_grid += al(A);
        d.bufB = L.total_grid;
        L.total_grid += al(B);
        // FFT pass geometry
        for (int a = 0; a < dim; ++a) {
            long long F = 1, Sl = 1;
            for (int b = 0; b < a; ++b) F *= p.M[b];
            for (int b = a + 1; b < dim; ++b) Sl *= p.n1[b];
            // lines per workgroup: columns (fast extent F > 1) or rows (F == 1),
            // each line held as two transforms within 64 KB of LDS
            const int tps = tune.split ? 1 : 2;
            d.fft_split[a] = tune.split ? 1 : 0;
            const long long bylds = (65536LL - (long long)fft_tw_entries(p.n2[a]) * csz) /
                                    ((long long)tps * cline_pad(p.n1[a]) * csz);
            // short lines take more lines per workgroup so that every thread
            // has butterflies (about 4 TPB points per workgroup)
            const long long fill = 4LL * L.tpb[a] / (2LL * p.n1[a]);
            const long long lim = std::max(fill, F > 1 ? (long long)tune.lines : (long long)tune.rows);
            const int cx = (int)std::max(1LL, std::min({F > 1 ? F : Sl, bylds, lim}));
            const long long nwg = (F > 1 ? Sl * ((F + cx - 1) / cx) : (Sl + cx - 1) / cx) * (tune.split ? 2 : 1);
            d.cx[a] = cx;
            d.wg_base[a] = L.wg_total[a];
            L.wg_total[a] += nwg;
            L.fft_lds[a] = std::max(L.fft_lds[a], (size_t)tps * cx * cline_pad(p.n1[a]) * csz +
                                                      (size_t)fft_tw_entries(p.n2[a]) * csz);
            L.max_wg[a] = std::max(L.max_wg[a], nwg);
        }
        d.src = j.src;
        d.flux = j.flux;
        d.beam = j.beam;
        d.out = j.out;
        d.tb = j.tt->tb;
        d.tidx = j.tt->tidx;
        d.tphi = j.tt->tphi;
        const double beta = 2.3 * w;
        d.beta = beta;
        double post_norm = 1.0;
        for (int a = 0; a < dim; ++a) {
            d.gscale[a] = kSigma * p.X[a] / M_PI;
            d.s_c[a] = p.s_c[a];
            d.b_c[a] = p.b_c[a];
            // q = (n1/2) (x - x_c) / X with x = -k b
            d.qscale[a] = -(0.5 * p.n1[a]) * p.k / p.X[a];
            // xi = alpha1 kappa = w pi (x - x_c) / (2 sigma X)  (clamped axes)
            d.xi_deg[a] = -(w * M_PI) * p.k / (2.0 * kSigma * p.X[a]);
            d.pre_turn[a] = -(p.nu / kCLight) * p.b_c[a];
            post_norm *= 4.0 * M_PI / ((double)p.n2[a] * w);
        }
        d.post_turn = -(p.nu / kCLight);
        d.post_norm = post_norm;
        L.max_src = std::max<long long>(L.max_src, j.n_src);
        L.max_tgt = std::max<long long>(L.max_tgt, j.tt->n_tgt);
        L.any_degenerate = L.any_degenerate || p.degenerate != 0;
        L.max_ipsi = std::max(L.max_ipsi, nipsi);
        // algorithmic bytes of the grid stages: spread write, each pass
        // read + write of the live array, interp read of the final array
        double cells_in = (double)p.cells1(), b = cells_in;
        double live = cells_in;
        for (int a = 0; a < dim; ++a) {
            double outc = live / p.n1[a] * p.M[a];
            b += live + outc;
            live = outc;
        }
        b += live;
        L.model_bytes += b * csz;
        {
            // per stage: sort reads the directions twice, flux/beam once, writes
            // ranks and records; spread reads the records and writes the grid;
            // each pass reads and writes its live array; interpolation reads the
            // final array, the target table and writes the output
            const double rsz = (double)rec_bytes(dim, prec_bits);
            const double ns = (double)j.n_src, nt = (double)j.tt->n_tgt;
            L.sbytes[FV_STAGE_SORT] += ns * (2.0 * 8 * dim + 16 + 4 + 4 + 4 + rsz) + 8.0 * (double)nb;
            L.sbytes[FV_STAGE_SPREAD] += ns * rsz + cells_in * csz;
            double lv = cells_in;
            for (int a = 0; a < dim; ++a) {
                double oc = lv / p.n1[a] * p.M[a];
                L.sbytes[FV_STAGE_FFT_X + a] += (lv + oc) * csz;
                lv = oc;
            }
            L.sbytes[FV_STAGE_INTERP] += lv * csz + nt * (16.0 * dim + 4 + 16);
            L.sbytes[FV_STAGE_OTHER] += (double)nipsi * (prec_bits == 32 ? 4 : 8);
        }
        L.snaps.push_back(d);
    }
    // the planned FFT kernels take a pass when every snapshot's line length
    // has a plan (FP32 grids; FV_FFT_GENERAL=1 keeps the general kernel)
    static const bool general_only = env_int("FV_FFT_GENERAL", 0) != 0;
    for (int a = 0; a < dim && prec_bits == 32 && !general_only && !jobs.empty(); ++a) {
        bool ok = true;
        long long wg = 0;
        size_t lds = 0;
        for (size_t s = 0; s < jobs.size(); ++s) {
            const SnapJob &j = jobs[s];
            int nl = 0;
            size_t b = 0;
            if (!fft_reg_info(j.plan.n1[a], a > 0, &nl, &b)) {
                ok = false;
                break;
            }
            long long F = 1, Sl = 1;
            for (int c = 0; c < a; ++c) F *= j.plan.M[c];
            for (int c = a + 1; c < dim; ++c) Sl *= j.plan.n1[c];
            const long long n = a == 0 ? (Sl + nl - 1) / nl : Sl * ((F + nl - 1) / nl);
            L.snaps[s].reg_base[a] = wg;  // workgroups of the pass are numbered snapshot by snapshot
            wg += n;
            lds = std::max(lds, b);
        }
        L.reg[a] = ok;
        L.reg_wg[a] = ok ? wg : 0;
        L.reg_lds[a] = ok ? lds : 0;
    }
    // a shared source order pays off when several snapshots bin the same list
    std::map<std::pair<const double *, int>, std::vector<int>> lists;
    for (int i = 0; i < (int)jobs.size(); ++i)
        if (jobs[i].n_src > 0) lists[{jobs[i].src, jobs[i].n_src}].push_back(i);
    for (auto &kv : lists) {
        if (kv.second.size() < 2) continue;
        int best = kv.second[0];
        for (int i : kv.second)
            if (jobs[i].plan.cells1() > jobs[best].plan.cells1()) best = i;
        OrderGroup G;
        G.snap = best;
        G.n_src = kv.first.second;
        G.base = L.order_src;
        G.cnt_base = L.order_counts;
        G.nb = 1;
        for (int a = 0; a < dim; ++a) G.nb *= L.snaps[best].nsb[a];
        for (int i : kv.second) L.snaps[i].order_base = G.base;
        L.order_src += G.n_src;
        L.order_counts += (G.nb + 1 + 3) / 4 * 4;
        L.max_order_src = std::max<long long>(L.max_order_src, G.n_src);
        L.orders.push_back(G);
    }
    return L;
}


inline size_t layout_bytes(const Layout &L, int dim, int prec_bits, int n_snap) {
    const size_t csz = prec_bits == 32 ? 8 : 16, rsz = prec_bits == 32 ? 4 : 8;
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    return al(n_snap * sizeof(SnapDev)) + al(L.total_bins * 4) + al(L.total_src * 4) +
           al(L.total_src * rec_bytes(dim, prec_bits)) + al(L.total_ipsi * rsz) + al(L.total_grid * csz) +
           al(L.order_src * 4) + al(L.order_counts * 4) + al(L.order_src * 24) +
           al(L.orders.size() * sizeof(OrderGroup)) +
           (L.det ? al(L.total_src * rec_bytes(dim, prec_bits)) + al(L.total_src * 4) : 0) + 4096;
}


}  // namespace detail
}  // namespace fv
