// Type-3 NUFFT pipeline for gfx950 (paper section 2.2, steps 1-3):
//
//   bin      per (snapshot, source): first kernel cell l0 (FP64), sub-bin key,
//            rank inside its sub-bin (counting sort, pass 1)
//   scan     per snapshot: exclusive scan of the sub-bin counts
//   scatter  per (snapshot, source): sorted record {l0, fractional offset,
//            pre-phased strength c' = c exp(i x_c . (s - s_c))}
//   ipsi     per snapshot: 1/psi2hat(m) at the uniform modes
//   spread   one wavefront per output tile: records of the neighbouring
//            sub-bins are staged 64 at a time, kernel weights precomputed per
//            record in LDS, each record's w^d footprint added by the lanes
//            (one lane per footprint cell) into an LDS tile; the tile is
//            written once, already divided by psi2hat (the first
//            deconvolution) -- no global atomics, each cell written once
//   fft      per axis: lines loaded into LDS with the zero padding to n2 in
//            place, mixed-radix (2,3,4,5) Stockham FFT with the + sign, only
//            the M = 2P+1 outputs the interpolation can touch are written
//   interp   per (snapshot, target): w^d gather with the ES kernel, divided by
//            psi1hat at the target, centring phase exp(i x_k . s_c), and the
//            reflection undone by conjugation; written straight into the
//            caller's (i <= j) layout
//
// Grid arithmetic is R (float or double); every coordinate, phase and
// deconvolution factor is computed in FP64.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <utility>

#include <algorithm>
#include <map>
#include <cstdlib>
#include <cstring>
#include <stdexcept>
#include <vector>

#include "ctx.h"
#include "dev_common.h"
#include "fv_internal.h"
#include "nufft_layout.h"

namespace fv {
namespace {


__device__ inline int find_snap(const SnapDev *snaps, int n_snap, long long v, int which) {
    // last s with base(s) <= v; which: 0 tile_base, 1..3 wg_base[which-1]
    int lo = 0, hi = n_snap - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        long long b = which == 0 ? snaps[mid].tile_base : snaps[mid].wg_base[which - 1];
        if (b <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Workgroup coordinates (x within its snapshot, snapshot y).  gx == 0: the
// plain 2-D grid (x, y) = blockIdx.  gx > 0: a 1-D grid of 8 gx ceil(n_snap / 8)
// workgroups in which every workgroup of snapshot y runs on XCD y mod 8
// (workgroups are dispatched to the 8 XCDs round-robin), so the data of one
// snapshot stays in one L2.  Returns false for padding workgroups.
__device__ __forceinline__ bool snap_block(int gx, int n_snap, int &x, int &y) {
    if (gx <= 0) {
        x = blockIdx.x;
        y = blockIdx.y;
        return true;
    }
    const int per = 8 * gx, id = blockIdx.x;
    const int hi = id / per, r = id - hi * per;
    y = hi * 8 + (r & 7);
    x = r >> 3;
    return y < n_snap;
}

// First kernel cell and sub-bin of a source (FP64 coordinates).
template <int D>
__device__ __forceinline__ int src_cell(const SnapDev &S, const double *s, double *g, int *l0) {
    int key = 0, mult = 1;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double gg = 0.5 * S.n1[a] + (s[a] - S.s_c[a]) * S.gscale[a];
        int l = (int)ceil(gg - 0.5 * S.w);
        l = min(max(l, 0), S.n1[a] - S.w);
        g[a] = gg;
        l0[a] = l;
        key += (l / sub_bin_edge(a)) * mult;
        mult *= S.nsb[a];
    }
    return key;
}

__global__ void k_fill_int(int *p, long long n, int v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Rank of this lane's key among the lanes of its wavefront that share the key,
// plus the count already in counts[key]: one returning atomic per distinct key
// in the wavefront (lanes of a spatially ordered source list mostly share a
// few sub-bins).  The groups of equal keys are found with ballots first (the
// first remaining lane's key read into a scalar register; each lane keeps its
// own group's mask); then the first lane of every group adds its group's size
// in one atomic instruction for all groups, and each lane reads its group's
// old count from its leader.  Every active lane of the wavefront must call it.
__device__ __forceinline__ int wave_rank(int *counts, int key) {
    const int lane = threadIdx.x & 63;
    unsigned long long todo = __ballot(1), mine = 0;
    while (todo) {
        const int l = __ffsll((long long)todo) - 1;  // wave-uniform
        const int lk = readlane_i(key, l);             // a scalar read, no LDS round trip
        const unsigned long long m = __ballot(key == lk) & todo;
        // a lane whose group was taken earlier never meets its key again
        if (key == lk) mine = m;
        todo &= ~m;
    }
    const int leader = __ffsll((long long)mine) - 1;
    const int below = __popcll(mine & ((1ull << lane) - 1ull));
    int old = 0;
    if (lane == leader) old = atomicAdd(&counts[key], __popcll(mine));
    return __shfl(old, leader, 64) + below;
}

// Per-snapshot counting sort of the sources by sub-bin.  Sources are visited
// in the order perm (a spatial order shared by all snapshots of one source
// list) when perm is non-null, else in input order; rank and the records are
// indexed by that visiting position i.
template <int D>
__global__ __launch_bounds__(256) void k_bin(const SnapDev *snaps, int gx, int n_snap, const double *src_ord,
                                             int *bins, int *rank) {
    int bx, sy;
    if (!snap_block(gx, n_snap, bx, sy)) return;
    const SnapDev &S = snaps[sy];
    const int i = bx * 256 + threadIdx.x;
    if (i >= S.n_src) return;
    const double *sp = S.order_base >= 0 ? src_ord + D * (S.order_base + i) : S.src + 3 * (size_t)i;
    double s[3], g[3];
    int l0[3];
    for (int a = 0; a < D; ++a) s[a] = sp[a];
    const int key = src_cell<D>(S, s, g, l0);
    rank[S.src_base + i] = wave_rank(bins + S.bin_base, key);
}

// Exclusive scan of nb counts in place (b[nb] receives the total), by one
// 1024-thread workgroup.  Chunks of 1024 x 16 counts: each thread takes 16
// consecutive counts, with all its loads in flight before any is used (16-byte
// loads when b is 16-byte aligned), scans them in registers, and adds the
// prefix of the thread sums before it (wavefront shuffles, then one value per
// wavefront through LDS).  A snapshot of up to 16384 sub-bins is one chunk,
// one round trip to memory.
__device__ void scan_counts(int *b, long long nb) {
    constexpr int PT = 16;
    constexpr long long CH = 1024LL * PT;
    __shared__ int wsum[16];
    __shared__ int carry_sh;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const bool vec = ((unsigned long long)b & 15ull) == 0;
    if (tid == 0) carry_sh = 0;
    __syncthreads();
    for (long long base = 0; base < nb; base += CH) {
        const long long i0 = base + (long long)PT * tid;
        int v[PT];
        if (vec && i0 + PT <= nb) {
            const int4 *q4 = (const int4 *)(b + i0);
#pragma unroll
            for (int q = 0; q < PT / 4; ++q) {
                const int4 t = q4[q];
                v[4 * q] = t.x;
                v[4 * q + 1] = t.y;
                v[4 * q + 2] = t.z;
                v[4 * q + 3] = t.w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < PT; ++q) v[q] = i0 + q < nb ? b[i0 + q] : 0;
        }
        int tsum = 0;
#pragma unroll
        for (int q = 0; q < PT; ++q) tsum += v[q];
        // inclusive scan of tsum across the wave
        int x = tsum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            int y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wv] = x;
        __syncthreads();
        int wpre = 0, total = 0;
        for (int k = 0; k < 16; ++k) {
            int t = wsum[k];
            if (k < wv) wpre += t;
            total += t;
        }
        int run = carry_sh + wpre + x - tsum;
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            const int c = v[q];
            v[q] = run;
            run += c;
        }
        if (vec && i0 + PT <= nb) {
            int4 *q4 = (int4 *)(b + i0);
#pragma unroll
            for (int q = 0; q < PT / 4; ++q) q4[q] = make_int4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
        } else {
#pragma unroll
            for (int q = 0; q < PT; ++q)
                if (i0 + q < nb) b[i0 + q] = v[q];
        }
        __syncthreads();
        if (tid == 0) carry_sh += total;
        __syncthreads();
    }
    if (tid == 0) b[nb] = carry_sh;
}

__global__ __launch_bounds__(1024) void k_scan(const SnapDev *snaps, int *bins) {
    const SnapDev &S = snaps[blockIdx.x];
    long long nb = 1;
    for (int a = 0; a < S.dim; ++a) nb *= S.nsb[a];
    scan_counts(bins + S.bin_base, nb);
}


template <int D>
__global__ __launch_bounds__(256) void k_order_count(const SnapDev *snaps, const OrderGroup *groups, int *counts,
                                                     int *rank) {
    const OrderGroup G = groups[blockIdx.y];
    const SnapDev &S = snaps[G.snap];
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= G.n_src) return;
    double s[3], g[3];
    int l0[3];
    for (int a = 0; a < D; ++a) s[a] = S.src[3 * (size_t)j + a];
    rank[G.base + j] = atomicAdd(&counts[G.cnt_base + src_cell<D>(S, s, g, l0)], 1);
}

__global__ __launch_bounds__(1024) void k_order_scan(const OrderGroup *groups, int *counts) {
    const OrderGroup G = groups[blockIdx.x];
    scan_counts(counts + G.cnt_base, G.nb);
}

template <int D>
__global__ __launch_bounds__(256) void k_order_place(const SnapDev *snaps, const OrderGroup *groups,
                                                     const int *starts, const int *rank, int *perm,
                                                     double *src_ord) {
    const OrderGroup G = groups[blockIdx.y];
    const SnapDev &S = snaps[G.snap];
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= G.n_src) return;
    double s[3], g[3];
    int l0[3];
    for (int a = 0; a < D; ++a) s[a] = S.src[3 * (size_t)j + a];
    const long long pos = G.base + starts[G.cnt_base + src_cell<D>(S, s, g, l0)] + rank[G.base + j];
    perm[pos] = j;
    for (int a = 0; a < D; ++a) src_ord[D * pos + a] = s[a];  // D coordinates per source
}

template <typename R, int D>
__global__ __launch_bounds__(256) void k_scatter(const SnapDev *snaps, int gx, int n_snap, const int *perm,
                                                 const double *src_ord, const int *bins, const int *rank,
                                                 Rec<R, D> *recs, int *srcid) {
    int bx, sy;
    if (!snap_block(gx, n_snap, bx, sy)) return;
    const SnapDev &S = snaps[sy];
    const int i = bx * 256 + threadIdx.x;
    if (i >= S.n_src) return;
    const bool ord = S.order_base >= 0;
    const int j = ord ? perm[S.order_base + i] : i;
    const double *sp = ord ? src_ord + D * (S.order_base + i) : S.src + 3 * (size_t)i;
    double s[3], g[3];
    int l0[3];
    for (int a = 0; a < D; ++a) s[a] = sp[a];
    int key = src_cell<D>(S, s, g, l0);
    long long pos = (long long)bins[S.bin_base + key] + rank[S.src_base + i];
    double c = S.flux[j];
    if (S.beam) c *= S.beam[j];
    double t = 0.0;
    for (int a = 0; a < D; ++a) t += S.pre_turn[a] * (s[a] - S.s_c[a]);
    double sn, cs;
    sincos_turns(t, &sn, &cs);
    Rec<R, D> r;
    for (int a = 0; a < D; ++a) {
        r.l0[a] = l0[a];
        r.off[a] = (R)(g[a] - l0[a]);
    }
    r.cr = (R)(c * cs);
    r.ci = (R)(c * sn);
    recs[S.src_base + pos] = r;
    if (srcid) srcid[S.src_base + pos] = j;
}

// Deterministic mode: the scatter's ranks follow the order of returning
// atomics, so the records of one sub-bin land in an order that changes from
// run to run.  Here every record moves to its stable place in its sub-bin:
// the number of records of the same sub-bin with a smaller source index.
// One thread per record position; the sub-bin is found by binary search in
// the scanned counts, and the rank by a pass over the sub-bin's source
// indices (sub-bins hold few records).
template <typename R, int D>
__global__ __launch_bounds__(256) void k_stable(const SnapDev *snaps, int gx, int n_snap, const int *bins,
                                                const int *srcid, const Rec<R, D> *in, Rec<R, D> *out) {
    int bx, sy;
    if (!snap_block(gx, n_snap, bx, sy)) return;
    const SnapDev &S = snaps[sy];
    const int pos = bx * 256 + threadIdx.x;
    if (pos >= S.n_src) return;
    long long nb = 1;
    for (int a = 0; a < D; ++a) nb *= S.nsb[a];
    const int *b = bins + S.bin_base;
    // last sub-bin whose start is at or before pos
    long long lo = 0, hi = nb - 1;
    while (lo < hi) {
        const long long mid = (lo + hi + 1) >> 1;
        if (b[mid] <= pos) lo = mid;
        else hi = mid - 1;
    }
    const int st = b[lo], en = b[lo + 1];
    const int *ids = srcid + S.src_base;
    const int me = ids[pos];
    int r = 0;
    for (int q = st; q < en; ++q) r += ids[q] < me;
    out[S.src_base + st + r] = in[S.src_base + pos];
}

// 1/psi2hat(m) for m = l - n1/2, psi2hat(m) = alpha2 phihat(alpha2 m), alpha2 = w pi / n2.
template <typename R>
__global__ __launch_bounds__(256) void k_ipsi(const SnapDev *snaps, R *ipsi) {
    const SnapDev &S = snaps[blockIdx.y];
    int idx = blockIdx.x * 256 + threadIdx.x;
    int a = 0, l = idx;
    while (a < S.dim && l >= S.n1[a]) {
        l -= S.n1[a];
        ++a;
    }
    if (a >= S.dim) return;
    double alpha2 = S.w * M_PI / S.n2[a];
    double m = (double)(l - S.n1[a] / 2);
    double v = alpha2 * phihat_quad(alpha2 * m, S.qn);
    ipsi[S.ipsi_base + idx] = (R)(1.0 / v);
}

template <typename R, int D, int W>
struct SpreadCfg {
    static constexpr int BX = TileShape<D>::X, BY = TileShape<D>::Y, BZ = TileShape<D>::Z;
    static constexpr int WPB = BX / 8;      // wavefronts per block, one 8-column slice each
    static constexpr int NT = BY / 8;       // 8 x 8 sub-tiles per slice (along y)
    static constexpr int TZ = BZ;           // z slices per sub-tile (registers per lane)
    static constexpr int MAXROWS = 64;      // sub-bin rows of one sub-tile (bounded below)
    static constexpr int WAVE_BYTES = 64 * D * W * (int)sizeof(R) + 2 * MAXROWS * (int)sizeof(int);
    static_assert(((8 + W - 1 + kSubBin - 1) / kSubBin + 1) *
                          (D == 3 ? ((TZ + W - 1 + kSubBinZ - 1) / kSubBinZ + 1) : 1) <= MAXROWS,
                  "too many sub-bin rows per sub-tile");
    static_assert(WPB * WAVE_BYTES <= 160 * 1024, "spread staging does not fit in LDS");
};


// Spreading (gather form).  Each lane owns one cell of an 8 x 8 sub-tile (and
// TZ z slices in 3-D) and keeps its sum in registers.  The records of the
// sub-tile's neighbourhood (a few contiguous ranges of the sorted records, one
// per sub-bin row) are taken 64 at a time: each lane loads one record and
// writes that record's w kernel weights per axis to LDS; then, record by
// record, every lane looks up the two (three) weights of its own cell and
// accumulates.  No atomics; each grid cell is written once, after
// multiplication by 1/psi2hat (the first deconvolution).
template <typename R, int D, int W>
__global__ __launch_bounds__(256) void k_spread(const SnapDev *snaps, int gx, int n_snap, const int *bins,
                                                const Rec<R, D> *recs, const R *ipsi, cplx<R> *grid, EsPoly ep) {
    using Cfg = SpreadCfg<R, D, W>;
    extern __shared__ __align__(16) char smem[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int blk, sy;
    if (!snap_block(gx, n_snap, blk, sy)) return;
    const SnapDev &S = snaps[sy];
    const int nbx = (S.n1[0] + Cfg::BX - 1) / Cfg::BX, nby = (S.n1[1] + Cfg::BY - 1) / Cfg::BY;
    const int nbz = D == 3 ? (S.n1[2] + Cfg::BZ - 1) / Cfg::BZ : 1;
    if (blk >= nbx * nby * nbz) return;
    const int x0 = (blk % nbx) * Cfg::BX + 8 * wave;
    if (x0 >= S.n1[0]) return;
    const int yb = ((blk / nbx) % nby) * Cfg::BY;
    const int z0 = D == 3 ? (blk / (nbx * nby)) * Cfg::BZ : 0;
    R *kw = (R *)(smem + wave * Cfg::WAVE_BYTES);  // [64][D][W]
    int *rstart = (int *)(kw + 64 * D * W);
    int *rpre = rstart + Cfg::MAXROWS;
    const int cx = lane & 7, cy = lane >> 3;
    const R beta = (R)S.beta;
    const R inv_hw = (R)(2.0 / W);
    const Rec<R, D> *rs = recs + S.src_base;
    const int *bb = bins + S.bin_base;
    const R *ix_t = ipsi + S.ipsi_base;
    const R *iy_t = ix_t + S.n1[0];
    const R *iz_t = iy_t + S.n1[1];
    cplx<R> *dst = grid + S.bufA;
    const int sx_lo = max(0, x0 - W + 1) / kSubBin, sx_hi = min(S.n1[0] - W, x0 + 7) / kSubBin;
    int sz_lo = 0, sz_hi = 0;
    if (D == 3) {
        sz_lo = max(0, z0 - W + 1) / kSubBinZ;
        sz_hi = min(S.n1[2] - W, z0 + Cfg::TZ - 1) / kSubBinZ;
    }
    for (int t = 0; t < Cfg::NT; ++t) {
        const int y0 = yb + 8 * t;
        if (y0 >= S.n1[1]) break;
        const int sy_lo = max(0, y0 - W + 1) / kSubBin, sy_hi = min(S.n1[1] - W, y0 + 7) / kSubBin;
        const int ny = sy_hi - sy_lo + 1;
        const int nrows = ny * (sz_hi - sz_lo + 1);
        int cnt = 0, st = 0;
        if (lane < nrows) {
            const int sy = sy_lo + lane % ny, sz = sz_lo + lane / ny;
            const long long row = ((long long)sz * S.nsb[1] + sy) * S.nsb[0];
            st = bb[row + sx_lo];
            cnt = bb[row + sx_hi + 1] - st;
        }
        int inc = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(inc, off, 64);
            if (lane >= off) inc += y;
        }
        const int total = __shfl(inc, 63, 64);
        wave_sync();
        if (lane < nrows) {
            rstart[lane] = st;
            rpre[lane] = inc - cnt;
        }
        wave_sync();
        R accr[Cfg::TZ], acci[Cfg::TZ];
#pragma unroll
        for (int k = 0; k < Cfg::TZ; ++k) accr[k] = acci[k] = 0;
        // FP32: per-batch sums added in FP64 (as in the matrix-core spread)
        constexpr bool kBlocked = std::is_same<R, float>::value;
        double sumr[Cfg::TZ], sumi[Cfg::TZ];
#pragma unroll
        for (int k = 0; k < Cfg::TZ; ++k) sumr[k] = sumi[k] = 0.0;
        for (int b0 = 0; b0 < total; b0 += 64) {
            const int e = b0 + lane;
            int ml0x = -1000000, ml0y = -1000000, ml0z = -1000000;
            R mcr = 0, mci = 0;
            bool hit = false;
            if (e < total) {
                int row = 0;
                while (row + 1 < nrows && rpre[row + 1] <= e) ++row;
                const Rec<R, D> r = rs[rstart[row] + (e - rpre[row])];
                ml0x = r.l0[0] - x0;
                ml0y = r.l0[1] - y0;
                if constexpr (D == 3) ml0z = r.l0[2] - z0;
                hit = ml0x > -W && ml0x < 8 && ml0y > -W && ml0y < 8 &&
                      (D == 2 || (ml0z > -W && ml0z < Cfg::TZ));
                mcr = r.cr;
                mci = r.ci;
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    R wt[W];
                    bool exact = true;
                    if constexpr (std::is_same<R, float>::value && W <= kPolyMaxW) {
                        // the offset lies in (W/2 - 1, W/2] up to rounding at the grid's edge
                        const float u = 2.0f * r.off[a] - (float)(W - 1);
                        if (fabsf(u) <= 1.001f) {
                            es_weights_poly<W>(ep, u, wt);
                            exact = false;
                        }
                    }
                    if (exact)
#pragma unroll
                        for (int i = 0; i < W; ++i) wt[i] = es_phi_fast((R)((R)i - r.off[a]) * inv_hw, beta);
#pragma unroll
                    for (int i = 0; i < W; ++i) kw[(lane * D + a) * W + i] = wt[i];
                }
            }
            wave_sync();
            unsigned long long hm = __ballot(hit);
            while (hm) {
                const int r = __ffsll((long long)hm) - 1;
                hm &= hm - 1;
                const int dx = cx - readlane_i(ml0x, r), dy = cy - readlane_i(ml0y, r);
                const R cr = readlane_r<R>(mcr, r), ci = readlane_r<R>(mci, r);
                const R *kr = kw + r * D * W;
                const bool in = (unsigned)dx < (unsigned)W && (unsigned)dy < (unsigned)W;
                const R wxy = in ? kr[dx] * kr[W + dy] : (R)0;
                if constexpr (D == 2) {
                    accr[0] += wxy * cr;
                    acci[0] += wxy * ci;
                } else {
                    const int l0z = readlane_i(ml0z, r);
#pragma unroll
                    for (int k = 0; k < Cfg::TZ; ++k) {
                        const int dz = k - l0z;
                        if ((unsigned)dz < (unsigned)W) {  // uniform across the wave
                            const R wz = kr[2 * W + dz];
                            accr[k] += wxy * wz * cr;
                            acci[k] += wxy * wz * ci;
                        }
                    }
                }
            }
            if constexpr (kBlocked) {
#pragma unroll
                for (int k = 0; k < Cfg::TZ; ++k) {
                    sumr[k] += (double)accr[k];
                    sumi[k] += (double)acci[k];
                    accr[k] = acci[k] = 0;
                }
            }
            wave_sync();
        }
        // flush: divide by psi2hat at the modes and store each owned cell once
        const int ox = x0 + cx, oy = y0 + cy;
        if (ox < S.n1[0] && oy < S.n1[1]) {
            const R fxy = ix_t[ox] * iy_t[oy];
#pragma unroll
            for (int k = 0; k < Cfg::TZ; ++k) {
                const int oz = z0 + k;
                if (D == 3 && oz >= S.n1[2]) break;
                const R f = D == 3 ? fxy * iz_t[oz] : fxy;
                if constexpr (kBlocked)
                    dst[((long long)oz * S.n1[1] + oy) * S.n1[0] + ox] =
                        cmake<R>((R)(sumr[k] * (double)f), (R)(sumi[k] * (double)f));
                else
                    dst[((long long)oz * S.n1[1] + oy) * S.n1[0] + ox] = cmake<R>(accr[k] * f, acci[k] * f);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// 2-D spreading on the matrix cores.  The spread into one 16 x 16 tile is a
// sum of outer products over the tile's records r,
//     b[y][x] = sum_r ky_r(y) * (c'_r kx_r(x)),
// i.e. the 16 x 16 x R product KY^T (C KX), accumulated 4 records at a time
// by v_mfma_{f32,f64}_16x16x4 (A = y weights of 4 records, B = strength-scaled
// x weights, real and imaginary parts in two accumulators).  Each lane stages
// one record at a time in LDS with its 2 W kernel weights (evaluated once per
// record and tile), then builds one A and one B element per step by lookup:
// its cell's byte offsets from the record's first cell along both axes, as the
// two 16-bit halves of one register, taken as unsigned and capped at the zero
// that sits between the record's y and x weights (cells before or past the
// footprint land there; the x weights are stored in reverse, so that the same
// cap reaches the zero from their side).
template <typename R, int W>
struct SpreadMfmaCfg {
    static constexpr int T = 16;            // tile edge
    // one wavefront per workgroup: tiles differ widely in record count, and a
    // workgroup's LDS stays held until its slowest wavefront ends
    static constexpr int WPB = 1;           // wavefronts (tiles) per block, along x
    static constexpr int BX = T * WPB, BY = T;
    static constexpr int MAXROWS = 8;       // sub-bin rows per tile
    // FP32 with w <= 8 (every FP32 width in use) fits 7 wavefronts per SIMD
    // without spills; wider and FP64 kernels take what their registers allow
    static constexpr int MIN_WAVES = std::is_same<R, float>::value && W <= 8 ? 7 : 1;
    // staged records: cr, ci (R); the first cell's offsets from the tile
    // corner in bytes, x and y as the two 16-bit halves of one int; one row of
    // 2 W + 1 weights (R): y weights 0 .. W - 1, a zero, x weights W - 1 .. 0
    static constexpr int WS = 2 * W + 1;    // weight row stride (odd: rows start in distinct banks)
    static constexpr int WAVE_BYTES = 64 * ((int)sizeof(int) + (2 + WS) * (int)sizeof(R));
    static_assert((T + W - 1 + kSubBin - 1) / kSubBin + 1 <= MAXROWS, "too many sub-bin rows per tile");
};
// first-cell offset, in bytes, of the staged slots past a batch's last record:
// every lane's offset from it is negative as a 16-bit value
constexpr int kFarBytes = 0x3000;
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

template <typename R, int W>
__global__ __launch_bounds__((64 * SpreadMfmaCfg<R, W>::WPB))
__attribute__((amdgpu_waves_per_eu(SpreadMfmaCfg<R, W>::MIN_WAVES))) void k_spread_mfma(const SnapDev *snaps, int gx,
                                                                             int n_snap, const int *bins,
                                                                             const Rec<R, 2> *recs,
                                                                             const R *ipsi, cplx<R> *grid,
                                                                             EsPoly ep) {
    using Cfg = SpreadMfmaCfg<R, W>;
    using MA = MfmaAcc<R>;
    extern __shared__ __align__(16) char smem[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int blk, sy;
    if (!snap_block(gx, n_snap, blk, sy)) return;
    const SnapDev &S = snaps[sy];
    const int nbx = (S.n1[0] + Cfg::BX - 1) / Cfg::BX, nby = (S.n1[1] + Cfg::BY - 1) / Cfg::BY;
    if (blk >= nbx * nby) return;
    const int x0 = (blk % nbx) * Cfg::BX + Cfg::T * wave;
    if (x0 >= S.n1[0]) return;
    const int y0 = (blk / nbx) * Cfg::BY;
    using R2 = typename std::conditional<std::is_same<R, float>::value, float2, double2>::type;
    char *wbase = smem + wave * Cfg::WAVE_BYTES;
    R2 *sc = (R2 *)wbase;                 // strength (re, im) per staged record
    int *sl0 = (int *)(sc + 64);          // first-cell offsets (x low, y high 16 bits) per staged record
    R *skw = (R *)(sl0 + 64);             // [64][2 W + 1] kernel weights per staged record
    skw[lane * Cfg::WS + W] = 0;          // the zero between the y and x weights, never overwritten
    const R beta = (R)S.beta;
    const R inv_hw = (R)(2.0 / W);
    const Rec<R, 2> *rs = recs + S.src_base;
    const int *bb = bins + S.bin_base;
    // sub-bin rows of records whose footprint meets the tile
    const int sx_lo = max(0, x0 - W + 1) / kSubBin, sx_hi = min(S.n1[0] - W, x0 + Cfg::T - 1) / kSubBin;
    const int sy_lo = max(0, y0 - W + 1) / kSubBin, sy_hi = min(S.n1[1] - W, y0 + Cfg::T - 1) / kSubBin;
    const int nrows = (sx_lo > sx_hi || sy_lo > sy_hi) ? 0 : sy_hi - sy_lo + 1;
    // the deconvolution factors of the owned cells (1/psi2hat at the modes),
    // loaded now so that their latency overlaps the tile's record chain
    const R *ix_t = ipsi + S.ipsi_base;
    const R *iy_t = ix_t + S.n1[0];
    const int cx_ = x0 + (lane & 15);
    const bool cx_in = cx_ < S.n1[0];
    const R fx = cx_in ? ix_t[cx_] : (R)0;
    R fy[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int cy_ = y0 + MfmaAcc<R>::row(lane, r);
        fy[r] = cy_ < S.n1[1] ? iy_t[cy_] : (R)0;
    }
    int cnt = 0, st = 0;
    if (lane < nrows) {
        const long long row = (long long)(sy_lo + lane) * S.nsb[0];
        st = bb[row + sx_lo];
        cnt = bb[row + sx_hi + 1] - st;
    }
    // per sub-bin row (wave-uniform, in scalar registers): the window position
    // of its first record, and the change from the previous row of the offset
    // from window position to record index; rows past nrows start at total,
    // beyond every position.  The rows' counts are read lane by lane into
    // scalar registers and summed there (no shuffle round trips).
    int rpre[Cfg::MAXROWS], rdd[Cfg::MAXROWS];
    int pre = 0, prev = 0;
#pragma unroll
    for (int r = 0; r < Cfg::MAXROWS; ++r) {
        const int c = readlane_i(cnt, r), s0 = readlane_i(st, r);
        rpre[r] = pre;
        const int del = s0 - pre;
        rdd[r] = del - prev;
        prev = del;
        pre += c;
    }
    const int total = pre;
    typename MA::T accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
    // FP32 tiles: each batch of 64 records is summed on the matrix cores from
    // zero and the batch sums are added in FP64, so the rounding error of a
    // cell does not grow with the number of records that reach it
    constexpr bool kBlocked = std::is_same<R, float>::value;
    double sumr[4] = {0, 0, 0, 0}, sumi[4] = {0, 0, 0, 0};
    const int li = lane & 15, lk = lane >> 4;  // A row / B column index, record slot of the 4
    const int lib = li * (int)sizeof(R);
    // the lane's cell offset in bytes, twice, for the 16-bit differences of
    // both axes at once; their cap is the zero weight (offsets before or past
    // a record's footprint wrap or exceed it)
    const s16x2 lib2 = {(short)lib, (short)lib};
    const u16x2 span2 = {(unsigned short)(W * sizeof(R)), (unsigned short)(W * sizeof(R))};
    // record e of the tile's neighbourhood (a position in its sub-bin rows):
    // its row is the last one starting at or before e, and the row starts are
    // nondecreasing, so the changes of the rows starting at or before e add up
    // to that row's offset
    auto fetch = [&](int e) {
        int d = rdd[0];
#pragma unroll
        for (int r = 1; r < Cfg::MAXROWS; ++r) d += rpre[r] <= e ? rdd[r] : 0;
        return rs[e + d];
    };
    // each batch's records are loaded while the previous batch is on the matrix cores
    Rec<R, 2> nxt;
    if (lane < total) nxt = fetch(lane);
    for (int b0 = 0; b0 < total; b0 += 64) {
        const int e = b0 + lane;
        if (e < total) {
            const Rec<R, 2> r = nxt;
            // first-cell offsets from the tile corner, in bytes of R
            // |offset| <= (W + 2 kSubBin) cells: well inside 16 bits
            sl0[lane] = (int)(((unsigned)((r.l0[1] - y0) * (int)sizeof(R)) << 16) |
                              ((unsigned)((r.l0[0] - x0) * (int)sizeof(R)) & 0xffffu));
            sc[lane].x = r.cr;
            sc[lane].y = r.ci;
            R wx[W], wy[W];
            bool exact = true;
            if constexpr (std::is_same<R, float>::value && W <= kPolyMaxW) {
                // the offsets lie in (W/2 - 1, W/2] (up to rounding where the first
                // cell is clamped at the grid's edge; the exact kernel takes any other)
                const float ux = 2.0f * r.off[0] - (float)(W - 1), uy = 2.0f * r.off[1] - (float)(W - 1);
                if (fabsf(ux) <= 1.001f && fabsf(uy) <= 1.001f) {
                    es_weights_poly<W>(ep, ux, wx);
                    es_weights_poly<W>(ep, uy, wy);
                    exact = false;
                }
            }
            if (exact) {
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    wx[i] = es_phi_fast((R)((R)i - r.off[0]) * inv_hw, beta);
                    wy[i] = es_phi_fast((R)((R)i - r.off[1]) * inv_hw, beta);
                }
            }
#pragma unroll
            for (int i = 0; i < W; ++i) {
                skw[lane * Cfg::WS + i] = wy[i];
                skw[lane * Cfg::WS + 2 * W - i] = wx[i];
            }
        } else {
            // past the last record: a corner no tile cell reaches, so the
            // steps below read in-bounds weights and contribute zero
            sl0[lane] = (kFarBytes << 16) | kFarBytes;
            sc[lane].x = 0;
            sc[lane].y = 0;
        }
        wave_sync();
        if (e + 64 < total) nxt = fetch(e + 64);
        const int nb = min(64, total - b0);
        // 16 records (4 matrix-core steps) at a time, with no branches, so that
        // the steps' LDS reads are in flight together; slots past nb hold the
        // corner above
        for (int g0 = 0; g0 < nb; g0 += 16) {
            R a[4], bre[4], bim[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int rr = g0 + 4 * u + lk;
                const int o = sl0[rr];
                const R2 c = sc[rr];
                // bytes from the record's first cell, or the row's zero
                const u16x2 d = __builtin_elementwise_min(
                    __builtin_bit_cast(u16x2, (s16x2)(lib2 - __builtin_bit_cast(s16x2, o))), span2);
                const char *row = (const char *)(skw + rr * Cfg::WS);
                a[u] = *(const R *)(row + (unsigned)d.y);
                const R k = *(const R *)(row + 2 * W * sizeof(R) - (unsigned)d.x);
                bre[u] = c.x * k;
                bim[u] = c.y * k;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                accr = MA::step(a[u], bre[u], accr);
                acci = MA::step(a[u], bim[u], acci);
            }
        }
        if constexpr (kBlocked) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                sumr[r] += (double)accr[r];
                sumi[r] += (double)acci[r];
                accr[r] = 0;
                acci[r] = 0;
            }
        }
        wave_sync();
    }
    // flush: divide by psi2hat at the modes, store each owned cell once
    cplx<R> *dst = grid + S.bufA;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int cy_ = y0 + MA::row(lane, r);
        if (cx_in && cy_ < S.n1[1]) {
            const R f = fx * fy[r];
            if constexpr (kBlocked)
                dst[(long long)cy_ * S.n1[0] + cx_] = cmake<R>((R)(sumr[r] * (double)f), (R)(sumi[r] * (double)f));
            else
                dst[(long long)cy_ * S.n1[0] + cx_] = cmake<R>(accr[r] * f, acci[r] * f);
        }
    }
}

// ---------------------------------------------------------------------------
// FFT: mixed-radix decimation in frequency, in place in LDS, + sign.  A
// radix-r stage on sub-transforms of Ls points (q = Ls / r) takes, for each
// sub-transform start s0 and k < q, the r points s0 + k + j q, forms their
// r-point DFT and multiplies output j' by W_Ls^(j' k) before storing it back
// at s0 + k + j' q.  The input is in natural order; after the last stage
// X[q] sits at drev[q], with
//     drev(q) = (q mod r1) L / r1 + drev'(q div r1)
// over the radices r1, r2, ... in stage order (8s, 4s, 2s, 3s, 5s).
// a / b for 0 <= a < 2^23 with a float reciprocal and one correction step.
__device__ __forceinline__ int fdiv(int a, int b, float inv_b) {
    int q = (int)((float)a * inv_b);
    const int r = a - q * b;
    q += (r >= b) - (r < 0);
    return q;
}

template <typename R>
__device__ __forceinline__ void dft4(cplx<R> &x0, cplx<R> &x1, cplx<R> &x2, cplx<R> &x3) {
    const cplx<R> a = cadd<R>(x0, x2), b = csub<R>(x0, x2);
    const cplx<R> c = cadd<R>(x1, x3), d = cmuli<R>(csub<R>(x1, x3));
    x0 = cadd<R>(a, c);
    x2 = csub<R>(a, c);
    x1 = cadd<R>(b, d);
    x3 = csub<R>(b, d);
}

template <typename R, int RAD>
__device__ __forceinline__ void dft_small(cplx<R> *v) {
    if (RAD == 2) {
        cplx<R> a = v[0], b = v[1];
        v[0] = cadd<R>(a, b);
        v[1] = csub<R>(a, b);
    } else if (RAD == 3) {
        const R s3 = (R)0.86602540378443864676;
        cplx<R> t1 = cadd<R>(v[1], v[2]), t2 = csub<R>(v[1], v[2]);
        cplx<R> m = cmake<R>(v[0].x - (R)0.5 * t1.x, v[0].y - (R)0.5 * t1.y);
        cplx<R> it = cmuli<R>(cscale<R>(t2, s3));
        v[0] = cadd<R>(v[0], t1);
        v[1] = cadd<R>(m, it);
        v[2] = csub<R>(m, it);
    } else if (RAD == 4) {
        dft4<R>(v[0], v[1], v[2], v[3]);
    } else if (RAD == 5) {
        const R c1 = (R)0.30901699437494742410, c2 = (R)-0.80901699437494742410;
        const R s1 = (R)0.95105651629515357212, s2 = (R)0.58778525229247312917;
        cplx<R> a1 = cadd<R>(v[1], v[4]), b1 = csub<R>(v[1], v[4]);
        cplx<R> a2 = cadd<R>(v[2], v[3]), b2 = csub<R>(v[2], v[3]);
        cplx<R> x0 = v[0];
        cplx<R> r1 = cmake<R>(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
        cplx<R> r2 = cmake<R>(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
        cplx<R> i1 = cmuli<R>(cmake<R>(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
        cplx<R> i2 = cmuli<R>(cmake<R>(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
        v[0] = cadd<R>(x0, cadd<R>(a1, a2));
        v[1] = cadd<R>(r1, i1);
        v[4] = csub<R>(r1, i1);
        v[2] = cadd<R>(r2, i2);
        v[3] = csub<R>(r2, i2);
    } else if (RAD == 8) {
        // two 4-point DFTs of the even and odd inputs, combined with W_8^q
        const R h = (R)0.70710678118654752440;
        cplx<R> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
        cplx<R> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
        dft4<R>(e0, e1, e2, e3);
        dft4<R>(o0, o1, o2, o3);
        const cplx<R> t1 = cmake<R>(h * (o1.x - o1.y), h * (o1.x + o1.y));    // W8 o1
        const cplx<R> t2 = cmuli<R>(o2);                                       // W8^2 o2
        const cplx<R> t3 = cmake<R>(-h * (o3.x + o3.y), h * (o3.x - o3.y));   // W8^3 o3
        v[0] = cadd<R>(e0, o0);
        v[4] = csub<R>(e0, o0);
        v[1] = cadd<R>(e1, t1);
        v[5] = csub<R>(e1, t1);
        v[2] = cadd<R>(e2, t2);
        v[6] = csub<R>(e2, t2);
        v[3] = cadd<R>(e3, t3);
        v[7] = csub<R>(e3, t3);
    }
}

// W_N^t from the two LDS tables: coarse[t / 64] * fine[t % 64].
template <typename R>
__device__ __forceinline__ cplx<R> twiddle(const cplx<R> *coarse, const cplx<R> *fine, int t) {
    return cmul<R>(coarse[t >> 6], fine[t & 63]);
}

// LDS index of element e of a line: one pad complex every 16.
__device__ __forceinline__ int cpad(int e) { return e + (e >> 4); }

// One radix-RAD stage over the m lines of the workgroup.  Work item wi maps
// to butterfly b = wi mod L/RAD of line group g = wi div L/RAD; its indices
// and twiddles are formed once and applied to lines g, g + G, g + 2G, ...
template <typename R, int TPB, int RAD>
__device__ __forceinline__ void dif_stage(cplx<R> *buf, int L, int Lp, int m, int Ls, int p, const cplx<R> *twc,
                                          const cplx<R> *twf) {
    const int q = Ls / RAD;
    const int nb = L / RAD;
    const int G = max(1, min(m, TPB / nb));
    const float invnb = 1.0f / (float)nb, invq = 1.0f / (float)q;
#pragma unroll 1
    for (int wi = threadIdx.x; wi < nb * G; wi += TPB) {
        const int g = G == 1 ? 0 : fdiv(wi, nb, invnb);
        const int b = wi - g * nb;
        const int blk = q == 1 ? b : fdiv(b, q, invq);
        const int k = b - blk * q;
        const int base = blk * Ls + k;
        int addr[RAD];
#pragma unroll
        for (int j = 0; j < RAD; ++j) addr[j] = cpad(base + j * q);
        cplx<R> tw[RAD];
#pragma unroll
        for (int j = 1; j < RAD; ++j) tw[j] = twiddle<R>(twc, twf, 2 * j * k * p);  // W_N^(2 j k p) = W_Ls^(j k)
#pragma unroll 1
        for (int line = g; line < m; line += G) {
            cplx<R> *s_ = buf + line * Lp;
            cplx<R> v[RAD];
#pragma unroll
            for (int j = 0; j < RAD; ++j) v[j] = s_[addr[j]];
            dft_small<R, RAD>(v);
#pragma unroll
            for (int j = 1; j < RAD; ++j) v[j] = cmul<R>(v[j], tw[j]);
#pragma unroll
            for (int j = 0; j < RAD; ++j) s_[addr[j]] = v[j];
        }
    }
    __syncthreads();
}

template <typename R, int TPB>
__device__ void dif_fft(cplx<R> *buf, int L, int Lp, int m, const cplx<R> *twc, const cplx<R> *twf) {
    int Ls = L, p = 1;
    while (Ls % 8 == 0) { dif_stage<R, TPB, 8>(buf, L, Lp, m, Ls, p, twc, twf); Ls /= 8; p *= 8; }
    while (Ls % 4 == 0) { dif_stage<R, TPB, 4>(buf, L, Lp, m, Ls, p, twc, twf); Ls /= 4; p *= 4; }
    while (Ls % 2 == 0) { dif_stage<R, TPB, 2>(buf, L, Lp, m, Ls, p, twc, twf); Ls /= 2; p *= 2; }
    while (Ls % 3 == 0) { dif_stage<R, TPB, 3>(buf, L, Lp, m, Ls, p, twc, twf); Ls /= 3; p *= 3; }
    while (Ls % 5 == 0) { dif_stage<R, TPB, 5>(buf, L, Lp, m, Ls, p, twc, twf); Ls /= 5; p *= 5; }
}

// Output position of X[q] of an L-point transform (same radix order as dif_fft).
__global__ void k_digrev(int L, int *drev) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= L) return;
    int pos = 0, Ls = L, rem = q;
    const int radices[5] = {8, 4, 2, 3, 5};
    for (int ri = 0; ri < 5; ++ri) {
        const int r = radices[ri];
        while (Ls % r == 0) {
            Ls /= r;
            pos += (rem % r) * Ls;
            rem /= r;
        }
    }
    drev[q] = pos;
}

// grid loads per thread in flight in a pass's input phase (fewer FP64 values
// keep the FP64 passes' register count, and so their occupancy)
template <typename R>
constexpr int kFftLoads = sizeof(R) == 4 ? 8 : 4;

// Physical workgroup b runs on XCD b mod 8 (round-robin dispatch); logical
// workgroups are handed out so that each XCD gets one contiguous range, and
// neighbouring line groups, which share cache lines, share an L2.  nblk is a
// multiple of 8.
__device__ __forceinline__ long long xcd_order(long long b, long long nblk) {
    return (b & 7) * (nblk >> 3) + (b >> 3);
}

// One pass along axis `a` for every snapshot.  A line holds the n1 deconvolved
// mode values b~_m, m in [-n1/2, n1/2); the pass evaluates
// g_p = sum_m b~_m W_N^(m p), N = n2 = 2 n1, at p in [-P, P] only.  With
// a[j] = b~_m at j = m mod n1, the even outputs are g_2k = sum_j a[j] W_n1^(jk)
// and the odd outputs g_2k+1 = sum_j s_j a[j] W_N^j W_n1^(jk), s_j = +1 for
// j < n1/2 and -1 otherwise (W_N^n1 = -1): each line becomes two n1-point
// transforms held side by side in LDS (2 cx transforms per workgroup, one
// index and twiddle computation per butterfly for all of them), with no zero
// padding stored.  Outputs of both parities are written interleaved, in order.
// Input layout [slow: n1 of axes > a][n1_a][fast: M of axes < a]; output
// [slow][M_a][fast].  When the fast extent is 1 (the x pass) a workgroup takes
// cx consecutive rows, else cx consecutive columns of one slow index.
// Passes alternate bufA -> bufB -> bufA (-> bufB).
template <typename R, int TPB>
__global__ __launch_bounds__(TPB) void k_fft(const SnapDev *snaps, int a, cplx<R> *grid) {
    extern __shared__ __align__(16) char smem[];
    const SnapDev &S = snaps[blockIdx.y];
    const int N = S.n2[a], L = S.n1[a], Ma = S.M[a], Pa = S.P[a], CX = S.cx[a];
    const int Lp = cline_pad(L), half = L / 2;
    long long F = 1, Sl = 1;
    for (int b = 0; b < a; ++b) F *= S.M[b];
    for (int b = a + 1; b < S.dim; ++b) Sl *= S.n1[b];
    const bool rows = F == 1;
    const long long ngrp = rows ? (Sl + CX - 1) / CX : (F + CX - 1) / CX;
    const long long nblk = rows ? ngrp : Sl * ngrp;
    long long wl = xcd_order((long long)blockIdx.x, (long long)gridDim.x);
    // split passes: workgroups 2 g and 2 g + 1 take the even and the odd
    // transforms of line group g (half the LDS each, twice the workgroups)
    const bool split = S.fft_split[a] != 0;
    int only = 0;
    if (split) {
        only = (int)(wl & 1);
        wl >>= 1;
    }
    if (wl >= nblk) return;
    const int tps = split ? 1 : 2;  // transforms per line held in LDS
    const bool fromA = (a % 2) == 0;
    const cplx<R> *in = grid + (fromA ? S.bufA : S.bufB);
    cplx<R> *out = grid + (fromA ? S.bufB : S.bufA);
    int cx;
    long long in_ls, out_ls;  // line strides; element strides are 1 (rows) or F (columns)
    if (rows) {
        const long long o0 = wl * CX;
        cx = (int)min((long long)CX, Sl - o0);
        in += o0 * L;
        out += o0 * Ma;
        in_ls = L;
        out_ls = Ma;
    } else {
        const long long o = wl / ngrp, i0 = (wl - o * ngrp) * CX;
        cx = (int)min((long long)CX, F - i0);
        in += o * ((long long)L * F) + i0;
        out += o * ((long long)Ma * F) + i0;
        in_ls = 1;
        out_ls = 1;
    }
    cplx<R> *twc = (cplx<R> *)smem;  // [N/64 + 1] coarse, then [64] fine twiddles of W_N
    cplx<R> *twf = twc + (N >> 6) + 1;
    cplx<R> *buf = twf + 64;              // [tps cx][Lp]: line tps c (+ 1): even (odd) outputs
    const cplx<R> *tw = (const cplx<R> *)S.tw[a];
    for (int t = threadIdx.x; t < (N >> 6) + 1 + 64; t += TPB) {
        const int g = t <= (N >> 6) ? t << 6 : t - (N >> 6) - 1;
        twc[t] = tw[g < N ? g : 0];
    }
    __syncthreads();
    // kFftLoads<R> grid loads per thread are issued before any is used (one load
    // at a time leaves the pass waiting on memory latency)
    const float invL = 1.0f / (float)L, invcx = 1.0f / (float)cx;
    for (int e0 = threadIdx.x; e0 < cx * L; e0 += kFftLoads<R> * TPB) {
        int lj[kFftLoads<R>], cj[kFftLoads<R>];
        cplx<R> v[kFftLoads<R>];
#pragma unroll
        for (int u = 0; u < kFftLoads<R>; ++u) {
            const int e = e0 + u * TPB;
            lj[u] = 0;
            cj[u] = 0;
            if (e < cx * L) {
                long long src;
                if (rows) {
                    cj[u] = fdiv(e, L, invL);
                    lj[u] = e - cj[u] * L;
                    src = cj[u] * in_ls + lj[u];
                } else {
                    lj[u] = fdiv(e, cx, invcx);
                    cj[u] = e - lj[u] * cx;
                    src = (long long)lj[u] * F + cj[u];
                }
                v[u] = in[src];
            }
        }
#pragma unroll
        for (int u = 0; u < kFftLoads<R>; ++u) {
            if (e0 + u * TPB < cx * L) {
                const int c = cj[u];
                int j = lj[u] + half;
                if (j >= L) j -= L;
                if (!split || only) {
                    cplx<R> vo = cmul<R>(v[u], twiddle<R>(twc, twf, j));
                    if (j >= half) vo = cmake<R>(-vo.x, -vo.y);
                    buf[(tps * c + tps - 1) * Lp + cpad(j)] = vo;
                }
                if (!split || !only) buf[(tps * c) * Lp + cpad(j)] = v[u];
            }
        }
    }
    __syncthreads();
    dif_fft<R, TPB>(buf, L, Lp, tps * cx, twc, twf);
    const int *drev = S.drev[a];
    // outputs p in [-P, P]; a split workgroup writes those of its parity,
    // p = p0 + 2 q (its partner fills the others)
    const int p0 = split ? (((-Pa) & 1) == only ? -Pa : -Pa + 1) : -Pa;
    const int step = split ? 2 : 1;
    const int cnt = (Pa - p0) / step + 1;
    const float invM = 1.0f / (float)cnt;
    for (int e = threadIdx.x; e < cx * cnt; e += TPB) {
        int qi, c;
        if (rows) {
            c = fdiv(e, cnt, invM);
            qi = e - c * cnt;
        } else {
            qi = fdiv(e, cx, invcx);
            c = e - qi * cx;
        }
        const int pp = p0 + step * qi, par = pp & 1;
        const long long pi = pp + Pa;
        const long long dst = rows ? c * out_ls + pi : pi * F + c;
        int k = (pp - par) >> 1;
        if (k < 0) k += L;
        if (k >= L) k -= L;
        out[dst] = buf[(tps * c + (split ? 0 : par)) * Lp + cpad(drev[k])];
    }
}

// Interpolation at the targets, deconvolution by psi1hat, centring phase,
// reflection undone, written to the caller's pair layout.
// DEG: some snapshot of the launch has a clamped axis, whose psi1hat is
// evaluated here by quadrature (a variant of its own: the quadrature's
// registers would halve the occupancy of the common case).
//
// Kernel weights of target t of snapshot S: per axis the W weights and the
// first cell of the window (from the window corner), and the target's
// coordinates b.
template <typename R, int D, int W>
__device__ __forceinline__ void interp_weights(const SnapDev &S, int t, const EsPoly &ep, R (&kw)[D][W],
                                               int (&p0)[3], double (&bb)[3]) {
    const R beta = (R)S.beta;
    const R inv_hw = (R)(2.0 / W);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double b = S.tb[(long long)a * S.n_tgt + t];
        bb[a] = b;
        const double q = S.qscale[a] * (b - S.b_c[a]);
        int p = (int)ceil(q - 0.5 * W);
        p = min(max(p, -S.P[a]), S.P[a] - W + 1);
        const R off = (R)(q - p);
        bool exact = true;
        if constexpr (std::is_same<R, float>::value && W <= kPolyMaxW) {
            // off lies in (W/2 - 1, W/2] unless the window clamp moved p
            const float u = 2.0f * off - (float)(W - 1);
            if (fabsf(u) <= 1.001f) {
                es_weights_poly<W>(ep, u, kw[a]);
                exact = false;
            }
        }
        if (exact)
#pragma unroll
            for (int i = 0; i < W; ++i) kw[a][i] = es_phi((R)((R)i - off) * inv_hw, beta);
        p0[a] = p + S.P[a];
    }
}

// The weighted sum of the W^D window cells of grid g (window dims of S).
template <typename R, int D, int W>
__device__ __forceinline__ void interp_sum(const SnapDev &S, const cplx<R> *g, const R (&kw)[D][W], const int (&p0)[3],
                                           R &ar, R &ai) {
    ar = 0;
    ai = 0;
    const long long My = S.M[1], Mx = S.M[0];
#pragma unroll 1
    for (int iz = 0; iz < (D == 3 ? W : 1); ++iz) {
        R zr = 0, zi = 0;
        const long long zoff = D == 3 ? (long long)(p0[2] + iz) * My * Mx : 0;
#pragma unroll 2
        for (int iy = 0; iy < W; ++iy) {
            const cplx<R> *row = g + zoff + (long long)(p0[1] + iy) * Mx + p0[0];
            R rr = 0, ri = 0;
#pragma unroll
            for (int ix = 0; ix < W; ++ix) {
                const cplx<R> v = row[ix];
                rr += v.x * kw[0][ix];
                ri += v.y * kw[0][ix];
            }
            zr += rr * kw[1][iy];
            zi += ri * kw[1][iy];
        }
        if (D == 3) {
            ar += zr * kw[D - 1][iz];
            ai += zi * kw[D - 1][iz];
        } else {
            ar = zr;
            ai = zi;
        }
    }
}

// Target t's factor after the sum: 1/psi1hat and the normalisation (fac),
// and the centring phase as (cos, sin).
template <int D, bool DEG>
__device__ __forceinline__ void interp_post(const SnapDev &S, int t, const double (&bb)[3], double &fac, double &cs,
                                            double &sn) {
    fac = S.post_norm;
    double dot = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double ph;
        if constexpr (DEG)
            ph = (S.degenerate >> a) & 1 ? phihat_quad(S.xi_deg[a] * (bb[a] - S.b_c[a]), S.qn)
                                         : S.tphi[(long long)a * S.n_tgt + t];
        else
            ph = S.tphi[(long long)a * S.n_tgt + t];
        fac /= ph;
        dot += bb[a] * S.s_c[a];
    }
    sincos_turns(S.post_turn * dot, &sn, &cs);
}

template <typename R, int D, int W, bool DEG>
__global__ __launch_bounds__(256) void k_interp(const SnapDev *snaps, int gx, int n_snap, const cplx<R> *grid,
                                                EsPoly ep) {
    int bx, sy;
    if (!snap_block(gx, n_snap, bx, sy)) return;
    const SnapDev &S = snaps[sy];
    const int t = bx * 256 + threadIdx.x;
    if (t >= S.n_tgt) return;
    R kw[D][W];
    int p0[3] = {0, 0, 0};
    double bb[3] = {0, 0, 0};
    interp_weights<R, D, W>(S, t, ep, kw, p0, bb);
    R ar, ai;
    interp_sum<R, D, W>(S, grid + (D == 2 ? S.bufA : S.bufB), kw, p0, ar, ai);
    double fac, cs, sn;
    interp_post<D, DEG>(S, t, bb, fac, cs, sn);
    const double vr = (double)ar, vi = (double)ai;
    double re = fac * (vr * cs - vi * sn);
    double im = fac * (vr * sn + vi * cs);
    const int ti = S.tidx[t];
    if (ti < 0) im = -im;
    double2 *o = (double2 *)S.out;
    o[ti & 0x7fffffff] = make_double2(re, im);
}

// Spectral basis (paper appendix A): the K snapshots of the launch are the K
// basis transforms of one plan and one target table (every frequency's
// baselines).  Per target the weights and the factor after the sum are
// formed once; the K grids are read at the same cells and combined with the
// basis values of the target's frequency q (vis = sum_k M[q][k] V_k), so the
// visibilities are written directly, with no per-basis output.
template <typename R, int D, int W, bool DEG>
__global__ __launch_bounds__(256) void k_interp_basis(const SnapDev *snaps, int K, const cplx<R> *grid, EsPoly ep,
                                                      const double *M, long long n_pairs, double2 *vis) {
    const SnapDev &S = snaps[0];
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= S.n_tgt) return;
    R kw[D][W];
    int p0[3] = {0, 0, 0};
    double bb[3] = {0, 0, 0};
    interp_weights<R, D, W>(S, t, ep, kw, p0, bb);
    const int ti = S.tidx[t];
    const long long o = ti & 0x7fffffff;
    const double *Mq = M + (o / n_pairs) * K;
    double re = 0.0, im = 0.0;
#pragma unroll 1
    for (int k = 0; k < K; ++k) {
        R ar, ai;
        interp_sum<R, D, W>(S, grid + (D == 2 ? snaps[k].bufA : snaps[k].bufB), kw, p0, ar, ai);
        re += Mq[k] * (double)ar;
        im += Mq[k] * (double)ai;
    }
    double fac, cs, sn;
    interp_post<D, DEG>(S, t, bb, fac, cs, sn);
    double vr = fac * (re * cs - im * sn);
    double vi = fac * (re * sn + im * cs);
    if (ti < 0) vi = -vi;
    vis[o] = make_double2(vr, vi);
}

// Target table of one array geometry.
// Target t of the table is pair perm[t] (a spatial order of the folded
// baselines, so that neighbouring lanes of the interpolation share grid cells),
// or pair t when perm is null.
__global__ __launch_bounds__(256) void k_targets(const double *ant, int n_ant, long long n_pairs, int dim,
                                                 int fold_axis, double3 b_c, double3 B, double xi0,
                                                 const double *qn, const int *perm, double *tb, int *tidx,
                                                 double *tphi) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_pairs) return;
    const long long p = perm ? (long long)perm[t] : t;
    int i, j;
    pair_decode(p, n_ant, &i, &j);
    double b[3], f[3];
    for (int a = 0; a < 3; ++a) b[a] = ant[3 * (size_t)i + a] - ant[3 * (size_t)j + a];
    bool flip = false;
    if (fold_axis >= 0) {
        int order[3] = {fold_axis, 0, 0};
        int k = 1;
        for (int a = 0; a < dim; ++a)
            if (a != fold_axis) order[k++] = a;
        for (int q = 0; q < dim; ++q) {
            const double v = b[order[q]];
            if (v < 0) { flip = true; break; }
            if (v > 0) break;
        }
    }
    const double bc[3] = {b_c.x, b_c.y, b_c.z}, Bh[3] = {B.x, B.y, B.z};
    for (int a = 0; a < dim; ++a) {
        f[a] = flip ? -b[a] : b[a];
        tb[(long long)a * n_pairs + t] = f[a];
        const double xi = Bh[a] > 0 ? xi0 * (f[a] - bc[a]) / Bh[a] : 0.0;
        tphi[(long long)a * n_pairs + t] = phihat_quad(xi, qn);
    }
    tidx[t] = (int)p | (flip ? (int)0x80000000 : 0);
}

template <typename R>
__global__ void k_twiddle(int n, cplx<R> *tw) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    double s, c;
    sincospi(2.0 * (double)t / (double)n, &s, &c);
    tw[t] = cmake<R>((R)c, (R)s);
}

}  // namespace

namespace detail {
// ---------------------------------------------------------------------------
// Host side.
template <typename R, int D, int W>
inline size_t spread_lds() {
    return (size_t)SpreadCfg<R, D, W>::WPB * SpreadCfg<R, D, W>::WAVE_BYTES;
}

// Device buffers of one pipeline run.
struct Bufs {
    const SnapDev *snaps = nullptr;  // device copy of Layout::snaps
    int *bins = nullptr, *rank = nullptr;
    void *recs = nullptr, *ipsi = nullptr, *grid = nullptr;
    int *perm = nullptr, *order_counts = nullptr;  // null unless Layout::orders is non-empty
    double *src_ord = nullptr;                     // source directions in the order perm
    OrderGroup *orders = nullptr;                  // device copy of Layout::orders
    void *recs_tmp = nullptr;                      // deterministic mode: records in scatter order
    int *srcid = nullptr;                          // deterministic mode: source index per scatter position
    // spectral basis: the snapshots are the basis transforms of one plan, and
    // the interpolation writes vis = sum_k M[q][k] V_k directly
    const double *basis_M = nullptr;  // [n_freq][K]
    double *basis_vis = nullptr;      // [n_freq][n_pairs] complex
    long long basis_np = 0;
    // ipsi already holds this plan's tables: the last launch on this
    // workspace had the same plan and buffers and computed them
    bool ipsi_ready = false;
};

// Snapshot-per-XCD launches when the snapshots fill the 8 XCDs evenly enough
// (FV_XCD_AFFINE=0 turns them off, =1 forces them on).
inline bool xcd_affine(int n_snap) {
    static const int mode = env_int("FV_XCD_AFFINE", -1);
    if (mode >= 0) return mode == 1;
    return n_snap % 8 == 0 || n_snap >= 32;
}

// One stage that is one kernel: with timing on, the dispatch itself records
// the stage's start and stop events (no separate marker packets); otherwise a
// plain launch (as under graph capture).
template <typename... KA, typename... A>
void launch_stage(StageTimer *tm, int stage, void (*kernel)(KA...), dim3 grid, dim3 block, size_t lds, hipStream_t st,
                  A... args) {
    hipEvent_t ea = nullptr, eb = nullptr;
    tm->kernel_events(stage, &ea, &eb);
    if (ea)
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, st, ea, eb, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
}

// stages: bit 0 sort + spread, bit 1 FFT passes, bit 2 interpolation.
template <typename R, int D, int W>
void run_pipeline(const Layout &L, const Bufs &B, int n_snap, hipStream_t st, int stages, StageTimer *tm) {
    StageTimer dummy;
    if (!tm) tm = &dummy;
    const SnapDev *snaps_dev = B.snaps;
    int *bins = B.bins, *rank = B.rank;
    auto recs = (Rec<R, D> *)B.recs;
    R *ipsi = (R *)B.ipsi;
    cplx<R> *grid = (cplx<R> *)B.grid;
    const int *perm = L.orders.empty() ? nullptr : B.perm;
    // per-snapshot launches: XCD-affine 1-D grids when the snapshots spread
    // evenly over the 8 XCDs, else plain (x, snapshot) grids
    const bool affine = xcd_affine(n_snap);
    auto sgrid = [&](long long gx) {
        return affine ? dim3((unsigned)(8 * gx * ((n_snap + 7) / 8))) : dim3((unsigned)gx, (unsigned)n_snap);
    };
    auto sgx = [&](long long gx) { return affine ? (int)gx : 0; };
    auto blocks = [](long long n, int b) { return (unsigned)((n + b - 1) / b); };
    if (stages & 1) {
    if (L.total_bins)
        hipLaunchKernelGGL(k_fill_int, dim3(blocks(L.total_bins, 256)), dim3(256), 0, st, bins, L.total_bins, 0);
    if (L.max_ipsi && !B.ipsi_ready) {
        launch_stage(tm, FV_STAGE_OTHER, k_ipsi<R>, dim3(blocks(L.max_ipsi, 256), n_snap), dim3(256), 0, st,
                     snaps_dev, ipsi);
        tm->add(FV_STAGE_OTHER, L.sbytes[FV_STAGE_OTHER], 1);
    }
    tm->begin(FV_STAGE_SORT, st);
    int sort_launches = 3;
    if (perm) {
        // the shared spatial orders (rank is scratch here; k_bin rewrites it)
        const unsigned ng = (unsigned)L.orders.size();
        hipLaunchKernelGGL(k_fill_int, dim3(blocks(L.order_counts, 256)), dim3(256), 0, st, B.order_counts,
                           L.order_counts, 0);
        hipLaunchKernelGGL(k_order_count<D>, dim3(blocks(L.max_order_src, 256), ng), dim3(256), 0, st, snaps_dev,
                           (const OrderGroup *)B.orders, B.order_counts, rank);
        hipLaunchKernelGGL(k_order_scan, dim3(ng), dim3(1024), 0, st, (const OrderGroup *)B.orders,
                           B.order_counts);
        hipLaunchKernelGGL(k_order_place<D>, dim3(blocks(L.max_order_src, 256), ng), dim3(256), 0, st, snaps_dev,
                           (const OrderGroup *)B.orders, (const int *)B.order_counts, (const int *)rank, B.perm,
                           B.src_ord);
        sort_launches += 4;
    }
    if (L.max_src) {
        const long long gx = blocks(L.max_src, 256);
        hipLaunchKernelGGL(k_bin<D>, sgrid(gx), dim3(256), 0, st, snaps_dev, sgx(gx), n_snap,
                           (const double *)B.src_ord, bins, rank);
    }
    hipLaunchKernelGGL(k_scan, dim3(n_snap), dim3(1024), 0, st, snaps_dev, bins);
    if (L.max_src) {
        const long long gx = blocks(L.max_src, 256);
        hipLaunchKernelGGL((k_scatter<R, D>), sgrid(gx), dim3(256), 0, st, snaps_dev, sgx(gx), n_snap, perm,
                           (const double *)B.src_ord, (const int *)bins, (const int *)rank,
                           L.det ? (Rec<R, D> *)B.recs_tmp : recs, L.det ? B.srcid : nullptr);
        if (L.det) {
            hipLaunchKernelGGL((k_stable<R, D>), sgrid(gx), dim3(256), 0, st, snaps_dev, sgx(gx), n_snap,
                               (const int *)bins, (const int *)B.srcid, (const Rec<R, D> *)B.recs_tmp, recs);
            ++sort_launches;
        }
    }
    tm->end(st);
    tm->add(FV_STAGE_SORT, L.sbytes[FV_STAGE_SORT], sort_launches);
    {
        if constexpr (D == 2) {
            using MC = SpreadMfmaCfg<R, W>;
            const size_t lds = (size_t)MC::WPB * MC::WAVE_BYTES;
            ensure_lds((const void *)k_spread_mfma<R, W>, lds);
            launch_stage(tm, FV_STAGE_SPREAD, k_spread_mfma<R, W>, sgrid(L.max_tiles), dim3(64 * MC::WPB), lds, st,
                         snaps_dev, sgx(L.max_tiles), n_snap, (const int *)bins, (const Rec<R, 2> *)recs,
                         (const R *)ipsi, grid, es_poly(W));
        } else {
            using Cfg = SpreadCfg<R, D, W>;
            const size_t lds = spread_lds<R, D, W>();
            ensure_lds((const void *)k_spread<R, D, W>, lds);
            launch_stage(tm, FV_STAGE_SPREAD, k_spread<R, D, W>, sgrid(L.max_tiles), dim3(64 * Cfg::WPB), lds, st,
                         snaps_dev, sgx(L.max_tiles), n_snap, (const int *)bins, (const Rec<R, D> *)recs,
                         (const R *)ipsi, grid, es_poly(W));
        }
        tm->add(FV_STAGE_SPREAD, L.sbytes[FV_STAGE_SPREAD], 1);
    }
    }
    if (stages & 2)
    for (int a = 0; a < D; ++a) {
        const int fs = FV_STAGE_FFT_X + a;
        if constexpr (std::is_same<R, float>::value) {
            if (L.reg[a]) {
                hipEvent_t ea = nullptr, eb = nullptr;
                tm->kernel_events(fs, &ea, &eb);
                if (a == 0)
                    launch_fft_reg_rows(snaps_dev, n_snap, a, grid, L.reg_wg[a], L.reg_lds[a], st, ea, eb);
                else
                    launch_fft_reg_cols(snaps_dev, n_snap, a, grid, L.reg_wg[a], L.reg_lds[a], st, ea, eb);
                tm->add(fs, L.sbytes[fs], 1);
                continue;
            }
        }
        // a multiple of 8 workgroups along x, so that the XCD of (x, y) is x mod 8
        const dim3 nb((unsigned)((L.max_wg[a] + 7) / 8 * 8), (unsigned)n_snap);
        switch (L.tpb[a]) {
            case 128:
                ensure_lds((const void *)k_fft<R, 128>, L.fft_lds[a]);
                launch_stage(tm, fs, k_fft<R, 128>, nb, dim3(128), L.fft_lds[a], st, snaps_dev, a, grid);
                break;
            case 256:
                ensure_lds((const void *)k_fft<R, 256>, L.fft_lds[a]);
                launch_stage(tm, fs, k_fft<R, 256>, nb, dim3(256), L.fft_lds[a], st, snaps_dev, a, grid);
                break;
            case 512:
                ensure_lds((const void *)k_fft<R, 512>, L.fft_lds[a]);
                launch_stage(tm, fs, k_fft<R, 512>, nb, dim3(512), L.fft_lds[a], st, snaps_dev, a, grid);
                break;
            default:
                ensure_lds((const void *)k_fft<R, 1024>, L.fft_lds[a]);
                launch_stage(tm, fs, k_fft<R, 1024>, nb, dim3(1024), L.fft_lds[a], st, snaps_dev, a, grid);
                break;
        }
        tm->add(FV_STAGE_FFT_X + a, L.sbytes[FV_STAGE_FFT_X + a], 1);
    }
    if ((stages & 4) && L.max_tgt && B.basis_vis) {
        const dim3 g(blocks(L.snaps[0].n_tgt, 256));
        if (L.any_degenerate)
            launch_stage(tm, FV_STAGE_INTERP, k_interp_basis<R, D, W, true>, g, dim3(256), 0, st, snaps_dev, n_snap,
                         (const cplx<R> *)grid, es_poly(W), B.basis_M, B.basis_np, (double2 *)B.basis_vis);
        else
            launch_stage(tm, FV_STAGE_INTERP, k_interp_basis<R, D, W, false>, g, dim3(256), 0, st, snaps_dev, n_snap,
                         (const cplx<R> *)grid, es_poly(W), B.basis_M, B.basis_np, (double2 *)B.basis_vis);
        tm->add(FV_STAGE_INTERP, L.sbytes[FV_STAGE_INTERP], 1);
    } else if ((stages & 4) && L.max_tgt) {
        const long long gx = blocks(L.max_tgt, 256);
        if (L.any_degenerate)
            launch_stage(tm, FV_STAGE_INTERP, k_interp<R, D, W, true>, sgrid(gx), dim3(256), 0, st, snaps_dev,
                         sgx(gx), n_snap, (const cplx<R> *)grid, es_poly(W));
        else
            launch_stage(tm, FV_STAGE_INTERP, k_interp<R, D, W, false>, sgrid(gx), dim3(256), 0, st, snaps_dev,
                         sgx(gx), n_snap, (const cplx<R> *)grid, es_poly(W));
        tm->add(FV_STAGE_INTERP, L.sbytes[FV_STAGE_INTERP], 1);
    }
    FV_HIP(hipGetLastError());
}

using PipeFn = void (*)(const Layout &, const Bufs &, int, hipStream_t, int, StageTimer *);

template <typename R, int D, int W>
void pipe_entry(const Layout &L, const Bufs &B, int n, hipStream_t st, int stages, StageTimer *tm) {
    run_pipeline<R, D, W>(L, B, n, st, stages, tm);
}

template <typename R, int D, int... Ws>
PipeFn pick_w(int w, std::integer_sequence<int, Ws...>) {
    PipeFn f = nullptr;
    ((w == Ws ? (f = &pipe_entry<R, D, Ws>, 0) : 0), ...);
    return f;
}

using WList = std::integer_sequence<int, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16>;

PipeFn pick_f32_2d(int w);
PipeFn pick_f32_3d(int w);
PipeFn pick_f64_2d(int w);
PipeFn pick_f64_3d(int w);

}  // namespace detail
}  // namespace fv
