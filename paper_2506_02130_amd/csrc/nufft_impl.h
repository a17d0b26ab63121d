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
#include <hip/hip_runtime.h>
#include <utility>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <stdexcept>
#include <vector>

#include "ctx.h"
#include "dev_common.h"
#include "fv_internal.h"

namespace fv {
namespace {

template <typename R, int D>
struct Rec {
    int l0[D];
    R off[D];
    R cr, ci;
};

template <int D>
struct TileShape;
template <>
struct TileShape<2> {
    static constexpr int X = 32, Y = 32, Z = 1;
};
template <>
struct TileShape<3> {
    static constexpr int X = 16, Y = 16, Z = 8;
};

__host__ __device__ inline int sub_bin_edge(int a) { return a < 2 ? kSubBin : kSubBinZ; }

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

template <int D>
__global__ __launch_bounds__(256) void k_bin(const SnapDev *snaps, int *bins, int *rank) {
    const SnapDev &S = snaps[blockIdx.y];
    int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= S.n_src) return;
    double s[3], g[3];
    int l0[3];
    for (int a = 0; a < D; ++a) s[a] = S.src[3 * (size_t)j + a];
    int key = src_cell<D>(S, s, g, l0);
    rank[S.src_base + j] = atomicAdd(&bins[S.bin_base + key], 1);
}

// Exclusive scan of each snapshot's sub-bin counts, one 1024-thread block per
// snapshot, 4 counts per thread per chunk.
__global__ __launch_bounds__(1024) void k_scan(const SnapDev *snaps, int *bins) {
    const SnapDev &S = snaps[blockIdx.x];
    long long nb = 1;
    for (int a = 0; a < S.dim; ++a) nb *= S.nsb[a];
    int *b = bins + S.bin_base;
    __shared__ int wsum[16];
    __shared__ int carry_sh;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) carry_sh = 0;
    __syncthreads();
    for (long long base = 0; base < nb; base += 4096) {
        int v[4];
        int tsum = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            long long i = base + 4 * tid + q;
            v[q] = i < nb ? b[i] : 0;
            tsum += v[q];
        }
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
        for (int q = 0; q < 4; ++q) {
            long long i = base + 4 * tid + q;
            if (i < nb) b[i] = run;
            run += v[q];
        }
        __syncthreads();
        if (tid == 0) carry_sh += total;
        __syncthreads();
    }
    if (tid == 0) b[nb] = carry_sh;
}

template <typename R, int D>
__global__ __launch_bounds__(256) void k_scatter(const SnapDev *snaps, const int *bins, const int *rank,
                                                 Rec<R, D> *recs) {
    const SnapDev &S = snaps[blockIdx.y];
    int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= S.n_src) return;
    double s[3], g[3];
    int l0[3];
    for (int a = 0; a < D; ++a) s[a] = S.src[3 * (size_t)j + a];
    int key = src_cell<D>(S, s, g, l0);
    long long pos = (long long)bins[S.bin_base + key] + rank[S.src_base + j];
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
    static constexpr int TX = TileShape<D>::X, TY = TileShape<D>::Y, TZ = TileShape<D>::Z;
    static constexpr int CELLS = TX * TY * TZ;
    static constexpr int WAVE_BYTES = CELLS * (int)sizeof(cplx<R>) + 64 * D * W * (int)sizeof(R);
    static constexpr int WPB0 = 98304 / WAVE_BYTES;
    static constexpr int WPB = WPB0 >= 4 ? 4 : (WPB0 >= 2 ? 2 : 1);
    static constexpr int WD = D == 2 ? W * W : W * W * W;
};

template <typename R, int D, int W>
__global__ __launch_bounds__(256) void k_spread(const SnapDev *snaps, int n_snap, long long total_tiles,
                                                const int *bins, const Rec<R, D> *recs, const R *ipsi,
                                                cplx<R> *grid) {
    using Cfg = SpreadCfg<R, D, W>;
    extern __shared__ __align__(16) char smem[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long tile = (long long)blockIdx.x * Cfg::WPB + wave;
    if (tile >= total_tiles) return;
    const int s = find_snap(snaps, n_snap, tile, 0);
    const SnapDev &S = snaps[s];
    long long t = tile - S.tile_base;
    int org[3];
    org[0] = (int)(t % S.ntile[0]) * Cfg::TX;
    t /= S.ntile[0];
    org[1] = (int)(t % S.ntile[1]) * Cfg::TY;
    org[2] = D == 3 ? (int)(t / S.ntile[1]) * Cfg::TZ : 0;
    const int text[3] = {Cfg::TX, Cfg::TY, Cfg::TZ};

    cplx<R> *acc = (cplx<R> *)(smem + wave * Cfg::WAVE_BYTES);
    R *kw = (R *)(acc + Cfg::CELLS);  // [64][D][W]
    for (int c = lane; c < Cfg::CELLS; c += 64) acc[c] = cmake<R>(0, 0);

    const R beta = (R)S.beta;
    const R inv_hw = (R)(2.0 / W);
    int sblo[3] = {0, 0, 0}, sbhi[3] = {0, 0, 0};
    bool empty = false;
    for (int a = 0; a < D; ++a) {
        int lo = max(0, org[a] - W + 1);
        int hi = min(S.n1[a] - W, org[a] + text[a] - 1);
        if (lo > hi) empty = true;
        sblo[a] = lo / sub_bin_edge(a);
        sbhi[a] = hi / sub_bin_edge(a);
    }
    const Rec<R, D> *rs = recs + S.src_base;
    const int *bb = bins + S.bin_base;
    if (!empty) {
        for (int sz = sblo[2]; sz <= (D == 3 ? sbhi[2] : 0); ++sz) {
            for (int sy = sblo[1]; sy <= sbhi[1]; ++sy) {
                const long long row = ((long long)sz * S.nsb[1] + sy) * S.nsb[0];
                const int start = bb[row + sblo[0]];
                const int end = bb[row + sbhi[0] + 1];
                for (int b0 = start; b0 < end; b0 += 64) {
                    const int nrec = min(64, end - b0);
                    int ml0[D];
                    R mcr = 0, mci = 0;
                    bool hit = false;
                    if (lane < nrec) {
                        const Rec<R, D> r = rs[b0 + lane];
                        hit = true;
#pragma unroll
                        for (int a = 0; a < D; ++a) {
                            ml0[a] = r.l0[a];
                            hit = hit && (r.l0[a] + W - 1 >= org[a]) && (r.l0[a] <= org[a] + text[a] - 1);
#pragma unroll
                            for (int i = 0; i < W; ++i)
                                kw[(lane * D + a) * W + i] = es_phi((R)((R)i - r.off[a]) * inv_hw, beta);
                        }
                        mcr = r.cr;
                        mci = r.ci;
                    } else {
#pragma unroll
                        for (int a = 0; a < D; ++a) ml0[a] = 0;
                    }
                    wave_sync();
                    unsigned long long hm = __ballot(hit);
                    while (hm) {
                        const int r = __ffsll((long long)hm) - 1;
                        hm &= hm - 1;
                        int l0[D];
#pragma unroll
                        for (int a = 0; a < D; ++a) l0[a] = readlane_i(ml0[a], r) - org[a];
                        const R cr = readlane_r<R>(mcr, r), ci = readlane_r<R>(mci, r);
                        const R *kr = kw + r * D * W;
#pragma unroll 4
                        for (int q = 0; q < Cfg::WD; q += 64) {
                            const int cidx = q + lane;
                            if (cidx < Cfg::WD) {
                                const int ix = cidx % W;
                                const int iy = (cidx / W) % W;
                                const int iz = D == 3 ? cidx / (W * W) : 0;
                                const int gx = l0[0] + ix, gy = l0[1] + iy, gz = D == 3 ? l0[D - 1] + iz : 0;
                                if (gx >= 0 && gx < Cfg::TX && gy >= 0 && gy < Cfg::TY && gz >= 0 && gz < Cfg::TZ) {
                                    R wt = kr[ix] * kr[W + iy];
                                    if (D == 3) wt *= kr[2 * W + iz];
                                    cplx<R> &cell = acc[(gz * Cfg::TY + gy) * Cfg::TX + gx];
                                    cell.x += wt * cr;
                                    cell.y += wt * ci;
                                }
                            }
                        }
                        __builtin_amdgcn_wave_barrier();
                    }
                    wave_sync();
                }
            }
        }
    }
    wave_sync();
    // flush: divide by psi2hat at the modes and store each owned cell once
    const R *ix_t = ipsi + S.ipsi_base;
    const R *iy_t = ix_t + S.n1[0];
    const R *iz_t = iy_t + S.n1[1];
    cplx<R> *dst = grid + S.bufA;
    for (int c = lane; c < Cfg::CELLS; c += 64) {
        const int lx = c % Cfg::TX, ly = (c / Cfg::TX) % Cfg::TY, lz = c / (Cfg::TX * Cfg::TY);
        const int gx = org[0] + lx, gy = org[1] + ly, gz = org[2] + lz;
        if (gx < S.n1[0] && gy < S.n1[1] && (D == 2 || gz < S.n1[2])) {
            R f = ix_t[gx] * iy_t[gy];
            if (D == 3) f *= iz_t[gz];
            dst[((long long)gz * S.n1[1] + gy) * S.n1[0] + gx] = cscale<R>(acc[c], f);
        }
    }
}

// ---------------------------------------------------------------------------
// FFT: mixed-radix Stockham (autosort) in LDS, + sign.  Butterfly b of a
// radix-r stage with p = product of earlier radices reads x[i + j N/r],
// multiplies input j by W_N^(j k N/(p r)) (k = i mod p), takes the r-point
// DFT and writes outputs q at (i - k) r + k + q p.
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
        cplx<R> a = cadd<R>(v[0], v[2]), b = csub<R>(v[0], v[2]);
        cplx<R> c = cadd<R>(v[1], v[3]), d = cmuli<R>(csub<R>(v[1], v[3]));
        v[0] = cadd<R>(a, c);
        v[2] = csub<R>(a, c);
        v[1] = cadd<R>(b, d);
        v[3] = csub<R>(b, d);
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
    }
}

template <typename R, int TPB, int RAD>
__device__ __forceinline__ void fft_stage(cplx<R> *buf, int N, int cx, int p, const cplx<R> *tw) {
    // every thread holds at most ceil(kFftSlots / RAD) butterflies; the host
    // keeps lines * N <= kFftSlots * TPB so all cx * N / RAD butterflies are covered
    constexpr int ROUNDS = (kFftSlots + RAD - 1) / RAD;
    const int T = N / RAD;
    const int nb = cx * T;
    const int tws = N / (p * RAD);
    cplx<R> v[ROUNDS][RAD];
#pragma unroll
    for (int rr = 0; rr < ROUNDS; ++rr) {
        const int b = threadIdx.x + rr * TPB;
        if (b < nb) {
            const int c = b / T, i = b - c * T;
            const cplx<R> *src = buf + (long long)c * N + i;
#pragma unroll
            for (int j = 0; j < RAD; ++j) v[rr][j] = src[j * T];
        }
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < ROUNDS; ++rr) {
        const int b = threadIdx.x + rr * TPB;
        if (b < nb) {
            const int c = b / T, i = b - c * T;
            const int k = i % p;
            if (k) {
#pragma unroll
                for (int j = 1; j < RAD; ++j) v[rr][j] = cmul<R>(v[rr][j], tw[j * k * tws]);
            }
            dft_small<R, RAD>(v[rr]);
            cplx<R> *dst = buf + (long long)c * N + (i - k) * RAD + k;
#pragma unroll
            for (int q = 0; q < RAD; ++q) dst[q * p] = v[rr][q];
        }
    }
    __syncthreads();
}

template <typename R, int TPB>
__device__ void fft_lds(cplx<R> *buf, int N, int cx, const cplx<R> *tw) {
    int p = 1, rem = N;
    while (rem % 4 == 0) { fft_stage<R, TPB, 4>(buf, N, cx, p, tw); p *= 4; rem /= 4; }
    while (rem % 2 == 0) { fft_stage<R, TPB, 2>(buf, N, cx, p, tw); p *= 2; rem /= 2; }
    while (rem % 3 == 0) { fft_stage<R, TPB, 3>(buf, N, cx, p, tw); p *= 3; rem /= 3; }
    while (rem % 5 == 0) { fft_stage<R, TPB, 5>(buf, N, cx, p, tw); p *= 5; rem /= 5; }
}

// One pass along axis `a` for every snapshot: lines of n1[a] inputs (already
// deconvolved), placed at (m mod n2), FFT of length n2, outputs p in [-P, P].
// Input layout [slow: n1 of axes > a][n1_a][fast: M of axes < a]; output
// [slow][M_a][fast].  Passes alternate bufA -> bufB -> bufA (-> bufB).
template <typename R, int TPB>
__global__ __launch_bounds__(TPB) void k_fft(const SnapDev *snaps, int n_snap, int a, cplx<R> *grid) {
    extern __shared__ __align__(16) char smem[];
    cplx<R> *buf = (cplx<R> *)smem;
    const int s = find_snap(snaps, n_snap, blockIdx.x, a + 1);
    const SnapDev &S = snaps[s];
    const int N = S.n2[a], n1a = S.n1[a], Ma = S.M[a], Pa = S.P[a], CX = S.cx[a];
    long long F = 1;
    for (int b = 0; b < a; ++b) F *= S.M[b];
    const long long ngrp = (F + CX - 1) / CX;
    const long long wl = (long long)blockIdx.x - S.wg_base[a];
    const long long o = wl / ngrp;
    const long long i0 = (wl - o * ngrp) * CX;
    const int cx = (int)min((long long)CX, F - i0);
    const bool fromA = (a % 2) == 0;
    const cplx<R> *in = grid + (fromA ? S.bufA : S.bufB) + o * ((long long)n1a * F) + i0;
    cplx<R> *out = grid + (fromA ? S.bufB : S.bufA) + o * ((long long)Ma * F) + i0;
    const cplx<R> *tw = (const cplx<R> *)S.tw[a];
    const int half = n1a / 2;
    for (int e = threadIdx.x; e < cx * N; e += TPB) {
        const int c = e / N, l2 = e - c * N;
        if (l2 >= half && l2 < N - half) buf[(long long)c * N + l2] = cmake<R>(0, 0);
    }
    for (int e = threadIdx.x; e < cx * n1a; e += TPB) {
        const int c = e % cx, l = e / cx;
        int idx = l - half;
        if (idx < 0) idx += N;
        buf[(long long)c * N + idx] = in[(long long)l * F + c];
    }
    __syncthreads();
    fft_lds<R, TPB>(buf, N, cx, tw);
    for (int e = threadIdx.x; e < cx * Ma; e += TPB) {
        const int c = e % cx, po = e / cx;
        int idx = (po - Pa) % N;
        if (idx < 0) idx += N;
        out[(long long)po * F + c] = buf[(long long)c * N + idx];
    }
}

// Interpolation at the targets, deconvolution by psi1hat, centring phase,
// reflection undone, written to the caller's pair layout.
template <typename R, int D, int W>
__global__ __launch_bounds__(256) void k_interp(const SnapDev *snaps, const cplx<R> *grid) {
    const SnapDev &S = snaps[blockIdx.y];
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= S.n_tgt) return;
    const cplx<R> *g = grid + (D == 2 ? S.bufA : S.bufB);
    const R beta = (R)S.beta;
    const R inv_hw = (R)(2.0 / W);
    double bb[3] = {0, 0, 0};
    int p0[3] = {0, 0, 0};
    R kw[D][W];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double b = S.tb[(long long)a * S.n_tgt + t];
        bb[a] = b;
        const double q = S.qscale[a] * (b - S.b_c[a]);
        int p = (int)ceil(q - 0.5 * W);
        p = min(max(p, -S.P[a]), S.P[a] - W + 1);
        const R off = (R)(q - p);
#pragma unroll
        for (int i = 0; i < W; ++i) kw[a][i] = es_phi((R)((R)i - off) * inv_hw, beta);
        p0[a] = p + S.P[a];
    }
    R ar = 0, ai = 0;
    const long long My = S.M[1], Mx = S.M[0];
#pragma unroll 1
    for (int iz = 0; iz < (D == 3 ? W : 1); ++iz) {
        R zr = 0, zi = 0;
        const long long zoff = D == 3 ? (long long)(p0[2] + iz) * My * Mx : 0;
#pragma unroll
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
    double fac = S.post_norm;
    double dot = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double ph = (S.degenerate >> a) & 1 ? phihat_quad(S.xi_deg[a] * (bb[a] - S.b_c[a]), S.qn)
                                                   : S.tphi[(long long)a * S.n_tgt + t];
        fac /= ph;
        dot += bb[a] * S.s_c[a];
    }
    double sn, cs;
    sincos_turns(S.post_turn * dot, &sn, &cs);
    const double vr = (double)ar, vi = (double)ai;
    double re = fac * (vr * cs - vi * sn);
    double im = fac * (vr * sn + vi * cs);
    const int ti = S.tidx[t];
    if (ti < 0) im = -im;
    double2 *o = (double2 *)S.out;
    o[ti & 0x7fffffff] = make_double2(re, im);
}

// Target table of one array geometry.
__global__ __launch_bounds__(256) void k_targets(const double *ant, int n_ant, long long n_pairs, int dim,
                                                 int fold_axis, double3 b_c, double3 B, double xi0,
                                                 const double *qn, double *tb, int *tidx, double *tphi) {
    const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    if (p >= n_pairs) return;
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
        tb[(long long)a * n_pairs + p] = f[a];
        const double xi = Bh[a] > 0 ? xi0 * (f[a] - bc[a]) / Bh[a] : 0.0;
        tphi[(long long)a * n_pairs + p] = phihat_quad(xi, qn);
    }
    tidx[p] = (int)p | (flip ? (int)0x80000000 : 0);
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

struct Layout {
    std::vector<SnapDev> snaps;
    long long total_tiles = 0, total_src = 0, total_bins = 0, total_ipsi = 0, total_grid = 0;
    long long max_src = 0, max_tgt = 0, max_ipsi = 0;
    long long wg_total[3] = {0, 0, 0};
    int tpb[3] = {256, 256, 256};
    size_t fft_lds[3] = {0, 0, 0};
    double model_bytes = 0;
};

// Upper bound on the lines one FFT workgroup transforms together (tunable
// through FV_FFT_MAX_LINES).
inline int fft_max_lines() {
    static int v = [] {
        const char *e = std::getenv("FV_FFT_MAX_LINES");
        int x = e ? std::atoi(e) : 16;
        return x < 1 ? 1 : (x > 64 ? 64 : x);
    }();
    return v;
}

inline int fft_tpb_for(int N) {
    if (N <= kFftSlots * 256) return 256;
    if (N <= kFftSlots * 512) return 512;
    return 1024;
}

inline Layout make_layout(const std::vector<SnapJob> &jobs, int dim, int prec_bits, int w) {
    Layout L;
    const size_t csz = prec_bits == 32 ? 8 : 16;
    const int T[3] = {dim == 2 ? TileShape<2>::X : TileShape<3>::X, dim == 2 ? TileShape<2>::Y : TileShape<3>::Y,
                      dim == 2 ? 1 : TileShape<3>::Z};
    // FFT threads per pass from the largest line length
    for (int a = 0; a < dim; ++a) {
        int nmax = 0;
        for (auto &j : jobs) nmax = std::max(nmax, j.plan.n2[a]);
        L.tpb[a] = fft_tpb_for(nmax);
        if ((long long)nmax > (long long)kFftSlots * 1024 || (size_t)nmax * csz > 160u * 1024)
            fail(FV_EUNSUPPORTED, "FFT line of " + std::to_string(nmax) + " points exceeds the LDS transform");
    }
    for (auto &j : jobs) {
        const SnapPlan &p = j.plan;
        SnapDev d;
        std::memset(&d, 0, sizeof(d));
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
        d.src_base = L.total_src;
        L.total_src += j.n_src;
        d.bin_base = L.total_bins;
        L.total_bins += nb + 1;
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
            int cx = 1;
            if (F > 1) {
                const long long byreg = (long long)kFftSlots * L.tpb[a] / p.n2[a];
                const long long bylds = 65536LL / ((long long)p.n2[a] * csz);
                cx = (int)std::max(1LL, std::min({F, byreg, bylds, (long long)fft_max_lines()}));
            }
            d.cx[a] = cx;
            d.wg_base[a] = L.wg_total[a];
            L.wg_total[a] += Sl * ((F + cx - 1) / cx);
            L.fft_lds[a] = std::max(L.fft_lds[a], (size_t)cx * p.n2[a] * csz);
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
        L.snaps.push_back(d);
    }
    return L;
}

inline size_t rec_bytes(int dim, int prec_bits) {
    if (prec_bits == 32) return dim == 2 ? sizeof(Rec<float, 2>) : sizeof(Rec<float, 3>);
    return dim == 2 ? sizeof(Rec<double, 2>) : sizeof(Rec<double, 3>);
}

inline size_t layout_bytes(const Layout &L, int dim, int prec_bits, int n_snap) {
    const size_t csz = prec_bits == 32 ? 8 : 16, rsz = prec_bits == 32 ? 4 : 8;
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    return al(n_snap * sizeof(SnapDev)) + al(L.total_bins * 4) + al(L.total_src * 4) +
           al(L.total_src * rec_bytes(dim, prec_bits)) + al(L.total_ipsi * rsz) + al(L.total_grid * csz) + 4096;
}

// Kernels asking for more than 64 KB of dynamic LDS must say so first.
inline void ensure_lds(const void *fn, size_t bytes) {
    if (bytes > 65536) FV_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

// stages: bit 0 sort + spread, bit 1 FFT passes, bit 2 interpolation.
template <typename R, int D, int W>
void run_pipeline(const Layout &L, const SnapDev *snaps_dev, int n_snap, int *bins, int *rank, void *recs_v,
                  R *ipsi, cplx<R> *grid, hipStream_t st, int stages) {
    auto recs = (Rec<R, D> *)recs_v;
    auto blocks = [](long long n, int b) { return (unsigned)((n + b - 1) / b); };
    if (stages & 1) {
    if (L.total_bins)
        hipLaunchKernelGGL(k_fill_int, dim3(blocks(L.total_bins, 256)), dim3(256), 0, st, bins, L.total_bins, 0);
    if (L.max_ipsi)
        hipLaunchKernelGGL(k_ipsi<R>, dim3(blocks(L.max_ipsi, 256), n_snap), dim3(256), 0, st, snaps_dev, ipsi);
    if (L.max_src) {
        hipLaunchKernelGGL(k_bin<D>, dim3(blocks(L.max_src, 256), n_snap), dim3(256), 0, st, snaps_dev, bins, rank);
    }
    hipLaunchKernelGGL(k_scan, dim3(n_snap), dim3(1024), 0, st, snaps_dev, bins);
    if (L.max_src) {
        hipLaunchKernelGGL((k_scatter<R, D>), dim3(blocks(L.max_src, 256), n_snap), dim3(256), 0, st, snaps_dev,
                           (const int *)bins, (const int *)rank, recs);
    }
    {
        using Cfg = SpreadCfg<R, D, W>;
        const size_t lds = spread_lds<R, D, W>();
        ensure_lds((const void *)k_spread<R, D, W>, lds);
        hipLaunchKernelGGL((k_spread<R, D, W>), dim3(blocks(L.total_tiles, Cfg::WPB)), dim3(64 * Cfg::WPB), lds, st,
                           snaps_dev, n_snap, L.total_tiles, (const int *)bins, (const Rec<R, D> *)recs,
                           (const R *)ipsi, grid);
    }
    }
    if (stages & 2)
    for (int a = 0; a < D; ++a) {
        const unsigned nb = (unsigned)L.wg_total[a];
        switch (L.tpb[a]) {
            case 256:
                ensure_lds((const void *)k_fft<R, 256>, L.fft_lds[a]);
                hipLaunchKernelGGL((k_fft<R, 256>), dim3(nb), dim3(256), L.fft_lds[a], st, snaps_dev, n_snap, a, grid);
                break;
            case 512:
                ensure_lds((const void *)k_fft<R, 512>, L.fft_lds[a]);
                hipLaunchKernelGGL((k_fft<R, 512>), dim3(nb), dim3(512), L.fft_lds[a], st, snaps_dev, n_snap, a, grid);
                break;
            default:
                ensure_lds((const void *)k_fft<R, 1024>, L.fft_lds[a]);
                hipLaunchKernelGGL((k_fft<R, 1024>), dim3(nb), dim3(1024), L.fft_lds[a], st, snaps_dev, n_snap, a,
                                   grid);
                break;
        }
    }
    if ((stages & 4) && L.max_tgt)
        hipLaunchKernelGGL((k_interp<R, D, W>), dim3(blocks(L.max_tgt, 256), n_snap), dim3(256), 0, st, snaps_dev,
                           (const cplx<R> *)grid);
    FV_HIP(hipGetLastError());
}

using PipeFn = void (*)(const Layout &, const SnapDev *, int, int *, int *, void *, void *, void *, hipStream_t,
                        int);

template <typename R, int D, int W>
void pipe_entry(const Layout &L, const SnapDev *sd, int n, int *bins, int *rank, void *recs, void *ipsi, void *grid,
                hipStream_t st, int stages) {
    run_pipeline<R, D, W>(L, sd, n, bins, rank, recs, (R *)ipsi, (cplx<R> *)grid, st, stages);
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
