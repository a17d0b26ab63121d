// Direct sum in antenna-factor form on the matrix cores (paper section 5.1,
// the review of the matrix-based simulator: the phase of baseline (i, j)
// splits into per-antenna phasors F_in conj(F_jn), so the visibilities of all
// pairs are the entries of one matrix product).  Per frequency
//
//     V = Z diag(c) Z^H,   Z[i][n] = exp(-2 pi i (nu / c) x_i . s_n),
//
// with c_n = beam * flux real and of any sign, so diag(c) stays between the
// two factors instead of being split into square roots.
//
//   k_zbuild  Z for a chunk of sources, stored source-major [n][ia] (antenna
//             fastest, antennas padded to a multiple of 32 with zeros), phase
//             formed in FP64 turns and reduced exactly before sin/cos; FP32 or
//             FP64 complex.  One 16x4 matrix-core operand is then four runs of
//             16 contiguous complex values.
//   k_zz      one wavefront per (32 x 32 antenna tile pair I <= J, source
//             split s), four splits of one tile pair per block.  The wave holds
//             2 x 2 tiles of 16 x 16 and accumulates, with A = c Z(I), B = Z(J),
//                 Re V += Ar Br^T + Ai Bi^T,   Im V += Ai Br^T - Ar Bi^T
//             on 16x16x4 MFMA steps.  In FP32 the tile accumulators are added
//             into FP64 registers every kFoldSrc sources, which bounds the
//             length of every FP32 sum; the FP64 partial tile is stored per
//             split.
//   k_zz_out  per pair i <= j: the partials of its tile pair summed over the
//             splits in FP64, in split order (deterministic), written to the
//             caller's layout, or added to it for the second and later source
//             chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "dev_common.h"
#include "fv_internal.h"

namespace fv {
namespace {


template <typename R>
__global__ __launch_bounds__(256) void k_zbuild(const double *ant, int n_ant, int na_pad, const double *src, int k0,
                                                int kc, int kc_pad, const double *flux, const double *beam,
                                                double kturn, int dim, cplx<R> *Z, R *cz) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)kc_pad * na_pad) return;
    const int k = (int)(t / na_pad), ia = (int)(t - (long long)k * na_pad);
    cplx<R> z = cmake<R>((R)0, (R)0);
    if (k < kc && ia < n_ant) {
        const double *s = src + 3 * (size_t)(k0 + k);
        const double *x = ant + 3 * (size_t)ia;
        double d = x[0] * s[0] + x[1] * s[1];
        if (dim == 3) d += x[2] * s[2];
        R sn, cs;
        sincos_turns(-kturn * d, &sn, &cs);
        z = cmake<R>(cs, sn);
    }
    Z[t] = z;
    if (ia == 0) {
        R c = (R)0;
        if (k < kc) c = (R)(beam ? flux[k0 + k] * beam[k0 + k] : flux[k0 + k]);
        cz[k] = c;
    }
}

template <typename R>
__device__ __forceinline__ void fold(typename MfmaAcc<R>::T &acc, double *d) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        d[r] += (double)acc[r];
        acc[r] = (R)0;
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_zz(const cplx<R> *Z, const R *cz, int na_pad, int kc_pad, int ntile,
                                            int nsplit, double2 *part) {
    using MA = MfmaAcc<R>;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int s = blockIdx.y * kWavesPerBlock + wave;
    if (s >= nsplit) return;
    int tp = blockIdx.x, I = 0;
    while (tp >= ntile - I) {
        tp -= ntile - I;
        ++I;
    }
    const int J = I + tp;
    const int ntp = ntile * (ntile + 1) / 2;
    const int kq = kc_pad / 4;
    const int q0 = (int)((long long)kq * s / nsplit), q1 = (int)((long long)kq * (s + 1) / nsplit);
    const int r = lane >> 4, c16 = lane & 15;
    const cplx<R> *za = Z + I * kZTile + c16;
    const cplx<R> *zb = Z + J * kZTile + c16;
    typename MA::T vr[2][2], vi[2][2];
    double dr[2][2][4], di[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                vr[a][b][e] = (R)0;
                vi[a][b][e] = (R)0;
                dr[a][b][e] = 0.0;
                di[a][b][e] = 0.0;
            }
    constexpr int FOLDQ = kFoldSrc / 4;
    int since = 0;
    for (int q = q0; q < q1; ++q) {
        const long long row = (long long)(4 * q + r) * na_pad;
        const R c = cz[4 * q + r];
        const cplx<R> a0 = za[row], a1 = za[row + 16];
        const cplx<R> b0 = zb[row], b1 = zb[row + 16];
        const R ar[2] = {a0.x * c, a1.x * c}, ai[2] = {a0.y * c, a1.y * c};
        const R br[2] = {b0.x, b1.x}, bi[2] = {b0.y, b1.y};
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                vr[a][b] = MA::step(ar[a], br[b], vr[a][b]);
                vr[a][b] = MA::step(ai[a], bi[b], vr[a][b]);
                vi[a][b] = MA::step(ai[a], br[b], vi[a][b]);
                vi[a][b] = MA::step(-ar[a], bi[b], vi[a][b]);
            }
        if (std::is_same<R, float>::value && ++since == FOLDQ) {
            since = 0;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    fold<R>(vr[a][b], dr[a][b]);
                    fold<R>(vi[a][b], di[a][b]);
                }
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            fold<R>(vr[a][b], dr[a][b]);
            fold<R>(vi[a][b], di[a][b]);
        }
    double2 *o = part + ((size_t)s * ntp + blockIdx.x) * (kZTile * kZTile);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = 16 * a + MA::row(lane, e), j = 16 * b + c16;
                o[i * kZTile + j] = make_double2(dr[a][b][e], di[a][b][e]);
            }
}

__global__ __launch_bounds__(256) void k_zz_out(const double2 *part, int n_ant, int ntile, int nsplit, int add,
                                                double *vis) {
    const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long n_pairs = (long long)n_ant * (n_ant + 1) / 2;
    if (p >= n_pairs) return;
    int i, j;
    pair_decode(p, n_ant, &i, &j);
    const int I = i / kZTile, J = j / kZTile;
    const int tp = I * ntile - I * (I - 1) / 2 + (J - I);
    const int ntp = ntile * (ntile + 1) / 2;
    const size_t off = (size_t)tp * (kZTile * kZTile) + (i % kZTile) * kZTile + (j % kZTile);
    double re = 0.0, im = 0.0;
    for (int s = 0; s < nsplit; ++s) {
        const double2 v = part[(size_t)s * ntp * (kZTile * kZTile) + off];
        re += v.x;
        im += v.y;
    }
    if (add) {
        re += vis[2 * p];
        im += vis[2 * p + 1];
    }
    vis[2 * p] = re;
    vis[2 * p + 1] = im;
}

template <typename R>
void run_zz(const double *ant, int n_ant, const double *src, int n_src, const double *freq_host, int n_freq,
            const double *flux, const double *beam, int dim, int prec_bits, double *vis, void *work, size_t cap,
            hipStream_t st, StageTimer *tm) {
    const ZZShape sh = zz_shape(n_ant, n_src, prec_bits, cap);
    char *w = (char *)work;
    cplx<R> *Z = (cplx<R> *)w;
    R *cz = (R *)(w + (sh.z_bytes + 255) / 256 * 256);
    double2 *part = (double2 *)(w + (sh.z_bytes + 255) / 256 * 256 + (sh.c_bytes + 255) / 256 * 256);
    const long long n_pairs = (long long)n_ant * (n_ant + 1) / 2;
    const double csz = (double)sizeof(cplx<R>);
    tm->begin(FV_STAGE_DIRECT, st);
    int launches = 0;
    double bytes = 0.0;
    for (int f = 0; f < n_freq; ++f) {
        const double kturn = freq_host[f] / kCLight;
        const double *fl = flux + (size_t)f * n_src;
        const double *bm = beam ? beam + (size_t)f * n_src : nullptr;
        double *o = vis + 2 * (size_t)f * n_pairs;
        for (int k0 = 0; k0 < n_src; k0 += sh.kc_pad) {
            const int kc = std::min(sh.kc_pad, n_src - k0);
            const int kc_pad = (kc + 3) / 4 * 4;
            const long long nz = (long long)kc_pad * sh.na_pad;
            hipLaunchKernelGGL(k_zbuild<R>, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, st, ant, n_ant,
                               sh.na_pad, src, k0, kc, kc_pad, fl, bm, kturn, dim, Z, cz);
            const int kq = kc_pad / 4;
            // at least 8 steps of 4 sources per split
            const int nsplit = std::min(sh.nsplit, std::max(kWavesPerBlock, kq / 8 / kWavesPerBlock * kWavesPerBlock));
            hipLaunchKernelGGL(k_zz<R>, dim3((unsigned)sh.ntp, (unsigned)(nsplit / kWavesPerBlock)), dim3(256), 0, st,
                               (const cplx<R> *)Z, (const R *)cz, sh.na_pad, kc_pad, sh.ntile, nsplit, part);
            hipLaunchKernelGGL(k_zz_out, dim3((unsigned)((n_pairs + 255) / 256)), dim3(256), 0, st,
                               (const double2 *)part, n_ant, sh.ntile, nsplit, k0 > 0 ? 1 : 0, o);
            launches += 3;
            // Z written once and read once per tile pair it feeds (2 per pair,
            // at least once from HBM), partials written and read, output written
            bytes += (double)nz * csz * 2.0 + 2.0 * (double)nsplit * sh.ntp * kZTile * kZTile * 16.0 +
                     16.0 * (double)n_pairs;
        }
    }
    tm->end(st);
    tm->add(FV_STAGE_DIRECT, bytes, launches);
    FV_HIP(hipGetLastError());
}

}  // namespace

void launch_zz(const double *ant_dev, int n_ant, const double *src_dev, int n_src, const double *freq_host,
               int n_freq, const double *flux_dev, const double *beam_dev, int dim, int prec_bits, double *vis_dev,
               void *work, size_t cap, hipStream_t st, StageTimer *tm) {
    StageTimer dummy;
    if (!tm) tm = &dummy;
    if (prec_bits == 32)
        run_zz<float>(ant_dev, n_ant, src_dev, n_src, freq_host, n_freq, flux_dev, beam_dev, dim, prec_bits, vis_dev,
                      work, cap, st, tm);
    else
        run_zz<double>(ant_dev, n_ant, src_dev, n_src, freq_host, n_freq, flux_dev, beam_dev, dim, prec_bits,
                       vis_dev, work, cap, st, tm);
}

}  // namespace fv
