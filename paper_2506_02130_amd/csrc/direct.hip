// Direct evaluation of the point-source sum (paper section 2.2, the sum the
// type-3 transform replaces): one thread per (frequency, pair), sources
// staged through LDS in chunks of 256.  The phase of every term is formed in
// FP64 in turns, reduced exactly to [-1/2, 1/2], then passed to sin/cos; in
// FP32 mode the terms of one chunk are summed in FP32 and the chunk sums in
// FP64.  Plus small utility kernels (input checks, zero fill).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "dev_common.h"
#include "fv_internal.h"

namespace fv {
namespace {

template <int D, typename ACC>
__global__ __launch_bounds__(256) void k_direct(const double *ant, int n_ant, long long n_pairs, const double *src,
                                                int n_src, const double *flux, const double *beam, double kturn,
                                                double *out) {
    __shared__ double sl[256], sm[256], sn[256], sc[256];
    const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    double u = 0, v = 0, w = 0;
    if (p < n_pairs) {
        int i, j;
        pair_decode(p, n_ant, &i, &j);
        // phase turns of source s: -(nu/c) (x_i - x_j) . s
        u = -kturn * (ant[3 * (size_t)i + 0] - ant[3 * (size_t)j + 0]);
        v = -kturn * (ant[3 * (size_t)i + 1] - ant[3 * (size_t)j + 1]);
        w = D == 3 ? -kturn * (ant[3 * (size_t)i + 2] - ant[3 * (size_t)j + 2]) : 0.0;
    }
    double accr = 0.0, acci = 0.0;
    for (int s0 = 0; s0 < n_src; s0 += 256) {
        const int s = s0 + threadIdx.x;
        if (s < n_src) {
            sl[threadIdx.x] = src[3 * (size_t)s + 0];
            sm[threadIdx.x] = src[3 * (size_t)s + 1];
            sn[threadIdx.x] = src[3 * (size_t)s + 2];
            sc[threadIdx.x] = beam ? flux[s] * beam[s] : flux[s];
        }
        __syncthreads();
        const int cnt = min(256, n_src - s0);
        ACC pr = 0, pi = 0;
        for (int k = 0; k < cnt; ++k) {
            double t = u * sl[k] + v * sm[k];
            if (D == 3) t += w * sn[k];
            ACC sn_, cs_;
            sincos_turns(t, &sn_, &cs_);
            const ACC c = (ACC)sc[k];
            pr += c * cs_;
            pi += c * sn_;
        }
        accr += (double)pr;
        acci += (double)pi;
        __syncthreads();
    }
    if (p < n_pairs) {
        out[2 * p] = accr;
        out[2 * p + 1] = acci;
    }
}

// Input check of the device entry point, one pass over the inputs: per block,
// min and max of each direction component, the count of non-unit or
// non-finite directions, and over the block's contiguous range of the
// strengths the count of non-finite flux and beam values (16-byte loads when
// aligned) and the largest |flux beam|; k_validate_reduce folds the block partials and
// gathers the frequencies and antenna positions behind them, so that the host
// fetches every planning scalar with one copy.
// Non-finite flux and beam values of x[0..n) (beam b may be null) and the
// largest |x b|; 16-byte loads when both arrays are 16-byte aligned.
__device__ __forceinline__ void check_strengths(const double *x, const double *b, long long n, int t, int nth,
                                                int &bad, double &cm) {
    long long done = 0;
    if (((uintptr_t)x & 15) == 0 && ((uintptr_t)b & 15) == 0) {
        const long long n2 = n / 2;
        // kChk pairs of 16-byte loads per thread in flight before any is used
        constexpr int kChk = 4;
        for (long long i0 = t; i0 < n2; i0 += kChk * (long long)nth) {
            double2 v[kChk], g[kChk];
#pragma unroll
            for (int u = 0; u < kChk; ++u) {
                const long long i = i0 + u * (long long)nth;
                v[u] = make_double2(0.0, 0.0);
                g[u] = make_double2(1.0, 1.0);
                if (i < n2) {
                    v[u] = ((const double2 *)x)[i];
                    if (b) g[u] = ((const double2 *)b)[i];
                }
            }
#pragma unroll
            for (int u = 0; u < kChk; ++u) {
                bad += !isfinite(v[u].x) + !isfinite(v[u].y);
                if (b) bad += !isfinite(g[u].x) + !isfinite(g[u].y);
                cm = fmax(cm, fmax(fabs(v[u].x * g[u].x), fabs(v[u].y * g[u].y)));
            }
        }
        done = 2 * n2;
    }
    for (long long i = done + t; i < n; i += nth) {
        const double g = b ? b[i] : 1.0;
        bad += !isfinite(x[i]) + (b ? !isfinite(g) : 0);
        cm = fmax(cm, fabs(x[i] * g));
    }
}

// Block `blk` of `nblk` (256 threads) of the input check of one problem.
__device__ __forceinline__ void validate_block(const double *src, int n_src, const double *flux, const double *beam,
                                               long long n_fs, long long span, double *part, int blk, int nblk) {
    __shared__ double red[6][256];
    __shared__ int bsh[2][256];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    const long long tid = (long long)blk * 256 + threadIdx.x, nth = (long long)nblk * 256;
    for (long long j = tid; j < n_src; j += nth) {
        const double a = src[3 * j], b = src[3 * j + 1], c = src[3 * j + 2];
        if (!(isfinite(a) && isfinite(b) && isfinite(c)) || fabs(sqrt(a * a + b * b + c * c) - 1.0) > 1e-9) ++bad;
        lo[0] = fmin(lo[0], a);
        hi[0] = fmax(hi[0], a);
        lo[1] = fmin(lo[1], b);
        hi[1] = fmax(hi[1], b);
        lo[2] = fmin(lo[2], c);
        hi[2] = fmax(hi[2], c);
    }
    // this block's contiguous range of the strengths: non-finite count and
    // the largest |flux beam|
    const long long f0 = min((long long)blk * span, n_fs), f1 = min(f0 + span, n_fs);
    int badv = 0;
    double cm = 0.0;
    if (f1 > f0) check_strengths(flux + f0, beam ? beam + f0 : nullptr, f1 - f0, threadIdx.x, 256, badv, cm);
    for (int off = 32; off > 0; off >>= 1) cm = fmax(cm, __shfl_xor(cm, off, 64));
    __shared__ double wcm[4];
    if ((threadIdx.x & 63) == 0) wcm[threadIdx.x >> 6] = cm;
    for (int a = 0; a < 3; ++a) {
        red[2 * a][threadIdx.x] = lo[a];
        red[2 * a + 1][threadIdx.x] = hi[a];
    }
    bsh[0][threadIdx.x] = bad;
    bsh[1][threadIdx.x] = badv;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            for (int a = 0; a < 3; ++a) {
                red[2 * a][threadIdx.x] = fmin(red[2 * a][threadIdx.x], red[2 * a][threadIdx.x + off]);
                red[2 * a + 1][threadIdx.x] = fmax(red[2 * a + 1][threadIdx.x], red[2 * a + 1][threadIdx.x + off]);
            }
            bsh[0][threadIdx.x] += bsh[0][threadIdx.x + off];
            bsh[1][threadIdx.x] += bsh[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *q = part + (size_t)kValStride * blk;
        for (int k = 0; k < 6; ++k) q[k] = red[k][0];
        q[6] = (double)bsh[0][0];
        q[7] = (double)bsh[1][0];
        q[kValCmax] = fmax(fmax(wcm[0], wcm[1]), fmax(wcm[2], wcm[3]));
        q[9] = 0.0;
    }
}

__global__ __launch_bounds__(256) void k_validate(const double *src, int n_src, const double *flux,
                                                  const double *beam, long long n_fs, long long span, double *part) {
    validate_block(src, n_src, flux, beam, n_fs, span, part, blockIdx.x, gridDim.x);
}

// A batch of problems: blockIdx.y picks the problem, which has its own
// number of blocks.
__global__ __launch_bounds__(256) void k_validate_b(const ValItem *items) {
    const ValItem &v = items[blockIdx.y];
    if ((int)blockIdx.x >= v.nblk) return;
    validate_block(v.src, v.n_src, v.flux, v.beam, v.n_fs, v.span, v.part, blockIdx.x, v.nblk);
}

// The kValReduceThreads threads fold the per-block partials (thread t takes
// blocks t, t + kValReduceThreads, ...), then a butterfly across each
// wavefront's lanes and a pass over the wavefronts; every thread also helps
// gather the frequencies and antenna positions.
constexpr int kValReduceThreads = 1024;
__device__ __forceinline__ void validate_reduce(const double *part, int nblk, const double *freq, int n_freq,
                                                const double *ant, int n_ant, double *out) {
    constexpr int NW = kValReduceThreads / 64;
    __shared__ double wred[NW][8];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    double v[8] = {INFINITY, -INFINITY, INFINITY, -INFINITY, INFINITY, -INFINITY, 0.0, 0.0};
#pragma unroll 2
    for (int b = t; b < nblk; b += kValReduceThreads) {
        const double *q = part + (size_t)kValStride * b;
        for (int k = 0; k < 6; k += 2) {
            v[k] = fmin(v[k], q[k]);
            v[k + 1] = fmax(v[k + 1], q[k + 1]);
        }
        v[6] += q[6];
        v[7] += q[7];
    }
    for (int off = 32; off > 0; off >>= 1) {
        for (int k = 0; k < 6; k += 2) {
            v[k] = fmin(v[k], __shfl_xor(v[k], off, 64));
            v[k + 1] = fmax(v[k + 1], __shfl_xor(v[k + 1], off, 64));
        }
        v[6] += __shfl_xor(v[6], off, 64);
        v[7] += __shfl_xor(v[7], off, 64);
    }
    if (lane == 0)
        for (int k = 0; k < 8; ++k) wred[wave][k] = v[k];
    __syncthreads();
    if (t < 8) {
        double r = wred[0][t];
        for (int w = 1; w < NW; ++w) {
            const double x = wred[w][t];
            r = t < 6 ? ((t & 1) ? fmax(r, x) : fmin(r, x)) : r + x;
        }
        out[t] = r;
    }
    for (int i = t; i < n_freq; i += kValReduceThreads) out[8 + i] = freq[i];
    for (int i = t; i < 3 * n_ant; i += kValReduceThreads) out[8 + n_freq + i] = ant[i];
}

__global__ __launch_bounds__(kValReduceThreads) void k_validate_reduce(const double *part, int nblk,
                                                                       const double *freq, int n_freq,
                                                                       const double *ant, int n_ant, double *out) {
    validate_reduce(part, nblk, freq, n_freq, ant, n_ant, out);
}

__global__ __launch_bounds__(kValReduceThreads) void k_validate_reduce_b(const ValItem *items) {
    const ValItem &v = items[blockIdx.x];
    validate_reduce(v.part, v.nblk, v.freq, v.n_freq, v.ant, v.n_ant, v.hdr);
}

__global__ void k_zero_f64(double *p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

}  // namespace

void launch_direct(const double *ant_dev, int n_ant, const double *src_dev, int n_src, const double *freq_host,
                   int n_freq, const double *flux_dev, const double *beam_dev, int dim, int prec_bits, double *vis_dev,
                   hipStream_t st, StageTimer *tm) {
    const long long n_pairs = (long long)n_ant * (n_ant + 1) / 2;
    const unsigned nb = (unsigned)((n_pairs + 255) / 256);
    StageTimer dummy;
    if (!tm) tm = &dummy;
    tm->begin(FV_STAGE_DIRECT, st);
    for (int f = 0; f < n_freq; ++f) {
        const double kturn = freq_host[f] / kCLight;
        const double *fl = flux_dev + (size_t)f * n_src;
        const double *bm = beam_dev ? beam_dev + (size_t)f * n_src : nullptr;
        double *o = vis_dev + 2 * (size_t)f * n_pairs;
        if (dim == 2) {
            if (prec_bits == 32)
                hipLaunchKernelGGL((k_direct<2, float>), dim3(nb), dim3(256), 0, st, ant_dev, n_ant, n_pairs, src_dev,
                                   n_src, fl, bm, kturn, o);
            else
                hipLaunchKernelGGL((k_direct<2, double>), dim3(nb), dim3(256), 0, st, ant_dev, n_ant, n_pairs, src_dev,
                                   n_src, fl, bm, kturn, o);
        } else {
            if (prec_bits == 32)
                hipLaunchKernelGGL((k_direct<3, float>), dim3(nb), dim3(256), 0, st, ant_dev, n_ant, n_pairs, src_dev,
                                   n_src, fl, bm, kturn, o);
            else
                hipLaunchKernelGGL((k_direct<3, double>), dim3(nb), dim3(256), 0, st, ant_dev, n_ant, n_pairs, src_dev,
                                   n_src, fl, bm, kturn, o);
        }
    }
    tm->end(st);
    // inputs read once per frequency (directions, strengths), outputs written once
    tm->add(FV_STAGE_DIRECT, (double)n_freq * ((double)n_src * (24.0 + (beam_dev ? 16.0 : 8.0)) + 16.0 * n_pairs),
            n_freq);
    FV_HIP(hipGetLastError());
}

size_t validate_doubles(int n_ant, int n_freq) {
    return 8 + (size_t)n_freq + 3 * (size_t)n_ant + (size_t)kValStride * kSrcCheckBlocks;
}

void launch_validate(const double *src, int n_src, const double *flux, const double *beam, int n_freq,
                     const double *ant, int n_ant, const double *freq, double *out, hipStream_t st) {
    double *part = out + 8 + n_freq + 3 * (size_t)n_ant;
    const long long n_fs = n_src > 0 ? (long long)n_src * n_freq : 0;
    hipLaunchKernelGGL(k_validate, dim3(kSrcCheckBlocks), dim3(256), 0, st, n_src > 0 ? src : nullptr, n_src,
                       n_src > 0 ? flux : nullptr, n_src > 0 ? beam : nullptr, n_fs, validate_span(n_fs), part);
    hipLaunchKernelGGL(k_validate_reduce, dim3(1), dim3(kValReduceThreads), 0, st, (const double *)part, kSrcCheckBlocks, freq,
                       n_freq, ant, n_ant, out);
    FV_HIP(hipGetLastError());
}

int validate_blocks_batch(long long n_src, long long n_fs) {
    // about 16k strengths and 2k directions per block, at least one block
    const long long b = std::max((n_fs + 16383) / 16384, (n_src + 2047) / 2048);
    return (int)std::max(1LL, std::min(b, (long long)kSrcCheckBlocks));
}

void launch_validate_batch(const ValItem *items_dev, int n, int max_blk, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_validate_b, dim3((unsigned)max_blk, (unsigned)n), dim3(256), 0, st, items_dev);
    hipLaunchKernelGGL(k_validate_reduce_b, dim3((unsigned)n), dim3(kValReduceThreads), 0, st, items_dev);
    FV_HIP(hipGetLastError());
}

void launch_zero_c128(double *out, long long n_complex, hipStream_t st) {
    const long long n = 2 * n_complex;
    const unsigned nb = (unsigned)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_zero_f64, dim3(std::max(1u, nb)), dim3(256), 0, st, out, n);
    FV_HIP(hipGetLastError());
}

}  // namespace fv
