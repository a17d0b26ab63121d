// Drift-scan front end on the device (paper section 2.3: a rigid rotation
// set by the local sidereal time and the latitude takes pre-corrected
// equatorial positions to the local East-North-Up frame; section 2.4: an
// analytic beam evaluated in closed form at the source positions).  Sources
// at or below the horizon have zero beam; they are dropped, and the ones
// above are packed in their input order, so every later stage works on the
// visible sky only.
//
//   k_fe_count  one thread per (source, time): is the rotated source above
//               the horizon; per block of 256 sources the count.  The blocks
//               of the first time also count invalid inputs (non-finite or
//               non-unit vectors, non-finite fluxes).
//   k_fe_scan   one workgroup per time: exclusive offsets of the block counts
//               and the number of visible sources.
//   k_frontend  one thread per (source, time): the ENU direction R(t) s_eq
//               (FP64) and the strengths flux * 2^(-k_f theta^2),
//               k_f = 4 / F_f^2, written at the source's packed index.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fv_internal.h"

namespace fv {
namespace {


__device__ __forceinline__ void fe_rotate(const double *R, double x, double y, double z, double &e, double &n,
                                          double &u) {
    e = R[0] * x + R[1] * y + R[2] * z;
    n = R[3] * x + R[4] * y + R[5] * z;
    u = R[6] * x + R[7] * y + R[8] * z;
}

__global__ __launch_bounds__(kFeBlock) void k_fe_count(const double *src_eq, int n_src, const double *rot,
                                                       const double *flux, int n_freq, int nb, int *bcnt,
                                                       int *bbad) {
    const int s = blockIdx.x * kFeBlock + threadIdx.x, t = blockIdx.y;
    int up = 0, bad = 0;
    if (s < n_src) {
        const double x = src_eq[3 * (size_t)s], y = src_eq[3 * (size_t)s + 1], z = src_eq[3 * (size_t)s + 2];
        double e, n, u;
        fe_rotate(rot + 9 * t, x, y, z, e, n, u);
        up = u > 0.0;
        if (t == 0) {
            bad = !(isfinite(x) && isfinite(y) && isfinite(z)) || fabs(sqrt(x * x + y * y + z * z) - 1.0) > 1e-9;
            for (int f = 0; f < n_freq; ++f) bad |= !isfinite(flux[(size_t)f * n_src + s]);
        }
    }
    const int c = __syncthreads_count(up);
    const int nbad = __syncthreads_count(bad);
    if (threadIdx.x == 0) {
        bcnt[(size_t)t * nb + blockIdx.x] = c;
        if (t == 0) bbad[blockIdx.x] = nbad;
    }
}

// Inclusive sum over the 1024 threads of the workgroup.
__device__ int block_scan_1024(int v, int *wsum) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    if (lane == 63) wsum[wave] = v;
    __syncthreads();
    int base = 0;
    for (int w = 0; w < wave; ++w) base += wsum[w];
    __syncthreads();
    return v + base;
}

__global__ __launch_bounds__(1024) void k_fe_scan(int *bcnt, int nb, const int *bbad, int *tot) {
    __shared__ int wsum[16];
    __shared__ int total;
    const int t = blockIdx.x;
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 1024) {
        const int i = b0 + threadIdx.x;
        const int v = i < nb ? bcnt[(size_t)t * nb + i] : 0;
        const int incl = block_scan_1024(v, wsum);
        if (i < nb) bcnt[(size_t)t * nb + i] = carry + incl - v;
        if (threadIdx.x == 1023) total = incl;
        __syncthreads();
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) tot[t] = carry;
    if (t == 0) {  // invalid inputs, counted by the first time's blocks
        int bad = 0;
        for (int i = threadIdx.x; i < nb; i += 1024) bad += bbad[i];
        const int all = block_scan_1024(bad, wsum);
        if (threadIdx.x == 1023) tot[gridDim.x] = all;
    }
}

__global__ __launch_bounds__(kFeBlock) void k_frontend(const double *src_eq, int n_src, const double *rot,
                                                       const double *flux, int n_freq, const double *kbeam,
                                                       int unit_beam, int nb, const int *boff, const int *tot,
                                                       long long dir_stride, long long str_stride, double *dir,
                                                       double *str) {
    __shared__ int wcnt[kFeBlock / 64];
    const int s = blockIdx.x * kFeBlock + threadIdx.x, t = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double e = 0.0, n = 0.0, u = 0.0;
    if (s < n_src) fe_rotate(rot + 9 * t, src_eq[3 * (size_t)s], src_eq[3 * (size_t)s + 1], src_eq[3 * (size_t)s + 2],
                             e, n, u);
    const bool up = s < n_src && u > 0.0;
    // packed index: block offset + visible sources before this one in the block
    const unsigned long long m = __ballot(up);
    if (lane == 0) wcnt[wave] = __popcll(m);
    __syncthreads();
    int k = boff[(size_t)t * nb + blockIdx.x] + __popcll(m & ((1ull << lane) - 1ull));
    for (int w = 0; w < wave; ++w) k += wcnt[w];
    if (!up) return;
    double *d = dir + t * dir_stride + 3 * (size_t)k;
    d[0] = e;
    d[1] = n;
    d[2] = u;
    const int cnt = tot[t];
    double *c = str + t * str_stride + k;
    if (unit_beam) {
        for (int f = 0; f < n_freq; ++f) c[(size_t)f * cnt] = flux[(size_t)f * n_src + s];
        return;
    }
    const double th = atan2(sqrt(e * e + n * n), u);  // zenith angle, accurate near the zenith
    const double th2 = th * th;
    for (int f = 0; f < n_freq; ++f) c[(size_t)f * cnt] = flux[(size_t)f * n_src + s] * exp2(-kbeam[f] * th2);
}

}  // namespace


void launch_frontend_count(const double *src_eq, int n_src, int n_time, const double *rot_dev, const double *flux,
                           int n_freq, int *bcnt, int *bbad, int *tot, hipStream_t st) {
    const int nb = frontend_blocks(n_src);
    if (nb > 0) {
        hipLaunchKernelGGL(k_fe_count, dim3((unsigned)nb, (unsigned)n_time), dim3(kFeBlock), 0, st, src_eq, n_src,
                           rot_dev, flux, n_freq, nb, bcnt, bbad);
    }
    hipLaunchKernelGGL(k_fe_scan, dim3((unsigned)n_time), dim3(1024), 0, st, bcnt, nb, (const int *)bbad, tot);
    FV_HIP(hipGetLastError());
}

void launch_frontend(const double *src_eq, int n_src, int n_time, const double *rot_dev, const double *flux,
                     int n_freq, const double *kbeam_dev, bool unit_beam, const int *boff, const int *tot, double *dir,
                     long long dir_stride, double *str, long long str_stride, hipStream_t st) {
    const int nb = frontend_blocks(n_src);
    if (nb <= 0 || n_time <= 0) return;
    hipLaunchKernelGGL(k_frontend, dim3((unsigned)nb, (unsigned)n_time), dim3(kFeBlock), 0, st, src_eq, n_src,
                       rot_dev, flux, n_freq, kbeam_dev, unit_beam ? 1 : 0, nb, boff, tot, dir_stride, str_stride,
                       dir, str);
    FV_HIP(hipGetLastError());
}

}  // namespace fv
