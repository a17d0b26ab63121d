// Drift-scan front end on the device (paper section 2.3: a rigid rotation
// set by the local sidereal time and the latitude takes pre-corrected
// equatorial positions to the local East-North-Up frame; section 2.4: an
// analytic beam evaluated in closed form at the source positions).
//
//   k_frontend  one thread per (source, time): the ENU direction
//               R(t) s_eq in FP64, then the Gaussian power beam
//               2^(-k_f theta^2), k_f = 4 / F_f^2, for every frequency; zero
//               at and below the horizon.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fv_internal.h"

namespace fv {
namespace {

__global__ __launch_bounds__(256) void k_frontend(const double *src_eq, int n_src, const double *rot, int n_freq,
                                                  const double *kbeam, int unit_beam, long long dir_stride,
                                                  long long beam_stride, double *dir, double *beam) {
    const int s = blockIdx.x * 256 + threadIdx.x, t = blockIdx.y;
    if (s >= n_src) return;
    const double *R = rot + 9 * t;  // rows E, N, U
    const double x = src_eq[3 * (size_t)s], y = src_eq[3 * (size_t)s + 1], z = src_eq[3 * (size_t)s + 2];
    const double e = R[0] * x + R[1] * y + R[2] * z;
    const double n = R[3] * x + R[4] * y + R[5] * z;
    const double u = R[6] * x + R[7] * y + R[8] * z;
    double *d = dir + t * dir_stride + 3 * (size_t)s;
    d[0] = e;
    d[1] = n;
    d[2] = u;
    double *b = beam + t * beam_stride + s;
    if (!(u > 0.0)) {
        for (int f = 0; f < n_freq; ++f) b[(size_t)f * n_src] = 0.0;
        return;
    }
    if (unit_beam) {
        for (int f = 0; f < n_freq; ++f) b[(size_t)f * n_src] = 1.0;
        return;
    }
    const double th = atan2(sqrt(e * e + n * n), u);  // zenith angle, accurate near the zenith
    const double th2 = th * th;
    for (int f = 0; f < n_freq; ++f) b[(size_t)f * n_src] = exp2(-kbeam[f] * th2);
}

}  // namespace

void launch_frontend(const double *src_eq, int n_src, int n_time, const double *rot_dev, int n_freq,
                     const double *kbeam_dev, bool unit_beam, double *dir, long long dir_stride, double *beam,
                     long long beam_stride, hipStream_t st) {
    if (n_src <= 0 || n_time <= 0) return;
    const dim3 g((unsigned)((n_src + 255) / 256), (unsigned)n_time);
    hipLaunchKernelGGL(k_frontend, g, dim3(256), 0, st, src_eq, n_src, rot_dev, n_freq, kbeam_dev, unit_beam ? 1 : 0,
                       dir_stride, beam_stride, dir, beam);
    FV_HIP(hipGetLastError());
}

}  // namespace fv
