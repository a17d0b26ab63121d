// Spectral basis (paper appendix A): per-source product coefficients in an
// orthonormal spectral basis.  (The expansion of the basis transforms back to
// the frequencies is part of the interpolation, k_interp_basis.)
//
//   k_basis_coeffs  per source: s_hat = M^T flux, b_hat = M^T beam (M has
//                   orthonormal columns, so (M^T M)^-1 M^T = M^T), then
//                   v_k = sum_ij s_hat_i b_hat_j d_ijk (FP64)
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fv_internal.h"

namespace fv {
namespace {

constexpr int kMaxBasis = 16;

// A workgroup takes 64 sources; its 4 wavefronts split the frequencies
// (wavefront w takes q = w mod 4) so that each lane keeps several loads in
// flight, then the partial projections meet in LDS and wavefront w forms the
// outputs k = w mod 4.
__global__ __launch_bounds__(256) void k_basis_coeffs(const double *M, const double *d, int n_freq, int K, int n_src,
                                                      const double *flux, const double *beam, double *v) {
    extern __shared__ double sm[];  // M [n_freq][K], d [K][K][K], partials [4][2K][64]
    double *sM = sm, *sd = sm + n_freq * K, *part = sd + K * K * K;
    for (int i = threadIdx.x; i < n_freq * K; i += 256) sM[i] = M[i];
    for (int i = threadIdx.x; i < K * K * K; i += 256) sd[i] = d[i];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int s = blockIdx.x * 64 + lane;
    const bool act = s < n_src;
    double sh[kMaxBasis], bh[kMaxBasis];
#pragma unroll
    for (int i = 0; i < kMaxBasis; ++i) sh[i] = bh[i] = 0.0;
    if (act) {
        constexpr int U = 4;  // frequencies per lane whose loads are issued together
        for (int q0 = wave; q0 < n_freq; q0 += 4 * U) {
            double f[U], b[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = q0 + 4 * u;
                f[u] = q < n_freq ? flux[(size_t)q * n_src + s] : 0.0;
                b[u] = q < n_freq ? (beam ? beam[(size_t)q * n_src + s] : 1.0) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = q0 + 4 * u;
                if (q >= n_freq) break;
#pragma unroll
                for (int i = 0; i < kMaxBasis; ++i)
                    if (i < K) {
                        sh[i] += sM[q * K + i] * f[u];
                        bh[i] += sM[q * K + i] * b[u];
                    }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < kMaxBasis; ++i)
        if (i < K) {
            part[(wave * 2 * K + i) * 64 + lane] = sh[i];
            part[(wave * 2 * K + K + i) * 64 + lane] = bh[i];
        }
    __syncthreads();
    if (!act) return;
#pragma unroll
    for (int i = 0; i < kMaxBasis; ++i)
        if (i < K) {
            double a = 0.0, c = 0.0;
            for (int w = 0; w < 4; ++w) {
                a += part[(w * 2 * K + i) * 64 + lane];
                c += part[(w * 2 * K + K + i) * 64 + lane];
            }
            sh[i] = a;
            bh[i] = c;
        }
    for (int k = wave; k < K; k += 4) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < kMaxBasis; ++i)
            if (i < K) {
                double t = 0.0;
#pragma unroll
                for (int j = 0; j < kMaxBasis; ++j)
                    if (j < K) t += bh[j] * sd[(i * K + j) * K + k];
                acc += sh[i] * t;
            }
        v[(size_t)k * n_src + s] = acc;
    }
}

}  // namespace

int basis_max() { return kMaxBasis; }

void launch_basis_coeffs(const double *M_dev, const double *d_dev, int n_freq, int K, int n_src, const double *flux,
                         const double *beam, double *v, hipStream_t st) {
    if (n_src <= 0) return;
    if (K < 1 || K > kMaxBasis) fail(FV_EINVAL, "basis size out of range");
    const size_t lds = sizeof(double) * ((size_t)n_freq * K + (size_t)K * K * K + (size_t)4 * 2 * K * 64);
    if (lds > 160 * 1024) fail(FV_EUNSUPPORTED, "basis tables exceed LDS (too many frequencies for this basis size)");
    ensure_lds((const void *)k_basis_coeffs, lds);
    hipLaunchKernelGGL(k_basis_coeffs, dim3((unsigned)((n_src + 63) / 64)), dim3(256), lds, st, M_dev, d_dev, n_freq,
                       K, n_src, flux, beam, v);
    FV_HIP(hipGetLastError());
}

}  // namespace fv
