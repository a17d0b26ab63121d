// Spectral basis (paper appendix A): per-source product coefficients in an
// orthonormal spectral basis, and the expansion of the basis transforms back
// to the frequencies.
//
//   k_basis_coeffs  per source: s_hat = M^T flux, b_hat = M^T beam (M has
//                   orthonormal columns, so (M^T M)^-1 M^T = M^T), then
//                   v_k = sum_ij s_hat_i b_hat_j d_ijk (FP64)
//   k_basis_expand  per (frequency, pair): V = sum_k M_qk F_k
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fv_internal.h"

namespace fv {
namespace {

constexpr int kMaxBasis = 16;

__global__ __launch_bounds__(256) void k_basis_coeffs(const double *M, const double *d, int n_freq, int K, int n_src,
                                                      const double *flux, const double *beam, double *v) {
    extern __shared__ double sm[];  // M [n_freq][K], d [K][K][K]
    double *sM = sm, *sd = sm + n_freq * K;
    for (int i = threadIdx.x; i < n_freq * K; i += 256) sM[i] = M[i];
    for (int i = threadIdx.x; i < K * K * K; i += 256) sd[i] = d[i];
    __syncthreads();
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n_src) return;
    double sh[kMaxBasis], bh[kMaxBasis];
    for (int i = 0; i < K; ++i) sh[i] = bh[i] = 0.0;
    for (int q = 0; q < n_freq; ++q) {
        const double f = flux[(size_t)q * n_src + s], b = beam ? beam[(size_t)q * n_src + s] : 1.0;
        for (int i = 0; i < K; ++i) {
            sh[i] += sM[q * K + i] * f;
            bh[i] += sM[q * K + i] * b;
        }
    }
    for (int k = 0; k < K; ++k) {
        double acc = 0.0;
        for (int i = 0; i < K; ++i) {
            double t = 0.0;
            for (int j = 0; j < K; ++j) t += bh[j] * sd[(i * K + j) * K + k];
            acc += sh[i] * t;
        }
        v[(size_t)k * n_src + s] = acc;
    }
}

__global__ __launch_bounds__(256) void k_basis_expand(const double *M, int K, int n_freq, long long n_pairs,
                                                      const double2 *F, double2 *vis) {
    const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    const int q = blockIdx.y;
    if (p >= n_pairs) return;
    double re = 0.0, im = 0.0;
    for (int k = 0; k < K; ++k) {
        const double m = M[q * K + k];
        const double2 f = F[((size_t)k * n_freq + q) * n_pairs + p];
        re += m * f.x;
        im += m * f.y;
    }
    vis[(size_t)q * n_pairs + p] = make_double2(re, im);
}

}  // namespace

int basis_max() { return kMaxBasis; }

void launch_basis_coeffs(const double *M_dev, const double *d_dev, int n_freq, int K, int n_src, const double *flux,
                         const double *beam, double *v, hipStream_t st) {
    if (n_src <= 0) return;
    if (K < 1 || K > kMaxBasis) fail(FV_EINVAL, "basis size out of range");
    const size_t lds = sizeof(double) * ((size_t)n_freq * K + (size_t)K * K * K);
    if (lds > 160 * 1024) fail(FV_EUNSUPPORTED, "basis tables exceed LDS (too many frequencies for this basis size)");
    ensure_lds((const void *)k_basis_coeffs, lds);
    hipLaunchKernelGGL(k_basis_coeffs, dim3((unsigned)((n_src + 255) / 256)), dim3(256), lds, st, M_dev, d_dev, n_freq,
                       K, n_src, flux, beam, v);
    FV_HIP(hipGetLastError());
}

void launch_basis_expand(const double *M_dev, int K, int n_freq, long long n_pairs, const double *F, double *vis,
                         hipStream_t st) {
    if (n_pairs <= 0) return;
    hipLaunchKernelGGL(k_basis_expand, dim3((unsigned)((n_pairs + 255) / 256), (unsigned)n_freq), dim3(256), 0, st,
                       M_dev, K, n_freq, n_pairs, (const double2 *)F, (double2 *)vis);
    FV_HIP(hipGetLastError());
}

}  // namespace fv
