// Per-antenna beams (paper section 2.2.3): the strengths of every pattern pair
// that occurs, and the gather of each visibility from its pair's transform.
//
//   k_beam_products  prod[v][f][s] = a_{p_v}[f][s] a_{q_v}[f][s]
//   k_beam_select    vis[f][k] = tmp[vec[k]][f][k]
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fv_internal.h"

namespace fv {
namespace {

__global__ __launch_bounds__(256) void k_beam_products(const double *beams, const int *pq, int n_vec, long long n_fs,
                                                       double *prod) {
    const int v = blockIdx.y;
    const double *a = beams + (size_t)pq[2 * v] * n_fs, *b = beams + (size_t)pq[2 * v + 1] * n_fs;
    double *o = prod + (size_t)v * n_fs;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n_fs; i += (long long)gridDim.x * 256)
        o[i] = a[i] * b[i];
}

__global__ __launch_bounds__(256) void k_beam_select(const double2 *tmp, const int *vec, long long n_pairs, int n_freq,
                                                     double2 *vis) {
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    const int f = blockIdx.y;
    if (k >= n_pairs) return;
    vis[(size_t)f * n_pairs + k] = tmp[((size_t)vec[k] * n_freq + f) * n_pairs + k];
}

}  // namespace

void launch_beam_products(const double *beams, const int *pq_dev, int n_vec, long long n_fs, double *prod,
                          hipStream_t st) {
    if (n_vec <= 0 || n_fs <= 0) return;
    const unsigned nb = (unsigned)std::min<long long>((n_fs + 255) / 256, 2048);
    hipLaunchKernelGGL(k_beam_products, dim3(nb, (unsigned)n_vec), dim3(256), 0, st, beams, pq_dev, n_vec, n_fs, prod);
    FV_HIP(hipGetLastError());
}

void launch_beam_select(const double *tmp, const int *vec_dev, long long n_pairs, int n_freq, double *vis,
                        hipStream_t st) {
    if (n_pairs <= 0) return;
    const dim3 g((unsigned)((n_pairs + 255) / 256), (unsigned)n_freq);
    hipLaunchKernelGGL(k_beam_select, g, dim3(256), 0, st, (const double2 *)tmp, vec_dev, n_pairs, n_freq,
                       (double2 *)vis);
    FV_HIP(hipGetLastError());
}

}  // namespace fv
