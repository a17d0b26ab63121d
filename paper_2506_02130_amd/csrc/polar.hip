// Polarised feed products (paper section 2.1, Jones form, one shared beam):
// the four real strength vectors of P = A C A^H, and the combination of their
// transforms into the 2 x 2 products.
//
//   k_polar_strengths  per (frequency, source): C from the Stokes parameters,
//                      P = A C A^H (FP64); out [P_xx, P_yy, Re P_xy, Im P_xy]
//   k_polar_combine    per (frequency, pair): xx = T0, xy = T2 + i T3,
//                      yx = T2 - i T3, yy = T1
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fv_internal.h"

namespace fv {
namespace {

__global__ __launch_bounds__(256) void k_polar_strengths(const double *stokes, const double2 *jones, long long n_fs,
                                                         double *out) {
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n_fs; e += (long long)gridDim.x * 256) {
        const double I = stokes[e], Q = stokes[n_fs + e], U = stokes[2 * n_fs + e], V = stokes[3 * n_fs + e];
        // C = [[c00, c01], [conj(c01), c11]] with c00, c11 real
        const double c00 = I + Q, c11 = I - Q;
        const double2 c01 = make_double2(U, V);
        double pxx, pyy, pre, pim;
        if (!jones) {
            pxx = c00;
            pyy = c11;
            pre = c01.x;
            pim = c01.y;
        } else {
            const double2 a = jones[4 * e], b = jones[4 * e + 1], c = jones[4 * e + 2], d = jones[4 * e + 3];
            // M = A C: rows (a, b) and (c, d) times C
            auto mul = [](double2 x, double2 y) { return make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x); };
            auto add = [](double2 x, double2 y) { return make_double2(x.x + y.x, x.y + y.y); };
            auto scl = [](double2 x, double r) { return make_double2(x.x * r, x.y * r); };
            const double2 c10 = make_double2(c01.x, -c01.y);
            const double2 m00 = add(scl(a, c00), mul(b, c10)), m01 = add(mul(a, c01), scl(b, c11));
            const double2 m10 = add(scl(c, c00), mul(d, c10)), m11 = add(mul(c, c01), scl(d, c11));
            // P = M A^H: P_rk = sum_l M_rl conj(A_kl)
            auto cj = [](double2 x) { return make_double2(x.x, -x.y); };
            const double2 p00 = add(mul(m00, cj(a)), mul(m01, cj(b)));
            const double2 p01 = add(mul(m00, cj(c)), mul(m01, cj(d)));
            const double2 p11 = add(mul(m10, cj(c)), mul(m11, cj(d)));
            pxx = p00.x;
            pyy = p11.x;
            pre = p01.x;
            pim = p01.y;
        }
        out[e] = pxx;
        out[n_fs + e] = pyy;
        out[2 * n_fs + e] = pre;
        out[3 * n_fs + e] = pim;
    }
}

__global__ __launch_bounds__(256) void k_polar_combine(const double2 *T, long long n_fp, double2 *vis) {
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n_fp; e += (long long)gridDim.x * 256) {
        const double2 t0 = T[e], t1 = T[n_fp + e], t2 = T[2 * n_fp + e], t3 = T[3 * n_fp + e];
        vis[e] = t0;
        vis[n_fp + e] = make_double2(t2.x - t3.y, t2.y + t3.x);
        vis[2 * n_fp + e] = make_double2(t2.x + t3.y, t2.y - t3.x);
        vis[3 * n_fp + e] = t1;
    }
}

}  // namespace

void launch_polar_strengths(const double *stokes, const double *jones, long long n_fs, double *out, hipStream_t st) {
    if (n_fs <= 0) return;
    const unsigned nb = (unsigned)std::min<long long>((n_fs + 255) / 256, 4096);
    hipLaunchKernelGGL(k_polar_strengths, dim3(nb), dim3(256), 0, st, stokes, (const double2 *)jones, n_fs, out);
    FV_HIP(hipGetLastError());
}

void launch_polar_combine(const double *tmp, long long n_fp, double *vis, hipStream_t st) {
    if (n_fp <= 0) return;
    const unsigned nb = (unsigned)std::min<long long>((n_fp + 255) / 256, 8192);
    hipLaunchKernelGGL(k_polar_combine, dim3(nb), dim3(256), 0, st, (const double2 *)tmp, n_fp, (double2 *)vis);
    FV_HIP(hipGetLastError());
}

}  // namespace fv
