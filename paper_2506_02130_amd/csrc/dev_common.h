// Device helpers shared by the HIP kernels: complex arithmetic, the ES kernel,
// sin/cos of phases given in turns, and the quadrature for the kernel's
// Fourier transform.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fv_internal.h"

namespace fv {

template <typename R>
using cplx = typename std::conditional<std::is_same<R, float>::value, float2, double2>::type;

template <typename R>
__device__ __forceinline__ cplx<R> cmake(R re, R im) {
    cplx<R> z;
    z.x = re;
    z.y = im;
    return z;
}
template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return cmake<R>(a.x + b.x, a.y + b.y); }
template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return cmake<R>(a.x - b.x, a.y - b.y); }
template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
    return cmake<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R>
__device__ __forceinline__ cplx<R> cscale(cplx<R> a, R s) { return cmake<R>(a.x * s, a.y * s); }
// multiply by +i
template <typename R>
__device__ __forceinline__ cplx<R> cmuli(cplx<R> a) { return cmake<R>(-a.y, a.x); }

// ES kernel phi(z) = exp(beta (sqrt(1 - z^2) - 1)) for |z| <= 1 (paper
// section 2.2, step 1).  Callers only pass |z| <= 1 up to rounding.  The
// exponent is formed as -beta z^2 / (1 + sqrt(1 - z^2)), the same value
// without the cancellation of sqrt(1 - z^2) - 1 near the kernel's centre
// (where the weights are largest): in FP32 that cancellation alone gave the
// weights a weighted rms error of 3.7e-7, against 6e-8 for this form.
__device__ __forceinline__ float es_phi(float z, float beta) {
    const float z2 = z * z;
    return expf(-beta * z2 / (1.0f + sqrtf(fmaxf(1.0f - z2, 0.0f))));
}
__device__ __forceinline__ double es_phi(double z, double beta) {
    const double z2 = z * z;
    return exp(-beta * z2 / (1.0 + sqrt(fmax(1.0 - z2, 0.0))));
}
// FP32 with hardware exp2, sqrt and reciprocal (about 1 ulp each).
__device__ __forceinline__ float es_phi_fast(float z, float beta) {
    const float z2 = z * z;
    return __expf(-beta * z2 * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_sqrtf(fmaxf(1.0f - z2, 0.0f))));
}
__device__ __forceinline__ double es_phi_fast(double z, double beta) { return es_phi(z, beta); }

// The W weights of the kernel from its piecewise polynomials (W <= kPolyMaxW),
// u = 2 offset - W + 1: piece i is E(u^2) + u O(u^2) with its even and odd
// parts, and its mirror W - 1 - i is E - u O.  No transcendental functions.
template <int W>
__device__ __forceinline__ void es_weights_poly(const EsPoly &P, float u, float *wt) {
    static_assert(W <= kPolyMaxW, "no polynomial table for this width");
    constexpr int D = W + 2, De = D - (D & 1), Do = D - 1 + (D & 1);
    const float v = u * u;
#pragma unroll
    for (int i = 0; i < (W + 1) / 2; ++i) {
        float e = P.c[i][De], od = P.c[i][Do];
#pragma unroll
        for (int k = De - 2; k >= 0; k -= 2) e = fmaf(e, v, P.c[i][k]);
#pragma unroll
        for (int k = Do - 2; k >= 1; k -= 2) od = fmaf(od, v, P.c[i][k]);
        wt[i] = fmaf(u, od, e);
        if (W - 1 - i != i) wt[W - 1 - i] = fmaf(-u, od, e);
    }
}

// sin and cos of 2 pi t, with t in turns reduced exactly in FP64 first.
__device__ __forceinline__ void sincos_turns(double t, double *s, double *c) {
    double r = t - rint(t);
    sincospi(2.0 * r, s, c);
}
__device__ __forceinline__ void sincos_turns(double t, float *s, float *c) {
    double r = t - rint(t);
    sincospif((float)(2.0 * r), s, c);
}

// phihat(xi) = int_{-1}^{1} phi(z) cos(xi z) dz by the 64-node Gauss-Legendre
// rule in theta (z = sin theta); qn[q] = sin(theta_q) for the positive nodes,
// qn[kQuadHalf + q] = 2 * weight * exp(beta (cos theta_q - 1)) cos theta_q.
__device__ __forceinline__ double phihat_quad(double xi, const double *qn) {
    double acc = 0.0;
#pragma unroll 8
    for (int q = 0; q < kQuadHalf; ++q) acc += qn[kQuadHalf + q] * cos(xi * qn[q]);
    return acc;
}

// One 16x16x4 matrix-core step D += A B on a wavefront: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].
typedef float mfma_f4 __attribute__((ext_vector_type(4)));
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <typename R>
struct MfmaAcc;
template <>
struct MfmaAcc<float> {
    typedef mfma_f4 T;
    static __device__ __forceinline__ T step(float a, float b, T c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // accumulator register r of lane l holds row 4 (l / 16) + r, column l % 16
    static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <>
struct MfmaAcc<double> {
    typedef mfma_d4 T;
    static __device__ __forceinline__ T step(double a, double b, T c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // accumulator register r of lane l holds row (l / 16) + 4 r, column l % 16
    static __device__ __forceinline__ int row(int l, int r) { return (l >> 4) + 4 * r; }
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float readlane_f(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double readlane_d(double v, int l) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename R>
__device__ __forceinline__ R readlane_r(R v, int l);
template <>
__device__ __forceinline__ float readlane_r<float>(float v, int l) { return readlane_f(v, l); }
template <>
__device__ __forceinline__ double readlane_r<double>(double v, int l) { return readlane_d(v, l); }

// Row of the (i <= j) row-major pair layout: start(i) = i n - i (i - 1) / 2.
__device__ __forceinline__ void pair_decode(long long p, int n, int *pi, int *pj) {
    double tt = 2.0 * n + 1.0;
    long long i = (long long)floor(0.5 * (tt - sqrt(fmax(tt * tt - 8.0 * (double)p, 0.0))));
    if (i < 0) i = 0;
    if (i > n - 1) i = n - 1;
    auto start = [n](long long r) { return r * n - r * (r - 1) / 2; };
    while (i + 1 < n && start(i + 1) <= p) ++i;
    while (i > 0 && start(i) > p) --i;
    *pi = (int)i;
    *pj = (int)(i + (p - start(i)));
}

}  // namespace fv
