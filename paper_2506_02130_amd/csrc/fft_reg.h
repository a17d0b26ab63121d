// Oversampled FFT pass with compile-time plans (paper section 2.2, step 2:
// the FFT of the deconvolved, zero-padded modes), FP32.
//
// A line holds the n1 = L deconvolved modes b~_m, m in [-L/2, L/2), and the
// pass needs g_p = sum_m b~_m W_2L^(m p) at p in [-P, P] only (W_n =
// exp(+2 pi i / n)).  As in the general kernel, the even outputs g_2k are the
// L-point transform of a[j] = b~ at j = m mod L, and the odd outputs g_2k+1
// the L-point transform of s_j W_2L^j a[j] (s_j = -1 for j >= L/2): two
// L-point transforms per line, no zero padding stored.  Here the two run one
// after the other (the "parity phases"), and each is a Stockham FFT whose
// steps are composite radices F_g computed in registers:
//
//   * thread t of a line (T = L / E threads per line) holds the E points at
//     positions t + T m, m < E, in every group: group g reads them, runs E/F_g
//     butterflies of radix F_g (butterfly u takes slots u + j E/F_g), and
//     writes its outputs to the Stockham positions of the next group in LDS;
//   * the line touches LDS only between groups (one write, one barrier, one
//     read), with each group's twiddles W_L^e read from a table in LDS;
//   * the first group's input comes straight from global memory (coalesced:
//     lanes t, t + 1, ... read neighbouring elements), and the last group's
//     outputs X[t + T m] go straight to global memory, only those inside the
//     window p in [-P, P].
//
// Every index is a compile-time constant plus the thread's t; there is no
// runtime division and no twiddle product.  The plans (E, the radices, lines
// per workgroup) are in fft_plans_rows.inc and fft_plans_cols.inc, one per supported L.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "dev_common.h"
#include "fft_plan_math.h"
#include "fv_internal.h"

namespace fv {
namespace fftr {

// ---------------------------------------------------------------------------
// cos and sin of 2 pi e / n at compile time: the angle is reduced to
// [0, pi/4] in integer arithmetic, then Taylor series in double.
struct CD {
    double c, s;
};
constexpr double kPiD = 3.14159265358979323846264338327950288;
constexpr double tsin(double x) {
    double t = x, s = x;
    for (int k = 1; k < 14; ++k) {
        t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        s += t;
    }
    return s;
}
constexpr double tcos(double x) {
    double t = 1.0, s = 1.0;
    for (int k = 1; k < 14; ++k) {
        t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        s += t;
    }
    return s;
}
constexpr CD turn(long long e, long long n) {
    e %= n;
    if (e < 0) e += n;
    const long long q = (8 * e) / (2 * n);  // quadrant
    const long long r = 8 * e - q * 2 * n;  // angle within the quadrant: (pi/4) r / n, r in [0, 2n)
    double c = 0, s = 0;
    if (r <= n) {
        const double a = kPiD / 4.0 * (double)r / (double)n;
        c = tcos(a);
        s = tsin(a);
    } else {
        const double b = kPiD / 4.0 * (double)(2 * n - r) / (double)n;
        c = tsin(b);
        s = tcos(b);
    }
    switch (q) {
        case 0: return CD{c, s};
        case 1: return CD{-s, c};
        case 2: return CD{-c, -s};
        default: return CD{s, -c};
    }
}

// static loop: f(std::integral_constant<int, i>) for i < N
template <typename Fn, int... I>
__device__ __forceinline__ void sfor_(Fn &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename Fn>
__device__ __forceinline__ void sfor(Fn &&f) {
    sfor_(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ float2 c2(float x, float y) { return make_float2(x, y); }
__device__ __forceinline__ float2 add(float2 a, float2 b) { return c2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 sub(float2 a, float2 b) { return c2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 mul(float2 a, float2 w) { return c2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x); }
__device__ __forceinline__ float2 muli(float2 a) { return c2(-a.y, a.x); }
// Streaming grid accesses: nontemporal, so that the twiddle tables stay cached.
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld_stream(const float2 *p) {
    const f2v v = __builtin_nontemporal_load((const f2v *)p);
    return c2(v.x, v.y);
}
__device__ __forceinline__ void st_stream(float2 *p, float2 x) {
    f2v v;
    v.x = x.x;
    v.y = x.y;
    __builtin_nontemporal_store(v, (f2v *)p);
}

// a * W_N^E with N, E compile-time; the multiples of pi/4 need no general product
template <int N, int E>
__device__ __forceinline__ float2 twc(float2 a) {
    constexpr int e = ((E % N) + N) % N;
    constexpr float h = 0.70710678118654752440f;
    if constexpr (e == 0) return a;
    else if constexpr (4 * e == N) return c2(-a.y, a.x);
    else if constexpr (2 * e == N) return c2(-a.x, -a.y);
    else if constexpr (4 * e == 3 * N) return c2(a.y, -a.x);
    else if constexpr (8 * e == N) return c2(h * (a.x - a.y), h * (a.x + a.y));
    else if constexpr (8 * e == 3 * N) return c2(-h * (a.x + a.y), h * (a.x - a.y));
    else if constexpr (8 * e == 5 * N) return c2(h * (a.y - a.x), -h * (a.x + a.y));
    else if constexpr (8 * e == 7 * N) return c2(h * (a.x + a.y), h * (a.y - a.x));
    else {
        constexpr CD w = turn(e, N);
        constexpr float wc = (float)w.c, ws = (float)w.s;
        return c2(a.x * wc - a.y * ws, a.x * ws + a.y * wc);
    }
}

// In-place F-point DFT with the + sign: X_k = sum_n x_n W_F^(n k).
template <int F>
struct Dft;
template <>
struct Dft<2> {
    static __device__ __forceinline__ void run(float2 *v) {
        const float2 a = v[0], b = v[1];
        v[0] = add(a, b);
        v[1] = sub(a, b);
    }
};
template <>
struct Dft<3> {
    static __device__ __forceinline__ void run(float2 *v) {
        const float s3 = 0.86602540378443864676f;
        const float2 t1 = add(v[1], v[2]), t2 = sub(v[1], v[2]);
        const float2 m = c2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
        const float2 it = c2(-s3 * t2.y, s3 * t2.x);
        v[0] = add(v[0], t1);
        v[1] = add(m, it);
        v[2] = sub(m, it);
    }
};
template <>
struct Dft<4> {
    static __device__ __forceinline__ void run(float2 *v) {
        const float2 a = add(v[0], v[2]), b = sub(v[0], v[2]);
        const float2 c = add(v[1], v[3]), d = muli(sub(v[1], v[3]));
        v[0] = add(a, c);
        v[2] = sub(a, c);
        v[1] = add(b, d);
        v[3] = sub(b, d);
    }
};
template <>
struct Dft<5> {
    static __device__ __forceinline__ void run(float2 *v) {
        const float c1 = 0.30901699437494742410f, c2_ = -0.80901699437494742410f;
        const float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;
        const float2 a1 = add(v[1], v[4]), b1 = sub(v[1], v[4]);
        const float2 a2 = add(v[2], v[3]), b2 = sub(v[2], v[3]);
        const float2 x0 = v[0];
        const float2 r1 = c2(x0.x + c1 * a1.x + c2_ * a2.x, x0.y + c1 * a1.y + c2_ * a2.y);
        const float2 r2 = c2(x0.x + c2_ * a1.x + c1 * a2.x, x0.y + c2_ * a1.y + c1 * a2.y);
        const float2 i1 = muli(c2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
        const float2 i2 = muli(c2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
        v[0] = add(x0, add(a1, a2));
        v[1] = add(r1, i1);
        v[4] = sub(r1, i1);
        v[2] = add(r2, i2);
        v[3] = sub(r2, i2);
    }
};
// first factor of a composite F (the plan generator assumes the same split)
template <int F>
constexpr int split_of() {
    if (F % 4 == 0 && F > 4) return 4;
    if (F % 2 == 0) return 2;
    if (F % 3 == 0) return 3;
    return 5;
}
// Composite F = A B (Cooley-Tukey): n = B n1 + n2, k = k1 + A k2,
// X[k1 + A k2] = sum_n2 W_B^(n2 k2) W_F^(n2 k1) sum_n1 x[B n1 + n2] W_A^(n1 k1).
template <int F>
struct Dft {
    static __device__ __forceinline__ void run(float2 *v) {
        constexpr int A = split_of<F>(), B = F / A;
        float2 y[F];
        sfor<B>([&](auto n2c) {
            constexpr int n2 = decltype(n2c)::value;
            float2 t[A];
            sfor<A>([&](auto n1c) { t[decltype(n1c)::value] = v[B * decltype(n1c)::value + n2]; });
            Dft<A>::run(t);
            sfor<A>([&](auto k1c) {
                constexpr int k1 = decltype(k1c)::value;
                y[n2 * A + k1] = twc<F, n2 * k1>(t[k1]);
            });
        });
        sfor<A>([&](auto k1c) {
            constexpr int k1 = decltype(k1c)::value;
            float2 s[B];
            sfor<B>([&](auto n2c) { s[decltype(n2c)::value] = y[decltype(n2c)::value * A + k1]; });
            Dft<B>::run(s);
            sfor<B>([&](auto k2c) { v[k1 + A * decltype(k2c)::value] = s[decltype(k2c)::value]; });
        });
    }
};

// ---------------------------------------------------------------------------
// A plan: L points per line, NL lines per workgroup of TPB threads, line
// stride LP in LDS, and the radices of the groups (1 past the last).  Group g
// has Q_g = L / F_g butterflies per line; the workgroup's NL Q_g butterflies
// are dealt to its threads in R_g rounds (butterfly b = thread + TPB r).
// Workgroups have 512 threads: a column workgroup then takes twice the
// columns of a 256-thread one for the same work per thread, so that each row
// segment it reads and writes in global memory is 64 bytes; a row workgroup
// twice the rows.
constexpr int kTpbRows = 512, kTpbCols = 512;

template <int L_, int NL_, int LP_, int F1, int F2, int F3, int F4, int F5, int F6, int TPB_>
struct Plan {
    static constexpr int L = L_, NL = NL_, LP = LP_, TPB = TPB_;
    static constexpr int G = (F1 > 1) + (F2 > 1) + (F3 > 1) + (F4 > 1) + (F5 > 1) + (F6 > 1);
    static constexpr int Fg(int g) {
        return g == 0 ? F1 : g == 1 ? F2 : g == 2 ? F3 : g == 3 ? F4 : g == 4 ? F5 : F6;
    }
    static constexpr int Pg(int g) { return g == 0 ? 1 : Pg(g - 1) * Fg(g - 1); }  // product of earlier radices
    static constexpr int Qg(int g) { return L / Fg(g); }
    static constexpr int Rg(int g) { return (NL * Qg(g) + TPB - 1) / TPB; }
    // Twiddle rows in LDS: a middle group g has one row per k < p_g holding
    // W_L^(j k Q_g / p_g) for j = 1 .. F_g - 1; the last group one row per
    // butterfly i holding (-1)^i W_L^(i j) for j = 0 .. F - 1 (the sign is
    // the half-line rotation of its outputs).  Row strides are odd, so that
    // the rows of neighbouring lanes start in different banks.
    static constexpr int Wg(int g) { return g == G - 1 ? Fg(g) : Fg(g) - 1; }  // entries per row
    static constexpr int Sg(int g) { return Wg(g) % 2 == 1 ? Wg(g) : Wg(g) + 1; }
    static constexpr int Og(int g) { return g <= 1 ? 0 : Og(g - 1) + Pg(g - 1) * Sg(g - 1); }  // row block offset
    static constexpr int TW = Og(G);
    static constexpr size_t lds_bytes() { return (size_t)(NL * LP + TW) * sizeof(float2); }
    static constexpr int kF[6] = {F1, F2, F3, F4, F5, F6};
    static_assert(lds_bytes() == plan_lds_bytes(NL, LP, kF), "host and device plan sizes differ");
    static_assert(F1 * F2 * F3 * F4 * F5 * F6 == L, "radices do not multiply to L");
    static_assert(L % 2 == 0 && G >= 2 && LP >= L, "bad plan");
};

// Butterfly b of group g: its line l and its index i (i < Q_g and l < NL for
// b < NL Q_g, which every caller tests first: the round's last lanes may lie
// past the work).  Along the line (consecutive butterflies, consecutive
// positions); or across the NL lines first (columns: neighbouring columns in
// global memory), NL a power of two.
template <class P, bool ACROSS, int g>
__device__ __forceinline__ void decode(unsigned b, unsigned &l, unsigned &i) {
    constexpr unsigned Q = P::Qg(g);
    if constexpr (ACROSS) {
        l = b % (unsigned)P::NL;
        i = b / (unsigned)P::NL;
    } else {
        l = b / Q;
        i = b - l * Q;
    }
}

// Per-workgroup view of its lines in global memory.
struct Lines {
    const float2 *in;   // first input element of line 0
    float2 *out;        // first output element of line 0
    long long in_ls, out_ls, es;  // line strides (input, output), element stride along a line
    int nvalid;         // lines of this workgroup that exist
};

// Group 0: butterfly i of a line takes the stored elements i + j Q (the
// natural transform index: the half-line rotation of the modes is applied to
// the outputs instead).  Every round's points are loaded before any is used,
// so that all the loads are in flight together.
template <class P, bool COLS>
__device__ __forceinline__ void load_first(unsigned tid, const Lines &ln, float2 (*xin)[P::Fg(0)]) {
    constexpr int F = P::Fg(0), Q = P::Qg(0), R = P::Rg(0);
    sfor<R>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        sfor<F>([&](auto jc) { xin[r][decltype(jc)::value] = c2(0.f, 0.f); });
        const unsigned b = tid + P::TPB * r;
        if ((r + 1) * P::TPB <= P::NL * Q || b < (unsigned)(P::NL * Q)) {
            unsigned l, i;
            decode<P, COLS, 0>(b, l, i);
            if ((int)l < ln.nvalid) {
                const float2 *src = ln.in + (long long)l * ln.in_ls + (long long)i * ln.es;
                const long long js = (long long)Q * ln.es;
                sfor<F>([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    xin[r][j] = src[j * js];
                });
            }
        }
    });
}

// For the odd phase the points are multiplied by W_2L^(i + j Q) =
// W_2L^i W_2F^j and by -i (the odd outputs' factor, by linearity); the
// F-point DFT goes to positions i F + j' of the line.
template <class P, bool COLS>
__device__ __forceinline__ void group_first(unsigned tid, int par, const float2 (*xin)[P::Fg(0)],
                                            const float2 *tw2, float2 *lines) {
    constexpr int F = P::Fg(0), Q = P::Qg(0), R = P::Rg(0);
    sfor<R>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        const unsigned b = tid + P::TPB * r;
        if ((r + 1) * P::TPB <= P::NL * Q || b < (unsigned)(P::NL * Q)) {
            unsigned l, i;
            decode<P, COLS, 0>(b, l, i);
            float2 x[F];
            sfor<F>([&](auto jc) { x[decltype(jc)::value] = xin[r][decltype(jc)::value]; });
            if (par) {
                const float2 w = tw2[i];
                const float2 wi = c2(w.y, -w.x);  // -i W_2L^i
                sfor<F>([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    x[j] = twc<2 * F, j>(mul(x[j], wi));
                });
            }
            Dft<F>::run(x);
            float2 *dst = lines + l * P::LP + i * F;
            sfor<F>([&](auto jc) { dst[decltype(jc)::value] = x[decltype(jc)::value]; });
        }
    });
}

// Middle group g: every round's inputs are read before the barrier, then each
// butterfly (k = i mod p) multiplies input j by its row entry W_L^(j k Q/p),
// transforms, and writes output j' to (i div p) p F + k + j' p.
template <class P, int g>
__device__ __forceinline__ void group_mid(unsigned tid, float2 *lines, const float2 *tw) {
    constexpr int F = P::Fg(g), Q = P::Qg(g), R = P::Rg(g), p = P::Pg(g);
    float2 x[R][F];
    sfor<R>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        const unsigned b = tid + P::TPB * r;
        if ((r + 1) * P::TPB <= P::NL * Q || b < (unsigned)(P::NL * Q)) {
            unsigned l, i;
            decode<P, false, g>(b, l, i);
            const float2 *src = lines + l * P::LP + i;
            sfor<F>([&](auto jc) { x[r][decltype(jc)::value] = src[decltype(jc)::value * Q]; });
        }
    });
    __syncthreads();  // every input read before any position is overwritten
    sfor<R>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        const unsigned b = tid + P::TPB * r;
        if ((r + 1) * P::TPB <= P::NL * Q || b < (unsigned)(P::NL * Q)) {
            unsigned l, i;
            decode<P, false, g>(b, l, i);
            const unsigned hq = i / (unsigned)p, k = i - hq * p;
            const float2 *row = tw + P::Og(g) + k * P::Sg(g);
            sfor<F - 1>([&](auto jc) {
                constexpr int j = decltype(jc)::value + 1;
                x[r][j] = mul(x[r][j], row[j - 1]);
            });
            Dft<F>::run(x[r]);
            float2 *dst = lines + l * P::LP + hq * (p * F) + k;
            sfor<F>([&](auto jc) { dst[decltype(jc)::value * p] = x[r][decltype(jc)::value]; });
        }
    });
    __syncthreads();
}

// Last group (p F = L, so p = Q and k = i): outputs X[i + j' Q].  The row
// carries (-1)^i; for odd Q the remaining sign (-1)^(j' Q) = (-1)^j' is a
// shift of the F (even) inputs by F/2.  Output k >= L/2 stands for k - L.
// The even phase keeps its outputs in registers; the odd phase, whose
// butterflies are the same, stores both: p = 2k and 2k + 1 side by side (the
// two parities of a line are written together, so that no cache line is
// left half written between the phases), each only inside [-P, P].
template <class P, bool COLS>
__device__ __forceinline__ void group_last(unsigned tid, int par, int Pa, const Lines &ln, const float2 *lines,
                                           const float2 *tw, float2 (*keep)[P::Fg(P::G - 1)]) {
    constexpr int g = P::G - 1;
    constexpr int F = P::Fg(g), Q = P::Qg(g), R = P::Rg(g), L = P::L;
    static_assert(P::Pg(g) == Q, "last group");
    sfor<R>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        const unsigned b = tid + P::TPB * r;
        if ((r + 1) * P::TPB <= P::NL * Q || b < (unsigned)(P::NL * Q)) {
            unsigned l, i;
            decode<P, COLS, g>(b, l, i);
            __builtin_assume(i < (unsigned)Q);  // b < NL Q here
            const float2 *src = lines + l * P::LP + i;
            const float2 *row = tw + P::Og(g) + i * P::Sg(g);
            float2 x[F];
            sfor<F>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                constexpr int js = Q % 2 == 1 ? (j + F / 2) % F : j;
                x[js] = mul(src[j * Q], row[j]);
            });
            Dft<F>::run(x);
            if (par == 0) {
                sfor<F>([&](auto jc) { keep[r][decltype(jc)::value] = x[decltype(jc)::value]; });
            } else if ((int)l < ln.nvalid) {
                float2 *dst = ln.out + (long long)l * ln.out_ls + (long long)(2 * (int)i + Pa) * ln.es;
                const int ii = (int)i;
                sfor<F>([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    // k = i + j Q; k >= L/2 is decided by j alone unless F is odd
                    // and j = (F - 1) / 2 (then by i >= Q/2)
                    constexpr bool lo = 2 * (j * Q + Q) <= L, hi = 2 * j * Q >= L;
                    const bool up = hi || (!lo && 2 * ii >= Q);
                    const int off = 2 * j * Q - (up ? 2 * L : 0);  // p_even - 2 i
                    const int pe = 2 * ii + off;
                    if (up ? pe >= -Pa : pe <= Pa) dst[(long long)off * ln.es] = keep[r][j];
                    if (up ? pe + 1 >= -Pa : pe + 1 <= Pa) dst[(long long)(off + 1) * ln.es] = x[j];
                });
            }
        }
    });
}

template <class P, int g>
__device__ __forceinline__ void middle_groups(unsigned tid, float2 *lines, const float2 *tw) {
    if constexpr (g < P::G - 1) {
        group_mid<P, g>(tid, lines, tw);
        middle_groups<P, g + 1>(tid, lines, tw);
    }
}

// Twiddle rows (see Plan), from the W_2L table in global memory.
template <class P, int g>
__device__ __forceinline__ void fill_rows(float2 *tw, const float2 *tw2) {
    if constexpr (g < P::G) {
        constexpr int S = P::Sg(g), W = P::Wg(g), n = P::Pg(g) * S, step = P::Qg(g) / P::Pg(g);
        for (unsigned e = threadIdx.x; e < (unsigned)n; e += P::TPB) {
            const unsigned k = e / (unsigned)S, c = e - k * S;
            float2 v = c2(0.f, 0.f);
            if (g == P::G - 1) {
                if (c < (unsigned)W) {
                    v = tw2[2 * (k * c)];  // k < Q, c < F: k c < L
                    if (k & 1) v = c2(-v.x, -v.y);
                }
            } else if (c < (unsigned)W) {
                v = tw2[2 * ((c + 1) * k * step)];  // (c + 1) k Q / p < L
            }
            tw[P::Og(g) + e] = v;
        }
        fill_rows<P, g + 1>(tw, tw2);
    }
}

// The pass for one workgroup: rows (x) take NL consecutive rows of one
// snapshot; columns (y, z) NL consecutive columns of one slow index.
template <class P, bool COLS>
__device__ __forceinline__ void run_plan(const SnapDev &S, int a, long long wl, cplx<float> *grid, char *smem) {
    constexpr int L = P::L, NL = P::NL;
    const int Ma = S.M[a], Pa = S.P[a];
    long long FC = 1, Sl = 1;
    for (int b = 0; b < a; ++b) FC *= S.M[b];
    for (int b = a + 1; b < S.dim; ++b) Sl *= S.n1[b];
    const bool fromA = (a % 2) == 0;
    Lines ln;
    ln.in = grid + (fromA ? S.bufA : S.bufB);
    ln.out = grid + (fromA ? S.bufB : S.bufA);
    if constexpr (COLS) {
        const long long ngrp = (FC + NL - 1) / NL;
        const long long o = wl / ngrp, i0 = (wl - o * ngrp) * NL;
        if (o >= Sl) return;
        ln.in += o * ((long long)L * FC) + i0;
        ln.out += o * ((long long)Ma * FC) + i0;
        ln.in_ls = ln.out_ls = 1;
        ln.es = FC;
        ln.nvalid = (int)min((long long)NL, FC - i0);
    } else {
        const long long r0 = wl * NL;
        if (r0 >= Sl) return;
        ln.in += r0 * (long long)L;
        ln.out += r0 * (long long)Ma;
        ln.in_ls = L;
        ln.out_ls = Ma;
        ln.es = 1;
        ln.nvalid = (int)min((long long)NL, Sl - r0);
    }
    float2 *lines = (float2 *)smem;
    float2 *tw = lines + NL * P::LP;
    const float2 *tw2 = (const float2 *)S.tw[a];  // W_2L^e, e < 2L
    float2 keep[P::Rg(P::G - 1)][P::Fg(P::G - 1)];
    fill_rows<P, 1>(tw, tw2);
#pragma unroll 1
    for (int par = 0; par < 2; ++par) {
        // formed inside the phase: hoisted out of this loop, the addresses of
        // every group would all stay live in registers
        unsigned tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        __builtin_assume(tid < (unsigned)P::TPB);
        // every round's loads in flight at once (the second phase reads the
        // same lines again, from cache)
        float2 xin[P::Rg(0)][P::Fg(0)];
        load_first<P, COLS>(tid, ln, xin);
        __syncthreads();  // rows written (first phase); the last group's reads done (second)
        group_first<P, COLS>(tid, par, xin, tw2, lines);
        __syncthreads();
        middle_groups<P, 1>(tid, lines, tw);
        group_last<P, COLS>(tid, par, Pa, ln, lines, tw, keep);
    }
}

}  // namespace fftr
}  // namespace fv
