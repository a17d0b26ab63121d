// Host-side planning of the type-3 transform (paper section 2.2: kernel width
// from eps, the grid-size equation, centring of both point sets) and the
// choice of dimension and precision.
//
// Host code here is compiled with -ffp-contract=off so that every grid size is
// the exact IEEE result of the documented expression.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "fv_internal.h"

namespace fv {

int kernel_width(double eps) {
    // paper rule ceil(log10(1/eps)) + 1, plus one point (the rule alone lands
    // at about eps, not below it)
    int w = (int)std::ceil(-std::log10(eps) - 1e-9) + 2;
    return std::max(2, std::min(kMaxW, w));
}

int kernel_width_type1(double eps) {
    // the paper's rule ceil(log10(1/eps)) + 1: type 1 applies the kernel once
    // (one spread, no interpolation), so the rule's error stays below eps
    const int w = (int)std::ceil(-std::log10(eps) - 1e-9) + 1;
    return std::max(3, std::min(kMaxW, w));
}

// Even numbers whose only prime factors are 2, 3 and 5, up to 2^31, sorted
// (about 1.5k of them), built once.
static const std::vector<long long> &smooth_even_table() {
    static const std::vector<long long> t = [] {
        std::vector<long long> v;
        const long long lim = 1LL << 31;
        for (long long a = 2; a <= lim; a *= 2)
            for (long long b = a; b <= lim; b *= 3)
                for (long long c = b; c <= lim; c *= 5) v.push_back(c);
        std::sort(v.begin(), v.end());
        return v;
    }();
    return t;
}

int next_smooth_even(long long n) {
    if (n < 2) n = 2;
    const auto &t = smooth_even_table();
    auto it = std::lower_bound(t.begin(), t.end(), n);
    if (it == t.end()) fail(FV_EUNSUPPORTED, "grid size beyond 2^31");
    return (int)*it;
}

void src_box(const double *src, int n_src, int dim, double *s_c, double *S) {
    for (int a = 0; a < 3; ++a) { s_c[a] = 0; S[a] = 0; }
    if (n_src <= 0) return;
    for (int a = 0; a < dim; ++a) {
        double lo = src[a], hi = src[a];
        for (int j = 1; j < n_src; ++j) {
            double v = src[3 * (size_t)j + a];
            lo = std::min(lo, v);
            hi = std::max(hi, v);
        }
        s_c[a] = 0.5 * (lo + hi);
        S[a] = 0.5 * (hi - lo);
    }
}

// Reflect b into the half-space b[axis] >= 0, zeros decided by the remaining
// axes in increasing order.  Real strengths give V(-b) = conj V(b).
void fold_baseline(const double *b, int dim, int axis, double *out, bool *flipped) {
    bool flip = false;
    if (axis >= 0) {
        int order[3] = {axis, 0, 0};
        int k = 1;
        for (int a = 0; a < dim; ++a)
            if (a != axis) order[k++] = a;
        for (int t = 0; t < dim; ++t) {
            double v = b[order[t]];
            if (v < 0) { flip = true; break; }
            if (v > 0) break;
        }
    }
    for (int a = 0; a < dim; ++a) out[a] = flip ? -b[a] : b[a];
    for (int a = dim; a < 3; ++a) out[a] = 0.0;
    *flipped = flip;
}

GeomPlan plan_geometry(const double *ant, int n_ant, int dim, double eps, const double *s_c, const double *S,
                       bool fold) {
    GeomPlan g;
    g.dim = dim;
    g.w = kernel_width(eps);
    g.n_ant = n_ant;
    g.n_pairs = (long long)n_ant * (n_ant + 1) / 2;
    for (int a = 0; a < 3; ++a) { g.s_c[a] = s_c[a]; g.S[a] = S[a]; }
    // unfolded extents pick the reflection axis (largest extent times S)
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) { lo[a] = std::numeric_limits<double>::infinity(); hi[a] = -lo[a]; }
    for (int i = 0; i < n_ant; ++i)
        for (int j = i; j < n_ant; ++j)
            for (int a = 0; a < dim; ++a) {
                double b = ant[3 * (size_t)i + a] - ant[3 * (size_t)j + a];
                lo[a] = std::min(lo[a], b);
                hi[a] = std::max(hi[a], b);
            }
    g.fold_axis = -1;
    if (fold) {
        double best = -1.0;
        for (int a = 0; a < dim; ++a) {
            double v = (hi[a] - lo[a]) * std::max(S[a], 1e-300);
            if (v > best) { best = v; g.fold_axis = a; }
        }
        for (int a = 0; a < 3; ++a) { lo[a] = std::numeric_limits<double>::infinity(); hi[a] = -lo[a]; }
        for (int i = 0; i < n_ant; ++i)
            for (int j = i; j < n_ant; ++j) {
                double b[3], f[3];
                bool fl;
                for (int a = 0; a < 3; ++a) b[a] = ant[3 * (size_t)i + a] - ant[3 * (size_t)j + a];
                fold_baseline(b, dim, g.fold_axis, f, &fl);
                for (int a = 0; a < dim; ++a) { lo[a] = std::min(lo[a], f[a]); hi[a] = std::max(hi[a], f[a]); }
            }
    }
    for (int a = 0; a < dim; ++a) {
        g.b_c[a] = 0.5 * (lo[a] + hi[a]);
        g.B[a] = 0.5 * (hi[a] - lo[a]);
    }
    return g;
}

SnapPlan plan_snapshot(const GeomPlan &g, double nu) {
    SnapPlan p;
    p.dim = g.dim;
    p.w = g.w;
    p.fold_axis = g.fold_axis;
    p.nu = nu;
    p.k = 2.0 * M_PI * nu / kCLight;
    for (int a = 0; a < 3; ++a) {
        p.s_c[a] = g.s_c[a];
        p.S[a] = g.S[a];
        p.b_c[a] = g.b_c[a];
        p.B[a] = g.B[a];
    }
    const int P0 = g.w / 2 + 1;
    for (int a = 0; a < g.dim; ++a) {
        double kB = p.k * g.B[a];
        double X = std::max(kB, 1.0);
        if (!(kB >= 1.0)) p.degenerate |= 1 << a;
        double Se = std::max(g.S[a], 1.0 / X);
        double v = 2.0 * kSigma / M_PI * X * Se + (double)g.w;
        p.X[a] = X;
        p.n1[a] = next_smooth_even((long long)std::ceil(v));
        p.n2[a] = (int)(kSigma * p.n1[a]);
        p.P[a] = p.n1[a] / 2 + P0;
        p.M[a] = 2 * p.P[a] + 1;
    }
    return p;
}

// Gauss-Legendre nodes on [-1, 1] by Newton iteration on P_n from the
// Chebyshev-like initial guesses (textbook construction).
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                // one more evaluation of the derivative at the converged node
                p0 = 1.0; p1 = z;
                for (int k = 2; k <= n; ++k) {
                    double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (z * p1 - p0) / (z * z - 1.0);
                break;
            }
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

int choose_dim(const double *ant, int n_ant, double eps, const double *freq, int n_freq, unsigned flags) {
    unsigned d = flags & FV_DIM_MASK;
    if (d == FV_DIM_2D) return 2;
    if (d == FV_DIM_3D) return 3;
    double zlo = ant[2], zhi = ant[2];
    for (int i = 1; i < n_ant; ++i) {
        zlo = std::min(zlo, ant[3 * (size_t)i + 2]);
        zhi = std::max(zhi, ant[3 * (size_t)i + 2]);
    }
    double numax = 0.0;
    for (int f = 0; f < n_freq; ++f) numax = std::max(numax, freq[f]);
    // dropped phase 2 pi nu dz n / c must stay below eps / 10
    double tol = eps * kCLight / (20.0 * M_PI * numax);
    return (zhi - zlo) <= tol ? 2 : 3;
}

int choose_prec(double eps, unsigned flags) {
    unsigned p = flags & FV_PREC_MASK;
    if (p == FV_PREC_FP32) return 32;
    if (p == FV_PREC_FP64) return 64;
    return eps >= 1e-6 ? 32 : 64;
}

}  // namespace fv

namespace fv {

// Quadrature table for phihat with kernel width w (beta = 2.3 w):
// out[q] = sin(theta_q), out[kQuadHalf + q] = 2 * (pi/2) wgl_q exp(beta (cos theta_q - 1)) cos theta_q
// over the positive nodes theta_q = (pi/2) x_q of the 64-point rule (the
// integrand is even in theta, so each positive node stands for its mirror).
void quad_table(int w, double *out) {
    std::vector<double> x, wt;
    gauss_legendre(2 * kQuadHalf, x, wt);
    const double beta = 2.3 * w;
    for (int q = 0; q < kQuadHalf; ++q) {
        double xq = x[kQuadHalf + q];
        double t = 0.5 * M_PI * xq;
        out[q] = std::sin(t);
        out[kQuadHalf + q] = 2.0 * 0.5 * M_PI * wt[kQuadHalf + q] * std::exp(beta * (std::cos(t) - 1.0)) * std::cos(t);
    }
}

static uint64_t spread_bits16(uint64_t v) {
    v &= 0xffff;
    v = (v | (v << 8)) & 0x00ff00ffull;
    v = (v | (v << 4)) & 0x0f0f0f0full;
    v = (v | (v << 2)) & 0x33333333ull;
    v = (v | (v << 1)) & 0x55555555ull;
    return v;
}

std::vector<int> target_order(const double *ant, const GeomPlan &g) {
    const int n_ant = g.n_ant, dim = g.dim;
    const long long n = g.n_pairs;
    std::vector<std::pair<uint64_t, int>> key((size_t)n);
    auto q = [](double x, double lo, double half, int bits) {
        const double u = half > 0 ? (x - lo) / (2.0 * half) : 0.5;
        const double m = (double)((1u << bits) - 1);
        return (uint64_t)std::min(m, std::max(0.0, std::floor(u * m)));
    };
    long long p = 0;
    for (int i = 0; i < n_ant; ++i)
        for (int j = i; j < n_ant; ++j, ++p) {
            double b[3], f[3];
            bool fl;
            for (int a = 0; a < 3; ++a) b[a] = ant[3 * (size_t)i + a] - ant[3 * (size_t)j + a];
            fold_baseline(b, dim, g.fold_axis, f, &fl);
            uint64_t k = spread_bits16(q(f[0], g.b_c[0] - g.B[0], g.B[0], 16)) |
                         (spread_bits16(q(f[1], g.b_c[1] - g.B[1], g.B[1], 16)) << 1);
            if (dim == 3) k = (k << 8) | q(f[2], g.b_c[2] - g.B[2], g.B[2], 8);
            key[(size_t)p] = {k, (int)p};
        }
    std::sort(key.begin(), key.end());
    std::vector<int> perm((size_t)n);
    for (long long t = 0; t < n; ++t) perm[(size_t)t] = key[(size_t)t].second;
    return perm;
}

bool find_lattice(const double *ant, int n_ant, double tol, LatticePlan *lp) {
    if (n_ant < 2) return false;
    // shortest baseline, then the shortest one not parallel to it
    double b1[2] = {0, 0}, l1 = std::numeric_limits<double>::infinity();
    for (int i = 0; i < n_ant; ++i)
        for (int j = i + 1; j < n_ant; ++j) {
            const double dx = ant[3 * (size_t)i] - ant[3 * (size_t)j], dy = ant[3 * (size_t)i + 1] - ant[3 * (size_t)j + 1];
            const double l = std::hypot(dx, dy);
            if (l > tol && l < l1) {
                l1 = l;
                b1[0] = dx;
                b1[1] = dy;
            }
        }
    if (!std::isfinite(l1)) return false;
    double b2[2] = {0, 0}, l2 = std::numeric_limits<double>::infinity();
    for (int i = 0; i < n_ant; ++i)
        for (int j = i + 1; j < n_ant; ++j) {
            const double dx = ant[3 * (size_t)i] - ant[3 * (size_t)j], dy = ant[3 * (size_t)i + 1] - ant[3 * (size_t)j + 1];
            const double l = std::hypot(dx, dy);
            if (l <= tol || l >= l2) continue;
            if (std::fabs(b1[0] * dy - b1[1] * dx) > 1e-6 * l1 * l) {
                l2 = l;
                b2[0] = dx;
                b2[1] = dy;
            }
        }
    if (!std::isfinite(l2)) return false;  // collinear
    // Gauss reduction
    for (int it = 0; it < 64; ++it) {
        double n1 = b1[0] * b1[0] + b1[1] * b1[1], n2 = b2[0] * b2[0] + b2[1] * b2[1];
        if (n2 < n1) {
            std::swap(b1[0], b2[0]);
            std::swap(b1[1], b2[1]);
            std::swap(n1, n2);
        }
        const double mu = std::nearbyint((b1[0] * b2[0] + b1[1] * b2[1]) / n1);
        if (mu == 0.0) break;
        b2[0] -= mu * b1[0];
        b2[1] -= mu * b1[1];
    }
    const double det = b1[0] * b2[1] - b1[1] * b2[0];
    if (!(std::fabs(det) > 0)) return false;
    lp->A[0][0] = b1[0];
    lp->A[1][0] = b1[1];
    lp->A[0][1] = b2[0];
    lp->A[1][1] = b2[1];
    lp->k.assign(2 * (size_t)n_ant, 0);
    int lo[2] = {0, 0}, hi[2] = {0, 0};
    for (int i = 0; i < n_ant; ++i) {
        const double dx = ant[3 * (size_t)i] - ant[0], dy = ant[3 * (size_t)i + 1] - ant[1];
        // solve A k = d (2 x 2, Cramer), round, check
        const double k0 = (dx * b2[1] - dy * b2[0]) / det, k1 = (b1[0] * dy - b1[1] * dx) / det;
        const double r0 = std::nearbyint(k0), r1 = std::nearbyint(k1);
        const double ex = r0 * b1[0] + r1 * b2[0] - dx, ey = r0 * b1[1] + r1 * b2[1] - dy;
        if (std::hypot(ex, ey) > tol || std::fabs(r0) > 1e6 || std::fabs(r1) > 1e6) return false;
        lp->k[2 * (size_t)i] = (int)r0;
        lp->k[2 * (size_t)i + 1] = (int)r1;
        for (int a = 0; a < 2; ++a) {
            lo[a] = std::min(lo[a], lp->k[2 * (size_t)i + a]);
            hi[a] = std::max(hi[a], lp->k[2 * (size_t)i + a]);
        }
    }
    lp->K[0] = hi[0] - lo[0];
    lp->K[1] = hi[1] - lo[1];
    return true;
}

// Piece i of the kernel of width w interpolated at the n = w + 3 Chebyshev
// nodes of u, then turned from a Chebyshev series into monomial coefficients.
// The fit's largest error is about exp(-beta): the kernel's square-root edge
// at |z| = 1 bounds any polynomial there.
static void es_poly_piece(int w, int i, float *out /* [w + 3] */) {
    const int n = w + 3;
    const double beta = 2.3 * w;
    std::vector<double> y(n), mono(n, 0.0), tprev(n, 0.0), tcur(n, 0.0);
    for (int j = 0; j < n; ++j) {
        const double u = std::cos(M_PI * (j + 0.5) / n), t = 0.5 * (u + 1.0);
        const double z = (i + 1 - 0.5 * w - t) * 2.0 / w, z2 = z * z;
        y[j] = z2 <= 1.0 ? std::exp(-beta * z2 / (1.0 + std::sqrt(1.0 - z2))) : 0.0;
    }
    // T_0 = 1, T_1 = u, T_{k+1} = 2 u T_k - T_{k-1}, as monomial coefficients
    tcur[0] = 1.0;
    for (int k = 0; k < n; ++k) {
        double ak = 0.0;  // Chebyshev coefficient k of the interpolant
        for (int j = 0; j < n; ++j) ak += y[j] * std::cos(M_PI * k * (j + 0.5) / n);
        ak *= (k == 0 ? 1.0 : 2.0) / n;
        for (int m = 0; m < n; ++m) mono[m] += ak * tcur[m];
        std::vector<double> next(n, 0.0);
        for (int m = 0; m + 1 < n; ++m) next[m + 1] = (k == 0 ? 1.0 : 2.0) * tcur[m];
        if (k > 0)
            for (int m = 0; m < n; ++m) next[m] -= tprev[m];
        tprev = tcur;
        tcur = next;
    }
    for (int m = 0; m < n; ++m) out[m] = (float)mono[m];
}

const EsPoly &es_poly(int w) {
    static const std::vector<EsPoly> tab = [] {
        std::vector<EsPoly> t(kPolyMaxW + 1);
        for (int w = 0; w <= kPolyMaxW; ++w) {
            std::memset(&t[w], 0, sizeof(EsPoly));
            if (w >= 2)
                for (int i = 0; i < (w + 1) / 2; ++i) es_poly_piece(w, i, t[w].c[i]);
        }
        return t;
    }();
    static const EsPoly zero = [] {
        EsPoly z;
        std::memset(&z, 0, sizeof(z));
        return z;
    }();
    return w >= 0 && w <= kPolyMaxW ? tab[w] : zero;
}

double phihat_host(double xi, const double *q) {
    double acc = 0.0;
    for (int i = 0; i < kQuadHalf; ++i) acc += q[kQuadHalf + i] * std::cos(xi * q[i]);
    return acc;
}

}  // namespace fv
