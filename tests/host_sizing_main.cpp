// Host checks of the library's sizing and planning helpers (no GPU), built
// with the address and undefined-behaviour sanitizers by
// tests/test_host_sizing.py.  Degenerate cases: an empty sky, one source, one
// antenna, one time, one frequency, zero and tiny HBM budgets.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <stdexcept>
#include <vector>

#include "fv_internal.h"

namespace fv {
// the runtime's error path (runtime.cpp is not linked here)
[[noreturn]] void fail(fv_status code, const std::string &msg) { throw Error{code, msg}; }
// lattice.hip frees a plan's device tables; the plans here never get any
LatticePlan::~LatticePlan() {
    if (dev) std::abort();
}
}  // namespace fv

using namespace fv;

static int g_fail = 0;
#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "%s:%d: CHECK failed: %s\n", __FILE__, __LINE__, #cond); \
            ++g_fail;                                                            \
        }                                                                        \
    } while (0)

static bool smooth5(long long n) {
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

static std::vector<double> hex7() {
    const double s = 14.6;
    std::vector<double> a = {0, 0, 0};
    for (int k = 0; k < 6; ++k) {
        const double t = k * M_PI / 3;
        a.insert(a.end(), {s * std::cos(t), s * std::sin(t), 0.0});
    }
    return a;
}

static void check_plan(const SnapPlan &p) {
    for (int a = 0; a < p.dim; ++a) {
        CHECK(p.n1[a] >= p.w);
        CHECK(p.n1[a] % 2 == 0 && smooth5(p.n1[a]));
        CHECK(p.n2[a] == 2 * p.n1[a]);
        CHECK(p.P[a] == p.n1[a] / 2 + p.w / 2 + 1);
        CHECK(p.M[a] == 2 * p.P[a] + 1);
        CHECK(std::isfinite(p.X[a]) && p.X[a] >= 1.0);
    }
}

int main() {
    // ---- drift scans: the grouping of times never divides by zero and fits
    for (int n_src : {0, 1, 1000, 100000})
        for (int n_freq : {1, 64})
            for (int n_time : {1, 5, 100000})
                for (size_t budget : {(size_t)0, (size_t)1 << 20, (size_t)200 << 30}) {
                    const DriftSizing z = drift_sizing(1, n_src, n_freq, n_time, budget);
                    CHECK(z.per_time >= 256);
                    CHECK(z.group >= 1 && z.group <= std::min(n_time, 65535));
                    CHECK(z.fixed + (size_t)z.group * z.per_time <= std::max(budget / 4, z.per_time + z.fixed) ||
                          z.group == 1);
                }
    CHECK(frontend_blocks(0) == 0 && frontend_blocks(1) == 1 && frontend_blocks(kFeBlock + 1) == 2);

    // ---- geometry and snapshot plans
    const std::vector<double> one = {3.0, -2.0, 0.0};
    const std::vector<double> h7 = hex7();
    const double zero3[3] = {0, 0, 0};
    const double sbox[3] = {0.1, -0.2, 0.5}, Sbox[3] = {0.9, 0.8, 0.4};
    for (int dim : {2, 3})
        for (double eps : {1e-4, 1e-6, 1e-10}) {
            // one antenna: autos only, the extent clamps (degenerate axes)
            GeomPlan g1 = plan_geometry(one.data(), 1, dim, eps, sbox, Sbox, true);
            CHECK(g1.n_pairs == 1);
            SnapPlan p1 = plan_snapshot(g1, 150e6);
            check_plan(p1);
            CHECK(p1.degenerate == (dim == 2 ? 3 : 7));
            // one source (zero box) on a real array
            GeomPlan g2 = plan_geometry(h7.data(), 7, dim, eps, sbox, zero3, true);
            for (double nu : {50e6, 150e6, 250e6}) check_plan(plan_snapshot(g2, nu));
            // an ordinary box
            GeomPlan g3 = plan_geometry(h7.data(), 7, dim, eps, sbox, Sbox, false);
            CHECK(g3.fold_axis == -1);
            check_plan(plan_snapshot(g3, 150e6));
        }
    CHECK(choose_dim(one.data(), 1, 1e-6, (const double[]){150e6}, 1, 0) == 2);
    CHECK(choose_prec(1e-6, 0) == 32 && choose_prec(1e-7, 0) == 64);
    CHECK(kernel_width(1e-6) == 8);
    for (long long n : {1LL, 2LL, 7LL, 97LL, 1501LL, 4099LL}) {
        const int m = next_smooth_even(n);
        CHECK(m >= n && m % 2 == 0 && smooth5(m));
    }

    // ---- lattice detection on the degenerate arrays
    LatticePlan lp;
    CHECK(!find_lattice(one.data(), 1, 1e-3, &lp));
    const std::vector<double> two = {0, 0, 0, 14.6, 0, 0};
    CHECK(!find_lattice(two.data(), 2, 1e-3, &lp));  // collinear
    CHECK(find_lattice(h7.data(), 7, 1e-3, &lp));

    // ---- type-3 workspace of launch groups with an empty sky, one source,
    // one antenna; deterministic mode adds its buffers
    TargetTable tt;
    for (int dim : {2, 3}) {
        GeomPlan g = plan_geometry(h7.data(), 7, dim, 1e-6, sbox, Sbox, true);
        tt.n_tgt = g.n_pairs;
        tt.dim = dim;
        for (int n_src : {0, 1, 5000}) {
            std::vector<SnapJob> jobs;
            for (double nu : {100e6, 200e6}) {
                SnapJob j;
                j.plan = plan_snapshot(g, nu);
                j.n_src = n_src;
                j.src = nullptr;
                j.tt = &tt;
                jobs.push_back(j);
            }
            const size_t b = nufft_workspace_bytes(jobs, dim, 32, g.w, false);
            const size_t bd = nufft_workspace_bytes(jobs, dim, 32, g.w, true);
            CHECK(b > 0 && bd >= b);
            CHECK(n_src == 0 || bd > b);
            const size_t b64 = nufft_workspace_bytes(jobs, dim, 64, g.w, false);
            CHECK(b64 > b);
        }
        GeomPlan g1 = plan_geometry(one.data(), 1, dim, 1e-6, sbox, Sbox, true);
        tt.n_tgt = 1;
        SnapJob j;
        j.plan = plan_snapshot(g1, 150e6);
        j.n_src = 1;
        j.tt = &tt;
        CHECK(nufft_workspace_bytes(std::vector<SnapJob>{j}, dim, 32, g1.w, false) > 0);
    }

    // ---- request footprints
    {
        GeomPlan g = plan_geometry(h7.data(), 7, 2, 1e-6, sbox, Sbox, true);
        const double freq[3] = {100e6, 150e6, 200e6};
        fv_problem p{};
        p.n_ant = 7;
        p.ant_enu = h7.data();
        p.n_freq = 3;
        p.freq_hz = freq;
        p.eps = 1e-6;
        p.n_src = 0;
        const size_t base0 = footprint_bytes(p, g, 2, 32, 1 << 20);
        CHECK(base0 == 24 * 7 + 16 * 28 * 3);
        p.n_src = 1;
        const size_t f1 = footprint_bytes(p, g, 2, 32, 1 << 20);
        CHECK(f1 > base0);
        p.n_src = 100000;
        const size_t fbig = footprint_bytes(p, g, 2, 32, 1 << 20);
        p.flags = FV_METHOD_DIRECT;
        const size_t fdirect = footprint_bytes(p, g, 2, 32, 1 << 20);
        CHECK(fdirect < fbig);
        p.flags = FV_METHOD_MFMA;  // the direct sum's inputs plus the Z chunk and partial tiles
        CHECK(footprint_bytes(p, g, 2, 32, 1 << 20) == fdirect + zz_work_bytes(7, 100000, 32, 1 << 20));
        p.n_ant = 1;
        p.ant_enu = one.data();
        GeomPlan g1 = plan_geometry(one.data(), 1, 2, 1e-6, sbox, Sbox, true);
        p.flags = 0;
        CHECK(footprint_bytes(p, g1, 2, 32, 1 << 20) > 0);
    }

    // ---- matrix-core chunking: degenerate sizes, and the chunk fits the cap
    for (int n_ant : {1, 37, 350})
        for (int n_src : {0, 1, 100000})
            for (int prec : {32, 64}) {
                const size_t cap = (size_t)64 << 20;
                const ZZShape s = zz_shape(n_ant, n_src, prec, cap);
                CHECK(s.kc_pad >= 4 && s.kc_pad % 4 == 0);
                CHECK(s.nsplit >= kWavesPerBlock && s.nsplit % kWavesPerBlock == 0);
                CHECK(zz_work_bytes(n_ant, n_src, prec, cap) <= cap || n_ant > 1024);
            }

    // ---- planned FFT table: every even 5-smooth length 16..2304 has a row
    // and a column plan, and 2306..4608 a row plan, within the LDS budget (16
    // wavefronts per compute unit: 80 KB per 512-thread workgroup); nothing
    // else has one; column plans take a power of two of lines, up to 128
    for (int L = 2; L <= 4700; ++L) {
        int nl = 0;
        size_t lds = 0;
        for (bool cols : {false, true}) {
            const bool want = L >= 16 && L <= (cols ? 2304 : 4608) && L % 2 == 0 && smooth5(L);
            const bool have = fft_reg_info(L, cols, &nl, &lds);
            CHECK(have == want);
            if (have) {
                CHECK(nl >= 1 && lds > (size_t)8 * L && lds <= 80 * 1024);
                if (cols) CHECK(nl >= 1 && nl <= 128 && (nl & (nl - 1)) == 0);  // a power of two
            }
        }
    }

    if (g_fail) {
        std::fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("host sizing checks: all passed\n");
    return 0;
}
