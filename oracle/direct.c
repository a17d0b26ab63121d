/*
 * oracle/direct.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
 *
 * Plain, slow, obviously-correct FP64 direct evaluation of the point-source
 * visibility sum (paper section 2.2, the point-source form of the measurement
 * equation, and the type-3 sum it is rewritten as):
 *
 *     V_f(i,j) = sum_s  beam[f][s] * flux[f][s]
 *                       * exp( -2*pi*i * (nu_f / c) * (x_i - x_j) . s_hat_s )
 *
 * with b_ij = x_i - x_j (the orientation fixed by the per-antenna phasor
 * factorisation of section 5.1) over pairs i <= j in row-major order.
 * Every pair is evaluated on its own with the host libm sin/cos, summed in
 * source order in FP64.  No recurrences, no factorisation, no transforms.
 * OpenMP only splits the independent output pairs across threads.
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg call this.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_C_LIGHT 299792458.0

/* Decode pair index p of the (i <= j) row-major layout by walking rows. */
static void pair_ij(int64_t n_ant, int64_t p, int64_t *pi, int64_t *pj)
{
    int64_t i = 0, row = n_ant;
    while (p >= row) { p -= row; ++i; --row; }
    *pi = i;
    *pj = i + p;
}

/*
 * ant[n_ant][3] metres ENU; lmn[n_src][3] unit vectors; freq[n_freq] Hz;
 * flux, beam: [n_freq][n_src] (beam may be NULL => 1).
 * drop_up != 0 evaluates the coplanar (2-D) form u*l + v*m (the Up term
 * dropped), used only to check a forced 2-D mode on a non-flat array.
 * pairs: NULL => all n_ant*(n_ant+1)/2 pairs, else n_out pair indices.
 * vis: [n_freq][n_out] interleaved (re, im) doubles.
 * Returns 0, or -1 on bad arguments.
 */
int oracle_direct_vis(int n_ant, const double *ant, int n_src, const double *lmn,
                      int n_freq, const double *freq, const double *flux,
                      const double *beam, int drop_up, int64_t n_out,
                      const int64_t *pairs, double *vis, int nthreads)
{
    if (n_ant < 1 || n_src < 0 || n_freq < 1 || n_out < 0 || !ant || !freq || !vis)
        return -1;
    if (n_src > 0 && (!lmn || !flux))
        return -1;
    const int64_t n_pairs = (int64_t)n_ant * (n_ant + 1) / 2;
    if (!pairs && n_out != n_pairs)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const double two_pi = 2.0 * M_PI;
    for (int f = 0; f < n_freq; ++f) {
        const double scale = freq[f] / ORACLE_C_LIGHT;
        const double *fl = flux ? flux + (int64_t)f * n_src : NULL;
        const double *bm = beam ? beam + (int64_t)f * n_src : NULL;
        double *out = vis + (int64_t)f * n_out * 2;
        int64_t k;
#pragma omp parallel for schedule(static)
        for (k = 0; k < n_out; ++k) {
            int64_t p = pairs ? pairs[k] : k;
            int64_t i, j;
            if (p < 0 || p >= n_pairs) { out[2 * k] = NAN; out[2 * k + 1] = NAN; continue; }
            pair_ij(n_ant, p, &i, &j);
            const double bx = ant[3 * i + 0] - ant[3 * j + 0];
            const double by = ant[3 * i + 1] - ant[3 * j + 1];
            const double bz = drop_up ? 0.0 : ant[3 * i + 2] - ant[3 * j + 2];
            double re = 0.0, im = 0.0;
            for (int s = 0; s < n_src; ++s) {
                const double c = bm ? bm[s] * fl[s] : fl[s];
                const double dot = bx * lmn[3 * s] + by * lmn[3 * s + 1] + bz * lmn[3 * s + 2];
                const double ph = -two_pi * scale * dot;
                re += c * cos(ph);
                im += c * sin(ph);
            }
            out[2 * k] = re;
            out[2 * k + 1] = im;
        }
    }
    return 0;
}

/* Threads the OpenMP runtime would use for the next parallel region. */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
