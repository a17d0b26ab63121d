/*
 * fv.h -- C ABI of the MI355X (gfx950) visibility simulator.
 *
 * The library evaluates, for every frequency nu_f and antenna pair i <= j,
 *
 *     V_f(i,j) = sum_s beam[f][s] * flux[f][s]
 *                      * exp(-2 pi i (nu_f / c) (x_i - x_j) . s_hat_s)
 *
 * (paper section 2.2: the point-source form of the measurement equation,
 * rewritten as a type-3 non-uniform FFT from sources s_j to target modes
 * x_k = -2 pi nu b_k / c; the pair orientation b_ij = x_i - x_j follows the
 * per-antenna phasor factorisation of section 5.1), either with the type-3
 * NUFFT (spread with the ES kernel, oversampled FFT, deconvolve and
 * interpolate; section 2.2 steps 1-3) or with a direct sum.
 *
 * Conventions for every entry point
 *   ant_enu  [n_ant][3]  antenna positions, metres, East/North/Up, FP64.
 *   src_lmn  [n_src][3]  unit direction vectors (l=East, m=North, n=Up), FP64;
 *                        |s| must be 1 within 1e-9.  No horizon cut is made.
 *   freq_hz  [n_freq]    frequencies, Hz, > 0.
 *   flux     [n_freq][n_src]  Stokes-I flux (any sign), FP64.
 *   beam     [n_freq][n_src]  real beam weight applied as-is (the source
 *                        strength is beam*flux); NULL means 1.
 *   vis      [n_freq][n_ant*(n_ant+1)/2] complex128 (interleaved re, im),
 *                        pairs (i <= j) in row-major order (autos included);
 *                        a device output must be 16-byte aligned (FV_EINVAL
 *                        otherwise).
 *   eps      requested relative l2 error of the whole output of the call
 *            (all frequencies, all pairs) against the exact sum;
 *            1e-14 <= eps <= 1e-1.
 *
 * Ownership: the caller owns every input and output buffer; the context owns
 * every device buffer it allocates.  On any non-OK status the output is left
 * untouched.  Status codes are returned; nothing aborts across the ABI.
 * A context serves one host thread, except the server entry points, which
 * are thread-safe.
 */
#ifndef FV_H
#define FV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FV_OK = 0,
    FV_EINVAL = -1,        /* bad size, pointer, non-finite value, eps out of range */
    FV_ENOMEM = -2,        /* footprint above the context's HBM budget or allocation failed */
    FV_EDEVICE = -3,       /* a HIP call failed; the context stays usable */
    FV_EUNSUPPORTED = -4,  /* e.g. FP32 forced with eps < 1e-6 */
    FV_EBUSY = -5,         /* server not running / already running / queue full */
    FV_ECANCELLED = -6,    /* request dropped by fv_server_stop */
    FV_ETIMEOUT = -7       /* fv_wait timed out; the ticket stays valid */
} fv_status;

/* flags (bitwise or) */
#define FV_DIM_AUTO        0x0u   /* 2-D if the array is flat within the eps tolerance, else 3-D */
#define FV_DIM_2D          0x1u   /* force u*l + v*m (the Up terms are dropped) */
#define FV_DIM_3D          0x2u   /* force u*l + v*m + w*n */
#define FV_DIM_MASK        0x3u
#define FV_PREC_AUTO       0x0u   /* FP32 grids if eps >= 1e-6, else FP64 */
#define FV_PREC_FP32       0x4u
#define FV_PREC_FP64       0x8u
#define FV_PREC_MASK       0xCu
#define FV_METHOD_NUFFT    0x00u  /* type-3 NUFFT (default) */
#define FV_METHOD_DIRECT   0x10u  /* direct sum, one thread per pair (vector ALU) */
#define FV_METHOD_MFMA     0x20u  /* direct sum as V = Z diag(c) Z^H on matrix cores */
#define FV_METHOD_MASK     0x30u
#define FV_NO_FOLD         0x100u /* do not reflect targets into a half-space */
#define FV_TIMING          0x200u /* record HIP events around every stage launch (the call then
                                     waits for its own work and fills the t_stage_ms fields) */
#define FV_AUTOTUNE        0x400u /* NUFFT: when this problem class (dimension, precision, grid and
                                     snapshot-count buckets) has no tuned FFT launch shape yet, time
                                     the candidates on this call's grids first and keep the fastest
                                     (in the context, and in the file set by fv_set_tune_cache) */
#define FV_GRAPH           0x800u /* NUFFT: capture the call's launch sequence as a HIP graph and
                                     replay it on later calls with the same sizes and workspace;
                                     needs a non-null stream; per-stage timing is then not recorded */
#define FV_NO_LATTICE      0x1000u /* NUFFT: do not use the type-1 path for lattice arrays (paper section
                                      2.2.1); by default a coplanar array whose East/North positions form
                                      a lattice within eps c / (20 pi nu_max) metres is simulated with a
                                      type-1 transform onto its integer baseline modes when that grid is
                                      the smaller one */
#define FV_TIMING_ACCUM    0x2000u /* device entry point: record the stage events like FV_TIMING but do
                                      not wait for them; fv_stage_times returns their sums over every
                                      such call since its last use (t_stage_ms stays 0 in each call's
                                      report, stage_bytes and stage_launches are filled) */
#define FV_TIMING_ONE_STAGE 0x4000u /* with FV_TIMING or FV_TIMING_ACCUM: only the stage in flag bits
                                      16-19 (FV_TIMING_STAGE) records events, two per launch of it; the
                                      other stages' times stay 0 */
#define FV_DETERMINISTIC   0x8000u /* NUFFT: bitwise reproducible output.  The type-3 spread adds each
                                      tile's records in an order fixed by the sources' indices (a stable
                                      rank inside every sort bin, one extra pass over the records)
                                      instead of the order in which atomic counters returned; the same
                                      problem then gives the same bits on every call, alone or among
                                      other requests of the serving loop.  The type-1 path and the direct
                                      sums are reproducible without it. */
#define FV_TIMING_STAGE(s) (FV_TIMING_ONE_STAGE | ((unsigned)(s) << 16))  /* s: an FV_STAGE_* index */
#define FV_TIMING_STAGE_OF(flags) ((int)(((flags) >> 16) & 0xFu))

/* stage indices of fv_report.t_stage_ms / stage_bytes / stage_launches */
#define FV_STAGE_SORT      0      /* key, count, scan and scatter of the source records */
#define FV_STAGE_SPREAD    1      /* ES spreading into LDS tiles, first deconvolution */
#define FV_STAGE_FFT_X     2
#define FV_STAGE_FFT_Y     3
#define FV_STAGE_FFT_Z     4
#define FV_STAGE_INTERP    5      /* interpolation, second deconvolution, phases */
#define FV_STAGE_DIRECT    6      /* direct-sum kernels */
#define FV_STAGE_OTHER     7      /* tables (1/psi2hat, targets) */
#define FV_NSTAGE          8

typedef struct fv_ctx fv_ctx;

typedef struct {
    int n_ant;  const double *ant_enu;
    int n_src;  const double *src_lmn;
    int n_freq; const double *freq_hz;
    const double *flux;
    const double *beam;     /* NULL => 1 */
    double eps;
    unsigned flags;
} fv_problem;

typedef struct {
    int dim;              /* 2 or 3 */
    int prec_bits;        /* 32 or 64 (grid arithmetic) */
    int method;           /* FV_METHOD_* */
    int w;                /* kernel points per dimension */
    int fold_axis;        /* -1 when targets are not reflected */
    int n1[3], n2[3];     /* spreading / FFT grid of the highest frequency */
    double t_total_ms;    /* wall time of the call (host clock, includes sync) */
    double model_bytes;   /* algorithmic HBM bytes of the grid stages (all frequencies) */
    double src_pairs;     /* n_src * n_pairs * n_freq */
    double t_stage_ms[FV_NSTAGE];     /* FV_TIMING: summed event time of each stage's launches */
    double stage_bytes[FV_NSTAGE];    /* algorithmic HBM bytes of each stage (all launches) */
    int stage_launches[FV_NSTAGE];    /* kernel launches per stage */
    int lattice;          /* 1 when the type-1 lattice path ran (then n1 holds its fine grid) */
    int reserved;
} fv_report;

/* Create a context on HIP device `device`.  hbm_budget_bytes = 0 means 90%
 * of the device's free memory.  Returns FV_EDEVICE if the device is absent. */
fv_status fv_create(int device, size_t hbm_budget_bytes, fv_ctx **out);
void fv_destroy(fv_ctx *ctx);
/* Message for the last non-OK status returned on the calling thread. */
const char *fv_last_error(void);

/* Host buffers in, host buffer out (blocking).  rep may be NULL. */
fv_status fv_simulate(fv_ctx *ctx, const fv_problem *p, double *vis, fv_report *rep);

/* Device buffers in and out: every array pointer in *p and vis are device
 * pointers on the context's device.  The work is enqueued on `stream`
 * (a hipStream_t; NULL = the null stream).  The call blocks only for the few
 * scalars planning needs (antenna positions, frequencies, the source box);
 * the buffers must stay alive until the stream has completed the work.
 * Successive calls on one context are ordered: a call made on another stream
 * first waits (on the device) for the previous call's work, whose workspace it
 * reuses. */
fv_status fv_simulate_dev(fv_ctx *ctx, const fv_problem *p, double *vis, void *stream, fv_report *rep);

/* Many snapshots (each a problem with its own sources, frequencies and
 * array) in one batched launch sequence; host buffers; vis[i] is the output
 * of snaps[i].  rep (nullable) receives the report of the whole batch. */
fv_status fv_simulate_batch(fv_ctx *ctx, int n_snap, const fv_problem *snaps, double *const *vis,
                            fv_report *rep);

/* Many snapshots whose arrays are on the device (the per-(time, frequency)
 * simulations of paper section 5.4 with their inputs already resident).
 * snaps and vis are host arrays of n_snap entries; every array pointer inside
 * snaps[i], and vis[i] (16-byte aligned, n_freq x n_pairs complex doubles),
 * is a device pointer on the context's device.  The call enqueues the input
 * check of the whole batch (two launches) and one copy of the planning
 * scalars (antenna positions, frequencies, source box), waits for them, then
 * enqueues the whole batch on `stream` (a hipStream_t; NULL = the null
 * stream) and returns:
 * lattice snapshots of one (precision, kernel width) run as one launch per
 * stage, and with FV_GRAPH in their flags that launch sequence is captured
 * once per shape and replayed.  Buffers stay alive until the stream has
 * completed.  Ordered with the context's other calls as fv_simulate_dev is.
 * A batch that repeats the previous batch's arguments (the same device
 * pointers, sizes, eps and flags) is enqueued right behind its input
 * check, planned on the previous batch's scalars, while the host waits for
 * the check; when the new scalars differ (the arrays' contents changed) the
 * batch is enqueued again with the new plan, and when the check fails the
 * outputs of such a batch may already have been written.
 * Errors: FV_EINVAL for a null or misaligned pointer, bad sizes or eps, and
 * invalid values the device check finds (nothing is computed then, except as
 * said for a repeated batch); FV_EUNSUPPORTED for more than 65535 snapshots, or more than 65535
 * (snapshot, frequency) rows in one lattice group; FV_ENOMEM / FV_EDEVICE
 * from the device. */
fv_status fv_simulate_batch_dev(fv_ctx *ctx, int n_snap, const fv_problem *snaps, double *const *vis, void *stream,
                                fv_report *rep);

/* Drift scan with the front end on the device (paper section 2.3: between
 * astrometric pre-corrections, a rigid rotation set by the local sidereal
 * time and the latitude takes pre-corrected equatorial positions to the local
 * East-North-Up frame; section 2.4: analytic beams evaluated in closed form at
 * the source positions).  For each time t and frequency f:
 *   s_t = R(lst[t], latitude) src_eq              (ENU unit vectors, FP64)
 *   beam = 2^(-(2 theta / F_f)^2), theta = zenith angle of s_t,
 *          F_f = beam_fwhm * beam_nu_ref / freq_hz[f]; 0 where Up <= 0
 *          (beam_fwhm = 0: 1 above the horizon, 0 at and below it)
 *   vis[t][f] = the visibilities of (ant_enu, s_t, freq_hz[f], flux[f], beam)
 * as fv_simulate_dev computes them (same eps contract, same path choice).
 * The sky stays on the device: no per-(time, frequency, source) array crosses
 * the bus.  Sources at or below the horizon (zero beam) are dropped before
 * the transform; fv_report.src_pairs counts the visible ones. */
typedef struct {
    int n_ant;  const double *ant_enu;   /* HOST [n_ant][3] metres (E, N, U) */
    int n_src;  const double *src_eq;    /* DEVICE [n_src][3] unit vectors, equatorial (x: RA 0 on the
                                            equator, z: north celestial pole), pre-corrected */
    int n_freq; const double *freq_hz;   /* HOST [n_freq] */
    const double *flux;                  /* DEVICE [n_freq][n_src] */
    int n_time; const double *lst;       /* HOST [n_time] local sidereal times, radians */
    double latitude;                     /* radians, in [-pi/2, pi/2] */
    double beam_fwhm;                    /* radians at beam_nu_ref; 0 = unit beam above the horizon */
    double beam_nu_ref;                  /* Hz (> 0 when beam_fwhm > 0) */
    double eps;
    unsigned flags;                      /* FV_* flags as in fv_problem; the NUFFT method only */
} fv_drift;

/* vis: DEVICE [n_time][n_freq][n_pairs] complex128 (interleaved re, im).
 * Work is enqueued on `stream`; the call blocks once per group of times for
 * the planning scalars (source box and input checks of each rotated
 * snapshot).  Workspace: the rotated directions and beam values of a group of
 * times, sized to a quarter of the context's HBM budget.  Errors: FV_EINVAL
 * for bad sizes, non-finite or out-of-range scalars, non-unit source vectors
 * or non-finite fluxes (the output is then undefined). */
fv_status fv_simulate_drift(fv_ctx *ctx, const fv_drift *d, double *vis, void *stream, fv_report *rep);

/* Per-antenna beams (paper section 2.2.3: when antennas carry different
 * beam patterns, each unordered pair of patterns defines its own response to
 * the sky, so one snapshot takes N_beam (N_beam + 1) / 2 transforms).  With
 * real amplitude patterns a_p and pattern p(i) on antenna i:
 *   V_ij(nu) = sum_s a_{p(i)}(nu, s) a_{p(j)}(nu, s) flux(nu, s)
 *              exp(-2 pi i (nu / c) (x_i - x_j) . s_hat_s)
 * to the eps contract of fv_simulate_dev.  One transform runs for each pattern
 * pair that occurs among the antenna pairs (strengths a_p a_q flux, formed on
 * the device); each visibility is taken from the transform of its pair. */
typedef struct {
    int n_ant;  const double *ant_enu;   /* DEVICE [n_ant][3] metres */
    int n_src;  const double *src_lmn;   /* DEVICE [n_src][3] unit vectors (l, m, n) */
    int n_freq; const double *freq_hz;   /* DEVICE [n_freq] */
    const double *flux;                  /* DEVICE [n_freq][n_src] */
    int n_beam; const double *beams;     /* DEVICE [n_beam][n_freq][n_src] amplitude patterns */
    const int *beam_of_ant;              /* HOST [n_ant] pattern index of each antenna, in [0, n_beam) */
    double eps;
    unsigned flags;                      /* FV_* flags as in fv_problem; the NUFFT method only */
} fv_beams;

/* vis: DEVICE [n_freq][n_pairs] complex128.  Work is enqueued on `stream`;
 * the call blocks once for the planning scalars.  Workspace: the product
 * strengths and one visibility array per pattern pair.  Errors: FV_EINVAL for
 * bad sizes, pattern indices out of range, non-unit directions or non-finite
 * values. */
fv_status fv_simulate_beams(fv_ctx *ctx, const fv_beams *b, double *vis, void *stream, fv_report *rep);

/* Polarised feed products (paper section 2.1, the measurement equation in
 * Jones form) with one beam shared by every antenna:
 *   V_ij = sum_s A(s) C(s) A(s)^H exp(-2 pi i (nu / c) (x_i - x_j) . s_hat_s),
 *   C = [[I + Q, U + i V], [U - i V, I - Q]],
 * a 2 x 2 complex matrix per pair and frequency, to the eps contract of
 * fv_simulate_dev for each product.  P = A C A^H is Hermitian, so four
 * transforms with real strengths (P_xx, P_yy, Re P_xy, Im P_xy, formed on the
 * device) give all four products. */
typedef struct {
    int n_ant;  const double *ant_enu;   /* DEVICE [n_ant][3] metres */
    int n_src;  const double *src_lmn;   /* DEVICE [n_src][3] unit vectors (l, m, n) */
    int n_freq; const double *freq_hz;   /* DEVICE [n_freq] */
    const double *stokes;                /* DEVICE [4][n_freq][n_src]: I, Q, U, V */
    const double *jones;                 /* DEVICE [n_freq][n_src][2][2] complex (interleaved re, im) feed
                                            response A, or NULL for ideal feeds (A = identity) */
    double eps;
    unsigned flags;                      /* FV_* flags as in fv_problem; the NUFFT method only */
} fv_polar;

/* vis: DEVICE [4][n_freq][n_pairs] complex128, products in the order xx, xy,
 * yx, yy (row-major 2 x 2), 16-byte aligned.  Work is enqueued on `stream`;
 * the call blocks once for the planning scalars.  Workspace: four strength
 * arrays and four visibility arrays.  Errors: FV_EINVAL for bad sizes,
 * non-unit directions or non-finite values. */
fv_status fv_simulate_polar(fv_ctx *ctx, const fv_polar *q, double *vis, void *stream, fv_report *rep);

/* Spectral basis (paper appendix A, which the paper leaves unvalidated): the
 * flux and beam spectra of every source are projected onto n_basis
 * orthonormal functions of frequency (discrete orthonormal polynomials in
 * (nu - nu_mid) / half-width), their product is expanded with the basis's
 * structure constants d_ijk = sum_q M_qi M_qj M_qk, and one type-3 transform
 * per basis function, planned at the highest frequency, is evaluated at the
 * baselines of every frequency; the visibilities are the expansion
 *   V(b, nu_q) = sum_k M_qk F_k(b nu_q / c).
 * The result approximates fv_simulate_dev's to within the basis's fit of the
 * spectra (exact for a complete basis, n_basis = n_freq) plus eps.  Arrays as
 * for fv_simulate_dev (device pointers); 1 <= n_basis <= min(n_freq, 16).
 * vis: DEVICE [n_freq][n_pairs] complex128, 16-byte aligned.  Workspace: the
 * coefficients and one [n_freq][n_pairs] array per basis function. */
fv_status fv_simulate_basis(fv_ctx *ctx, const fv_problem *p, int n_basis, double *vis, void *stream,
                            fv_report *rep);

/* Allocation-free variant of fv_simulate_dev for the matrix-core direct form
 * (flags must select FV_METHOD_MFMA), for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Arrays as for fv_simulate_dev (device pointers; vis
 * [n_freq][n_pairs] complex128, 16-byte aligned); it runs on the calling
 * thread's current HIP device and enqueues on `stream` (a hipStream_t of that
 * device; NULL = the null stream), blocking once for the planning scalars.
 * It needs no context and makes no device or pinned allocation: every buffer
 * beyond the inputs and the output (the input check's partials and scalars,
 * the Z chunk, the strengths, the partial tiles) lives in one 64 MiB array in
 * the library's device memory, one copy per device, held until the process
 * ends.  Limits: n_ant <= 1024 and n_freq <= 1024, and the partial tiles of
 * the pair triangle must fit the array (sources are processed in chunks that
 * fit); beyond them FV_EINVAL.  Every call on a device shares that device's
 * array, which keeps the last call's contents: calls that overlap on one
 * device (other streams or threads) race.  Errors as for fv_simulate_dev;
 * FV_EINVAL also for any other method. */
fv_status fv_simulate_mfma_noalloc(const fv_problem *p, double *vis, void *stream);

/* Serving loop: a worker thread admits submitted requests while HBM (the
 * context budget) and one of max_slots slots are free, and runs admitted
 * requests concurrently on per-slot streams.  Host buffers, which must stay
 * alive until fv_wait returns FV_OK / FV_ECANCELLED / an error for the
 * ticket. */
fv_status fv_server_start(fv_ctx *ctx, int max_slots);
fv_status fv_submit(fv_ctx *ctx, const fv_problem *p, double *vis, uint64_t *ticket);
/* A request whose arrays are on the device (device pointers in *p, vis as for
 * fv_simulate_dev), so that a serving loop can keep inputs resident.  The
 * call copies the antenna positions and frequencies back (two small blocking
 * copies) to size the request's footprint, with the source box taken as the
 * whole direction cube; the request runs on its slot's stream: input check,
 * planning, transform, then the slot waits for it.  The buffers stay alive
 * until fv_wait returns.  Errors as fv_submit, and argument errors as
 * fv_simulate_dev. */
fv_status fv_submit_dev(fv_ctx *ctx, const fv_problem *p, double *vis, uint64_t *ticket);
/* timeout_s < 0 waits forever.  rep (nullable) receives the request's report
 * with t_total_ms = submit -> completion latency. */
fv_status fv_wait(fv_ctx *ctx, uint64_t ticket, double timeout_s, fv_report *rep);
fv_status fv_server_stop(fv_ctx *ctx);

/* Autotuner cache file (JSON object: class key -> launch shape).  Entries in
 * the file are loaded now; new entries found by FV_AUTOTUNE calls are written
 * back.  path NULL or "" keeps the cache in memory only.  An unreadable or
 * missing file is not an error. */
/* Stage event times of the FV_TIMING_ACCUM calls on this context since the
 * last fv_stage_times: waits for them, writes the summed milliseconds and the
 * number of timed launches of each stage (arrays of FV_NSTAGE; either may be
 * NULL) and starts a new sum.  *n_calls (may be NULL) receives the number of
 * calls. */
fv_status fv_stage_times(fv_ctx *ctx, double *ms, int *launches, int *n_calls);

fv_status fv_set_tune_cache(fv_ctx *ctx, const char *path);

/* Diagnostic entry point for stage-by-stage checks of the NUFFT path
 * (section 2.2 steps 1-3) on one frequency `f` of a host problem.
 * Writes the plan scalars and, when the buffers are non-NULL and large
 * enough, copies out (as complex128):
 *   spread:  the deconvolved spreading grid b~, [n1z][n1y][n1x];
 *   fftout:  the pruned FFT output, [Mz][My][Mx], element (o) holding
 *            grid index p = o - P (mod n2) along each axis.
 * plan_out[0..]: dim, w, fold_axis, n1[3], n2[3], M[3], P[3] as doubles,
 *   then s_c[3], S[3], b_c[3], B[3]  (31 doubles).
 * Returns FV_EINVAL if the buffers are too small (sizes are in plan_out). */
fv_status fv_debug_stages(fv_ctx *ctx, const fv_problem *p, int f, double *plan_out,
                          double *spread, size_t spread_cap, double *fftout, size_t fftout_cap);

#ifdef __cplusplus
}
#endif
#endif /* FV_H */
