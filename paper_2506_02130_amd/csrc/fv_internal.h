// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>
#include <mutex>
#include <list>

#include "../../include/fv.h"

namespace fv {

constexpr double kCLight = 299792458.0;
constexpr double kSigma = 2.0;   // upsampling factor of the FFT grid
constexpr int kMaxW = 16;        // largest kernel width handled
constexpr int kMinW = 3;
constexpr int kQuadHalf = 32;    // positive nodes of the 64-node Gauss-Legendre rule
constexpr int kSubBin = 8;       // sub-bin edge (cells) of the source sort along x and y
constexpr int kSubBinZ = 4;      // sub-bin edge along z
constexpr int kSrcCheckBlocks = 2048;  // blocks of the input-check pass (one partial each)

// ---------------------------------------------------------------------------
// Errors: internal code throws fv::Error; every ABI entry converts it to a
// status code and records the message for fv_last_error().
struct Error {
    fv_status code;
    std::string msg;
};
[[noreturn]] void fail(fv_status code, const std::string &msg);
void set_last_error(const std::string &msg);  // the message fv_last_error() returns on this thread
void hip_check(hipError_t e, const char *what);
#define FV_HIP(call) ::fv::hip_check((call), #call)

// ---------------------------------------------------------------------------
// Per-snapshot parameters read by every stage kernel (plain data, in device
// memory as an array indexed by snapshot).  A snapshot is one (problem,
// frequency) pair.
struct SnapDev {
    int n1[3], n2[3], M[3], P[3];    // spreading grid, FFT grid, pruned output M = 2P+1
    int ntile[3];                    // spread tiles per axis
    int nsb[3];                      // sort sub-bins per axis
    int cx[3];                       // lines per workgroup of each FFT pass
    int fft_split[3];                // 1: one parity transform per workgroup
    int dim, w, n_src, n_tgt;
    int degenerate;                  // bit a: X_a was clamped to 1 rad
    int pad0;
    long long tile_base;             // first global spread tile of this snapshot
    long long src_base;              // offset in the rank / record arrays
    long long bin_base;              // offset in the sub-bin array (nbins + 1 entries)
    long long bufA, bufB;            // element offsets of the two grid regions
    long long ipsi_base;             // offset of the 1/psi2hat tables (n1[0] | n1[1] | n1[2])
    long long wg_base[3];            // first workgroup of each FFT pass
    long long reg_base[3];           // first workgroup of each planned FFT pass (fft_reg.h)
    long long order_base;            // offset of this source list's shared order, or -1
    const double *src;               // [n_src][3]
    const double *flux;              // [n_src] this frequency
    const double *beam;              // [n_src] this frequency, or nullptr
    double *out;                     // [n_pairs] complex128 of this frequency
    const double *tb;                // folded target baselines, [dim][n_tgt]
    const int *tidx;                 // pair index | (reflected << 31)
    const double *tphi;              // phihat at each target, [dim][n_tgt]
    const double *qn;                // quadrature table of this w
    const void *tw[3];               // twiddle table of n2[a]
    const int *drev[3];              // output position of each bin of an n1[a]-point transform
    double gscale[3];                // grid cells per unit of s: sigma X / pi
    double s_c[3];
    double qscale[3];                // target grid coordinate q = qscale (b - b_c)
    double b_c[3];
    double xi_deg[3];                // clamped axes: xi = xi_deg (b - b_c)
    double pre_turn[3];              // pre-phase turns = pre_turn . (s - s_c)
    double post_turn;                // post-phase turns = post_turn (b . s_c)
    double post_norm;                // prod_a 4 pi / (n2_a w)
    double beta;
};

// Host plan of one snapshot.
struct SnapPlan {
    int dim = 2, w = 8, fold_axis = -1;
    int n1[3] = {1, 1, 1}, n2[3] = {1, 1, 1}, M[3] = {1, 1, 1}, P[3] = {0, 0, 0};
    double X[3] = {1, 1, 1};
    double S[3] = {0, 0, 0}, s_c[3] = {0, 0, 0}, b_c[3] = {0, 0, 0}, B[3] = {0, 0, 0};
    double k = 0;  // 2 pi nu / c
    double nu = 0;
    int degenerate = 0;
    long long cells1() const { return (long long)n1[0] * n1[1] * n1[2]; }
    long long cellsM() const { return (long long)M[0] * M[1] * M[2]; }
};

// Geometry-level plan shared by all frequencies of one problem.
struct GeomPlan {
    int dim = 2, w = 8, fold_axis = -1, n_ant = 0;
    long long n_pairs = 0;
    double S[3] = {0, 0, 0}, s_c[3] = {0, 0, 0};
    double b_c[3] = {0, 0, 0}, B[3] = {0, 0, 0};
};

// Kernels asking for more than 64 KB of dynamic LDS must say so first; the
// attribute is set once per (kernel, device, size) and remembered.
void ensure_lds(const void *fn, size_t bytes);
int kernel_width(double eps);
int kernel_width_type1(double eps);  // the lattice path's width (one kernel application)
int next_smooth_even(long long n);
void src_box(const double *src, int n_src, int dim, double *s_c, double *S);
GeomPlan plan_geometry(const double *ant, int n_ant, int dim, double eps, const double *s_c, const double *S,
                       bool fold);
SnapPlan plan_snapshot(const GeomPlan &g, double nu);
void fold_baseline(const double *b, int dim, int axis, double *out, bool *flipped);
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);
int choose_dim(const double *ant, int n_ant, double eps, const double *freq, int n_freq, unsigned flags);
int choose_prec(double eps, unsigned flags);
void quad_table(int w, double *out64);  // host: the 2*kQuadHalf quadrature table of width w

// ---------------------------------------------------------------------------
// Device memory: a growable bump arena (one allocation).  Callers make sure
// no in-flight work uses the arena before `ensure` reallocates it.
// Pinned host staging (hipHostMalloc), grown on demand.  An upload from it
// records `ev`; wait() blocks until that upload has been read, so the buffer
// can be refilled.
struct PinnedBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
    void *get(size_t bytes);  // waits for a pending upload first
    void record(hipStream_t s);
    void wait();
    void release();
};

struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    PinnedBuf host;  // staging of the per-launch snapshot table
    // The snapshot and order tables the last type-3 launch uploaded to the
    // start of this arena (their bytes, back to back), so that a repeated
    // launch with the same plan and buffers skips the upload.  Dropped by
    // reset() and by reallocation: any other use of the arena may overwrite
    // that memory, and only the type-3 set-up takes the record out before
    // its own reset().
    std::vector<char> tables;
    bool ipsi = false;  // and a launch with those tables has computed its deconvolution tables
    void ensure(size_t bytes);          // reallocate (contents lost) if smaller
    void reset() {
        used = 0;
        tables.clear();
        ipsi = false;
    }
    void *take(size_t bytes, size_t align = 256);
    void release();
};

// Device tables reused across calls: twiddles per (n, precision), quadrature
// tables per w.
struct DevCache {
    std::mutex mu;  // the tables are shared by every slot of a context
    std::map<std::pair<int, int>, void *> twiddles;
    std::map<int, double *> qnodes;
    std::map<int, int *> drevs;
    const void *twiddle(int n, int prec_bits, hipStream_t s);
    const int *digit_reversal(int n, hipStream_t s);
    const double *quad(int w, hipStream_t s);
    void release();
};

// Target table of one (array, dim, fold axis, w): folded baselines, pair
// indices and phihat at the normalised target positions.
struct TargetTable {
    uint64_t key = 0;
    int dim = 0, w = 0, fold_axis = -1, n_ant = 0;
    long long n_tgt = 0;
    double *tb = nullptr;
    int *tidx = nullptr;
    double *tphi = nullptr;
    void release();
};

// Per-stage accounting of one call: algorithmic bytes and launch counts
// always; HIP event times around every stage when `on`.
struct StageTimer {
    bool on = false;
    double ms[FV_NSTAGE] = {0}, bytes[FV_NSTAGE] = {0};
    int launches[FV_NSTAGE] = {0};
    struct Mark {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    int cur = -1;
    hipEvent_t cur_a = nullptr;
    // accum: keep the events of earlier calls (FV_TIMING_ACCUM); collect()
    // then leaves them for take()
    bool accum = false;
    int calls = 0;
    int only = -1;  // >= 0: the one stage that records events
    void reset(bool enable, bool accum_mode = false, int only_stage = -1);
    // sums of the kept events per stage (waits for them) and starts anew
    void take(double *ms_out, int *launches_out, int *calls_out);
    void begin(int stage, hipStream_t s);
    void end(hipStream_t s);
    // Start and stop events for one kernel launched with hipExtLaunchKernel
    // (the dispatch itself records them: no separate marker packets), both
    // null when timing is off.
    void kernel_events(int stage, hipEvent_t *a, hipEvent_t *b);
    void add(int stage, double b, int n_launch) {
        bytes[stage] += b;
        launches[stage] += n_launch;
    }
    void collect();  // waits for the last recorded event, sums the stage times
    ~StageTimer();
};

// One (problem, frequency) snapshot of a NUFFT launch group.
struct SnapJob {
    SnapPlan plan;
    const double *src = nullptr;   // device [n_src][3]
    int n_src = 0;
    const double *flux = nullptr;  // device row of this frequency
    const double *beam = nullptr;  // device row or nullptr
    double *out = nullptr;         // device [n_pairs] complex128
    const TargetTable *tt = nullptr;
};

// Launch shape of the FFT passes: transforms per workgroup and threads per
// workgroup.  Defaults were measured on the 350-antenna workload;
// FV_FFT_ROWS, FV_FFT_MAX_LINES, FV_FFT_TPB1 and FV_FFT_TPBM override them,
// and the autotuner searches them per problem class.
struct Tuning {
    int rows = 1;    // rows per workgroup of the x pass
    int lines = 2;   // columns per workgroup of the other passes
    int tpb1 = 0;    // threads of the x pass (0: by line length)
    int tpbm = 256;  // threads of the other passes
    int split = 0;   // 1: even and odd transforms of a line in separate workgroups
    double fft_ms = 0.0;  // FFT time measured by the autotuner (0: not tuned)
    static Tuning defaults();
    int tpb(int line_len, bool multi) const;
};

// Autotuned launch shapes per problem class, optionally persisted as JSON.
struct TuneCache {
    std::mutex mu;
    std::map<std::string, Tuning> entries;
    std::string path;  // empty: in memory only
    bool find(const std::string &key, Tuning *t);
    void put(const std::string &key, const Tuning &t);
    void load(const std::string &file);
};

// Instantiated graphs of whole launch sequences, keyed by every launch
// argument and dimension they bake in.
struct GraphCache {
    std::list<std::pair<uint64_t, hipGraphExec_t>> entries;  // most recent at the back
    hipGraphExec_t find(uint64_t key);
    void put(uint64_t key, hipGraphExec_t g);
    void release();
};

struct ExecOpts {
    bool autotune = false;   // search the launch shape when the class is not cached
    bool graph = false;      // capture / replay the launch sequence as a HIP graph
    TuneCache *tunes = nullptr;
    GraphCache *graphs = nullptr;
    size_t cap = 0;          // > 0: refuse (set *too_big) when the workspace exceeds cap bytes
    bool det = false;        // deterministic record order in the spread (FV_DETERMINISTIC)
    // spectral basis: the jobs are the K basis transforms of one plan and one
    // target table (all n_freq frequencies' pairs); with basis_vis set, the
    // interpolation writes vis[q][p] = sum_k M[q][k] V_k directly (K = the
    // number of jobs, M [n_freq][K] on the device)
    const double *basis_M = nullptr;
    double *basis_vis = nullptr;
    long long basis_np = 0;
};

// Lattice of a coplanar array (paper section 2.2.1): every antenna offset
// x_i - x_0 (East, North) is A k_i with k_i integer; A's columns are a
// reduced basis (the shortest baseline and the shortest one not parallel to
// it, Gauss-reduced).  K[a] = max - min of k[.][a].
struct LatticePlan {
    double A[2][2] = {{0, 0}, {0, 0}};  // A[r][c]: row r (East, North), column c (basis vector)
    std::vector<int> k;                 // [n_ant][2]
    int K[2] = {0, 0};
    int w = 0;                          // kernel width the tables below are for
    std::vector<double> dc;             // [N0 + N1] deconvolution factor per mode and axis
    // device copy [dc][k as int pairs] on the context's device, made by
    // lattice_tables; freed (after a device synchronisation, since kernels may
    // still read it) when the plan goes
    void *dev = nullptr;
    LatticePlan() = default;
    LatticePlan(const LatticePlan &) = delete;
    LatticePlan &operator=(const LatticePlan &) = delete;
    ~LatticePlan();
};
// True when the array's East/North positions form a lattice within `tol`
// metres (n_ant >= 2, not collinear).
bool find_lattice(const double *ant, int n_ant, double tol, LatticePlan *lp);
// phihat(xi) of the ES kernel of width w (FP64 quadrature, host).
double phihat_host(double xi, const double *qtab);  // qtab from quad_table

// FP32 kernel weights as polynomials (widths w <= kPolyMaxW, every width of an
// FP32 grid).  The weight of the kernel's i-th cell, as a function of the
// source's offset from its first cell (in (w/2 - 1, w/2]), is piece i; in
// u = 2 offset - w + 1 in (-1, 1] it is interpolated at the w + 3 Chebyshev
// nodes (degree w + 2, monomial coefficients, lowest first).  The kernel is
// even, so piece w - 1 - i is piece i at -u and only the first (w + 1) / 2
// pieces are kept.  Passed to kernels by value (kernel arguments sit in
// scalar registers).
constexpr int kPolyMaxW = 8;
struct EsPoly {
    float c[(kPolyMaxW + 1) / 2][kPolyMaxW + 3];
};
// The table of width w (computed once per width; zeros for w > kPolyMaxW).
const EsPoly &es_poly(int w);

// Type-1 path for a lattice array: every frequency of one problem.  `work`
// holds lattice_work_bytes(); `stage` is pinned host staging.
size_t lattice_work_bytes(const LatticePlan &lp, int n_src, int n_freq, int n_ant, int prec_bits, int w);
bool lattice_fits(const LatticePlan &lp, int prec_bits, int w);  // LDS limits of the kernels
void lattice_tables(LatticePlan &lp, int w);  // fills lp.w, lp.dc and lp.dev (once per plan)
void lattice_grid(const LatticePlan &lp, int w, int nf[2]);       // fine periodic grid per axis
// freq_dev: the frequencies on the device.  cmax_part / cmax_span: the device
// input check's block partials (each holds the largest |flux beam| of a flat
// range of cmax_span values), or null to have the spreading kernel find each
// chunk's largest strength itself.  Enqueues kernels only (no copies).
// One problem of a batched lattice launch (device inputs, as for launch_lattice).
struct LatItem {
    const LatticePlan *lp = nullptr;
    const double *src = nullptr, *flux = nullptr, *beam = nullptr, *cmax = nullptr, *freq = nullptr;
    long long cmax_span = 0;
    int n_src = 0, n_freq = 0, n_ant = 0;
    double *vis = nullptr;
};
// Workspace bytes of a batch (every problem's partials, row and mode arrays,
// then the parameter array and row maps), and the batch's four launches, one
// per stage for every (problem, frequency); `stage` is pinned staging for the
// parameter upload; with `graphs` (non-null, no stage timing) the four launches
// are captured once per workspace and shape and replayed.  Returns the
// algorithmic bytes.
size_t lattice_batch_bytes(const std::vector<LatItem> &items, int prec_bits, int w);
double launch_lattice_batch(const std::vector<LatItem> &items, int prec_bits, int w, void *work, PinnedBuf &stage,
                            hipStream_t st, StageTimer *tm, GraphCache *graphs);
double launch_lattice(const LatticePlan &lp, const double *src_dev, int n_src, const double *freq_dev, int n_freq,
                      const double *flux_dev, const double *beam_dev, const double *cmax_part, long long cmax_span,
                      int n_ant, int prec_bits, int w, double *vis_dev, void *work, hipStream_t st,
                      StageTimer *timer);

// Enqueue the whole type-3 pipeline for jobs that share (dim, precision, w).
// Allocates its workspace from `arena` (which must be idle); returns the
// algorithmic HBM bytes of the grid stages.
double nufft_execute(const std::vector<SnapJob> &jobs, int dim, int prec_bits, int w, Arena &arena,
                     DevCache &cache, hipStream_t s, StageTimer *timer = nullptr, const ExecOpts *opts = nullptr,
                     bool *too_big = nullptr);
// Workspace bytes nufft_execute would take for these jobs.
// Planned FP32 FFT passes (fft_reg.hip): whether line length L has a
// compile-time plan, its lines per workgroup and LDS bytes; and the launches
// of the row pass (x) and of the column passes (y, z) over every snapshot.
bool fft_reg_info(int L, bool cols, int *lines_per_wg, size_t *lds_bytes);
void launch_fft_reg_rows(const SnapDev *snaps, int n_snap, int a, void *grid, long long n_wg, size_t lds,
                         hipStream_t st, hipEvent_t ea, hipEvent_t eb);
void launch_fft_reg_cols(const SnapDev *snaps, int n_snap, int a, void *grid, long long n_wg, size_t lds,
                         hipStream_t st, hipEvent_t ea, hipEvent_t eb);
size_t nufft_workspace_bytes(const std::vector<SnapJob> &jobs, int dim, int prec_bits, int w, bool det = false);

void build_targets(const double *ant_dev, int n_ant, int dim, int fold_axis, const double *b_c, const double *B,
                   int w, const double *qn_dev, const int *perm_dev, TargetTable &tt, hipStream_t s);
// The same table over n_scale frequencies of one snapshot: target
// q n_pairs + t is the folded baseline of pair perm[t] times scale_dev[q], with
// output index q n_pairs + pair (tt holds n_pairs n_scale targets).
void build_targets_multi(const double *ant_dev, int n_ant, int dim, int fold_axis, const double *b_c, const double *B,
                         int w, const double *qn_dev, const int *perm_dev, const double *scale_dev, int n_scale,
                         TargetTable &tt, hipStream_t st);
// Spatial order of the pairs of an array: Morton order of the folded baselines
// normalised to the target box (x, y interleaved; z as the least significant
// part in 3-D).
std::vector<int> target_order(const double *ant_host, const GeomPlan &g);
// Input check and planning-scalar gather of the device entry point (device
// buffer `out` of validate_doubles() doubles): out[0..5] = min/max of l, m, n;
// out[6] = count of non-unit or non-finite directions; out[7] = count of
// non-finite flux and beam values; out[8 .. 8 + n_freq) = frequencies; then
// the 3 n_ant antenna coordinates; then kSrcCheckBlocks block partials of
// kValStride doubles.  Block b checks the flat strength range
// [b span, (b + 1) span) of the [n_freq][n_src] arrays (span =
// validate_span(n_src n_freq)), and its partial's slot kValCmax holds the
// largest |flux beam| of that range.
constexpr int kValStride = 10;
constexpr int kValCmax = 8;
inline long long validate_span(long long n_fs) { return ((n_fs + kSrcCheckBlocks - 1) / kSrcCheckBlocks + 1) & ~1LL; }
inline const double *validate_partials(const double *out, int n_ant, int n_freq) {
    return out + 8 + n_freq + 3 * (size_t)n_ant;
}
size_t validate_doubles(int n_ant, int n_freq);
void launch_validate(const double *src, int n_src, const double *flux, const double *beam, int n_freq,
                     const double *ant, int n_ant, const double *freq, double *out, hipStream_t s);
// The input check of a batch of problems in two launches.  Each problem's
// nblk blocks write their partials to `part` (kValStride doubles each; block
// b covers the flat strength range [b span, (b + 1) span)), and the fold
// writes the 8 check values, the frequencies and the antenna positions to
// `hdr` (8 + n_freq + 3 n_ant doubles), so that the headers of a batch can be
// packed together and fetched with one copy.  items_dev is a device array of
// n entries; max_blk the largest nblk.
struct ValItem {
    const double *src, *flux, *beam, *freq, *ant;
    double *hdr, *part;
    long long n_fs, span;
    int n_src, n_freq, n_ant, nblk;
};
int validate_blocks_batch(long long n_src, long long n_fs);
inline long long validate_span_n(long long n_fs, int nblk) { return ((n_fs + nblk - 1) / nblk + 1) & ~1LL; }
void launch_validate_batch(const ValItem *items_dev, int n, int max_blk, hipStream_t s);
void launch_zero_c128(double *out, long long n_complex, hipStream_t s);

// Drift-scan front end.  rot_dev [n_time][9] holds the rotations (rows E, N,
// U).  launch_frontend_count: bcnt [n_time][frontend_blocks(n_src)] receives
// the exclusive offsets of the sources above the horizon per block of
// sources, tot [n_time] the visible counts and tot[n_time] the number of
// invalid inputs (non-finite or non-unit vectors, non-finite fluxes);
// bbad [frontend_blocks] is scratch.  launch_frontend: the visible sources of
// time t, packed in input order, go to dir + t dir_stride [tot[t]][3] (ENU)
// and str + t str_stride [n_freq][tot[t]] (flux times the beam
// 2^(-kbeam[f] theta^2), or times 1 if unit_beam).
// Per-antenna beams: prod [n_vec][n_fs] = beams[p_v] * beams[q_v] with
// pq_dev [n_vec][2] pattern pairs and beams [n_beam][n_fs]; vis [n_freq][n_pairs]
// (complex) = tmp [vec[k]][n_freq][n_pairs] at each pair k.
void launch_beam_products(const double *beams, const int *pq_dev, int n_vec, long long n_fs, double *prod,
                          hipStream_t st);
void launch_beam_select(const double *tmp, const int *vec_dev, long long n_pairs, int n_freq, double *vis,
                        hipStream_t st);
// Polarised products: out [4][n_fs] = P_xx, P_yy, Re P_xy, Im P_xy of
// P = A C A^H from stokes [4][n_fs] and jones [n_fs][2][2] complex (null =
// identity); vis [4][n_fp] complex = xx, xy, yx, yy from the four transforms
// tmp [4][n_fp] complex.
void launch_polar_strengths(const double *stokes, const double *jones, long long n_fs, double *out, hipStream_t st);
void launch_polar_combine(const double *tmp, long long n_fp, double *vis, hipStream_t st);
// Spectral basis: v [K][n_src] = product coefficients of flux and beam (null
// = 1) per source, from M [n_freq][K] (orthonormal columns) and d [K][K][K].
// K is at most basis_max().
int basis_max();
void launch_basis_coeffs(const double *M_dev, const double *d_dev, int n_freq, int K, int n_src, const double *flux,
                         const double *beam, double *v, hipStream_t st);
constexpr int kFeBlock = 256;  // sources per workgroup of the front-end kernels
int frontend_blocks(int n_src);

// Workspace sizing (sizing.cpp, host only).  Drift scans: the device bytes of
// the fixed part and of each time of a group, and the times per group for a
// workspace of a quarter of the HBM budget (at least one).
struct DriftSizing {
    size_t per_time = 0, fixed = 0;
    int group = 1;
};
DriftSizing drift_sizing(int n_ant, int n_src, int n_freq, int n_time, size_t budget);
// Device bytes a request holds while it runs (inputs, outputs, target table
// and the workspace of its frequencies, which run in groups of at most cap
// bytes), given its geometry plan g (NUFFT) and the chosen dim and precision.
size_t footprint_bytes(const fv_problem &p, const GeomPlan &g, int dim, int prec, size_t cap);
void launch_frontend_count(const double *src_eq, int n_src, int n_time, const double *rot_dev, const double *flux,
                           int n_freq, int *bcnt, int *bbad, int *tot, hipStream_t st);
void launch_frontend(const double *src_eq, int n_src, int n_time, const double *rot_dev, const double *flux,
                     int n_freq, const double *kbeam_dev, bool unit_beam, const int *boff, const int *tot, double *dir,
                     long long dir_stride, double *str, long long str_stride, hipStream_t st);

// Direct sums.
void launch_direct(const double *ant_dev, int n_ant, const double *src_dev, int n_src, const double *freq_host,
                   int n_freq, const double *flux_dev, const double *beam_dev, int dim, int prec_bits,
                   double *vis_dev, hipStream_t s, StageTimer *timer = nullptr);
// Matrix-core direct sum V = Z diag(c) Z^H.  The workspace holds Z for a chunk
// of sources sized so that the total stays within `cap` bytes.
// Matrix-core direct form (zz.hip): tiles of kZTile antennas, the source
// axis split over kTargetWaves wavefronts per frequency (at least kFoldSrc
// sources each, kWavesPerBlock splits per workgroup), the sources in chunks
// whose Z fits the workspace cap with the partial tiles.
constexpr int kZTile = 32;          // antennas per tile edge (one wavefront: 2 x 2 MFMA tiles)
constexpr int kFoldSrc = 128;       // FP32 mode: sources per FP32 partial sum
constexpr int kWavesPerBlock = 4;   // splits of one tile pair per block
constexpr int kTargetWaves = 8192;  // wavefronts per frequency the split count aims for
struct ZZShape {
    int na_pad, ntile, ntp, nsplit;
    int kc_pad;          // sources per chunk, padded to a multiple of 4
    size_t z_bytes, c_bytes, part_bytes;
};
ZZShape zz_shape(int n_ant, int n_src, int prec_bits, size_t cap);  // sizing.cpp
size_t zz_work_bytes(int n_ant, int n_src, int prec_bits, size_t cap);
void launch_zz(const double *ant_dev, int n_ant, const double *src_dev, int n_src, const double *freq_host,
               int n_freq, const double *flux_dev, const double *beam_dev, int dim, int prec_bits, double *vis_dev,
               void *work, size_t cap, hipStream_t s, StageTimer *timer = nullptr);

}  // namespace fv
