// The context object behind the opaque fv_ctx handle.
#pragma once

#include <condition_variable>
#include <deque>
#include <array>
#include <list>
#include <tuple>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "fv_internal.h"

namespace fv {

// Device pointers of one problem's inputs plus the host-side source box.
struct DevInputs {
    const double *ant = nullptr, *src = nullptr, *flux = nullptr, *beam = nullptr;
    const double *freq = nullptr;  // frequencies on the device
    double *vis = nullptr;
    double s_c[3] = {0, 0, 0}, S[3] = {0, 0, 0};
    // device input check's block partials (largest |flux beam| per flat range
    // of cmax_span values), or null
    const double *cmax = nullptr;
    long long cmax_span = 0;
};

// A stream with its own workspace and input arenas.
struct Slot {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    Arena arena;   // NUFFT workspace
    Arena inputs;  // uploaded inputs and the device output
    Arena lat;     // workspace of batched lattice launches
    PinnedBuf pin; // host staging of a device request's planning scalars
    StageTimer timer;
    GraphCache graphs;  // launch graphs captured on this slot's workspace
    // end of the last call's work on the caller's stream (device entry
    // point): the next call, on any stream, waits for it before it reuses the
    // workspace
    hipEvent_t done = nullptr;
    ~Slot();
};

struct Server;  // serving loop state (server.cpp)

}  // namespace fv

struct fv_ctx {
    int device = 0;
    size_t budget = 0;       // HBM budget in bytes
    size_t chunk_bytes = 0;  // NUFFT workspace cap per launch group
    fv::Slot main;
    fv::DevCache cache;
    std::mutex geo_mu;
    std::vector<std::pair<uint64_t, fv::GeomPlan>> geos;
    std::list<std::shared_ptr<fv::TargetTable>> targets;
    std::vector<std::pair<uint64_t, std::shared_ptr<fv::LatticePlan>>> lattices;  // null plan: not a lattice
    double *scalar_buf = nullptr;
    size_t scalar_cap = 0;  // doubles
    fv::PinnedBuf plan_pin;  // host staging of the planning scalars of fv_simulate_dev
    // The device entry point's last planning scalars, for calls that repeat its
    // arguments (same device pointers, sizes, eps and flags): the next such call
    // enqueues the last call's path (type 1 or type 3) right behind its input
    // check, planned on the last call's antenna positions, frequencies and
    // source box, while the host waits for the check; it then verifies those
    // (and the path choice) against the new check and recomputes on a mismatch.
    struct DevSpec {
        bool valid = false;
        const void *ptr[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // ant, freq, src, flux, beam
        int n_ant = 0, n_freq = 0, n_src = 0;
        double eps = 0;
        unsigned flags = 0;
        std::vector<double> ant, freq;
        double s_c[3] = {0, 0, 0}, S[3] = {0, 0, 0};
        bool lattice = false;  // the last call's path: type 1, else type 3 (whose plan follows the source box)
        int dim = 0;
        hipEvent_t ev = nullptr;  // the check's copy to the host
    } spec;
    // The same for fv_simulate_batch_dev: the last batch's arguments and each
    // problem's planning scalars (box: source box centre, half-width).
    struct BatchSpec {
        bool valid = false;
        std::vector<fv_problem> args;
        std::vector<double *> vis;
        std::vector<std::vector<double>> ant, freq;
        std::vector<std::array<double, 6>> box;
        std::vector<int> dim;
        hipEvent_t ev = nullptr;  // the check's copy to the host
    } bspec;
    // side stream of a repeated type-3 call's input check, and the event that
    // forks it from the caller's stream (default priority, like every stream)
    hipStream_t side = nullptr;
    hipEvent_t side_fork = nullptr;
    fv::TuneCache tunes;     // autotuned FFT launch shapes
    fv::Server *server = nullptr;  // owned; created by fv_server_start, freed by fv_server_stop
    double *scalars(size_t n_doubles) {
        if (n_doubles > scalar_cap) {
            if (scalar_buf) (void)hipFree(scalar_buf);
            scalar_buf = nullptr;
            scalar_cap = 0;
            FV_HIP(hipMalloc((void **)&scalar_buf, n_doubles * sizeof(double)));
            scalar_cap = n_doubles;
        }
        return scalar_buf;
    }
    ~fv_ctx();
};

namespace fv {

GeomPlan ctx_geometry(fv_ctx *ctx, const double *ant_host, int n_ant, int dim, double eps, const double *s_c,
                      const double *S, bool fold);
// Target table of an array (cached); with `scales`, all pairs at each of
// those frequency ratios of one snapshot (targets q n_pairs + t).
std::shared_ptr<TargetTable> ctx_targets(fv_ctx *ctx, const double *ant_host, const double *ant_dev,
                                         const GeomPlan &g, hipStream_t st,
                                         const std::vector<double> *scales = nullptr);
void validate_host(const fv_problem *p);
DevInputs upload(Slot &slot, const fv_problem *p, double *s_c, double *S);
void run_device(fv_ctx *ctx, Slot &slot, const fv_problem &host_meta, const DevInputs &in, double *vis_dev,
                fv_report *rep);
// Argument checks of a problem whose arrays are on the device.
void check_dev_args(const fv_problem &p, const double *vis);
// Host side of the device input check: hdr holds the 8 check values, the
// frequencies and the antenna positions (launch_validate's first doubles).
// Fails on invalid values; fills the host copies and the source box (centre,
// half-width per axis); returns the dimension choice.
int check_dev_scalars(const fv_problem &p, const double *hdr, std::vector<double> &ant, std::vector<double> &freq,
                      double box[6]);
// A problem with device arrays on `slot` (its stream, workspaces and staging),
// blocking until done: the serving loop's device requests.
void simulate_dev_sync(fv_ctx *ctx, Slot &slot, const fv_problem &p, double *vis, fv_report *rep);

// Kernel family of a group of NUFFT jobs.
struct NufftGroupKey {
    int dim = 2, prec = 32, w = 8, fold_axis = -1;
    unsigned flags = 0;  // FV_AUTOTUNE | FV_GRAPH | FV_DETERMINISTIC of the problem
    bool operator<(const NufftGroupKey &o) const {
        return std::tie(dim, prec, w, flags) < std::tie(o.dim, o.prec, o.w, o.flags);
    }
};
NufftGroupKey append_jobs(fv_ctx *ctx, const fv_problem &p, const DevInputs &in, double *vis_dev, hipStream_t st,
                          std::vector<SnapJob> &jobs, std::vector<std::shared_ptr<TargetTable>> &hold,
                          SnapPlan *top);
double execute_jobs(fv_ctx *ctx, Slot &slot, const std::vector<SnapJob> &jobs, const NufftGroupKey &k,
                    StageTimer *tm);
void run_direct(fv_ctx *ctx, Slot &slot, const fv_problem &p, const DevInputs &in, double *vis_dev, int dim,
                int prec, StageTimer *tm);
void fill_report(StageTimer &tm, fv_report &r);
// Adds the stage times, bytes, launches and pairs of one sub-call's report to
// r (the first sub-call's report is copied whole).
void accumulate_report(const fv_report &a, fv_report &r, bool first);
// n_vec transforms of one geometry (all arrays on the device), the v-th with
// strengths flux * prod[v] (or prod[v] alone when flux is null), into tmp + v
// [n_freq][n_pairs] complex, run as one batch (each stage one launch over
// every vector and frequency); one input check per vector and one wait for
// all their planning scalars.  `total` is the batch's report.
void run_vectors(fv_ctx *ctx, Slot &slot, hipStream_t st, const double *ant_dev, int n_ant, const double *src_dev,
                 int n_src, const double *freq_dev, int n_freq, double eps, unsigned flags, const double *flux,
                 const double *prod, int n_vec, double *tmp, fv_report &total);
// Lattice plan of an array (cached per array, tolerance and kernel width, with
// its deconvolution tables for that width), null when the
// East/North positions are not a lattice within tol metres.
std::shared_ptr<LatticePlan> ctx_lattice(fv_ctx *ctx, const double *ant_host, int n_ant, double tol, int w);
// The lattice plan and kernel width when the type-1 path should run for this
// problem (lattice array, fine grid no larger than the type-3 grid at the top
// frequency for the source box in `in`), else null.
std::shared_ptr<LatticePlan> lattice_choice(fv_ctx *ctx, const fv_problem &p, const DevInputs &in, int prec,
                                            int *w_out);
// The type-1 path (paper section 2.2.1) for a coplanar problem when its
// antennas form a lattice and its fine grid is the smaller one; false when
// the type-3 path should run instead.
bool run_lattice(fv_ctx *ctx, Slot &slot, const fv_problem &p, const DevInputs &in, double *vis_dev, int prec,
                 StageTimer *tm, fv_report &r);
void simulate_host(fv_ctx *ctx, Slot &slot, const fv_problem *p, double *vis, fv_report *rep);
void server_free(Server *s);  // stops the workers (cancelling queued requests) and frees
// src_on_host false: the source box is taken as the whole direction cube (a
// device request, whose directions the host does not hold).
size_t request_footprint(fv_ctx *ctx, const fv_problem &p, bool src_on_host = true);
void simulate_batch(fv_ctx *ctx, Slot &slot, int n, const fv_problem *ps, double *const *vis, fv_report *rep);
// Problems whose inputs are on the device: meta[i] holds host copies of the
// antenna positions and frequencies, in[i] the device arrays, source box and
// input-check partials.  Enqueues every problem's work on slot.stream with no
// host wait between problems.
// lattice_used (nullable) receives, per problem, whether it took the type-1 path.
void run_batch_device(fv_ctx *ctx, Slot &slot, int n, const fv_problem *meta, const DevInputs *in, fv_report &r,
                      std::vector<char> *lattice_used);
const char *last_error_cstr();
void set_last_error(const std::string &msg);

// Stage outputs of a single snapshot for the diagnostic entry point
// (complex128, host): the deconvolved spreading grid and the pruned FFT output.
void nufft_debug(const SnapJob &job, int dim, int prec_bits, int w, Arena &arena, DevCache &cache, double *spread,
                 double *fftout, hipStream_t s);

}  // namespace fv
