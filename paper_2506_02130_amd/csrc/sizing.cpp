// Workspace sizing of the library, host code only (no HIP calls), so that it
// can be built and checked with the address and undefined-behaviour
// sanitizers on a machine without a GPU: the type-3 workspace of a launch
// group, the matrix-core direct form's chunking, the drift scan's grouping of
// times, a serving request's footprint, and the FFT launch-shape defaults.
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "nufft_layout.h"

namespace fv {
using namespace detail;

size_t nufft_workspace_bytes(const std::vector<SnapJob> &jobs, int dim, int prec_bits, int w, bool det) {
    Layout L = make_layout(jobs, dim, prec_bits, w, Tuning::defaults(), det);
    return layout_bytes(L, dim, prec_bits, (int)jobs.size());
}

ZZShape zz_shape(int n_ant, int n_src, int prec_bits, size_t cap) {
    ZZShape s;
    s.na_pad = (n_ant + kZTile - 1) / kZTile * kZTile;
    s.ntile = s.na_pad / kZTile;
    s.ntp = s.ntile * (s.ntile + 1) / 2;
    const size_t csz = prec_bits == 32 ? 8 : 16, rsz = csz / 2;
    const int k_all = (std::max(n_src, 1) + 3) / 4 * 4;
    // splits: enough wavefronts to fill the chip, at least kFoldSrc sources
    // each, partials within half of the cap
    const size_t tile_bytes = (size_t)s.ntp * kZTile * kZTile * sizeof(double2);
    int ns = (kTargetWaves + s.ntp - 1) / s.ntp;
    ns = std::min(ns, std::max(1, k_all / kFoldSrc));
    ns = std::min<long long>(ns, std::max<long long>(kWavesPerBlock, (long long)(cap / 2 / tile_bytes)));
    s.nsplit = (ns + kWavesPerBlock - 1) / kWavesPerBlock * kWavesPerBlock;
    s.part_bytes = (size_t)s.nsplit * tile_bytes;
    // sources per chunk: Z and c of the chunk in the rest of the cap
    const size_t per_src = (size_t)s.na_pad * csz + rsz;
    size_t kc = k_all;
    const size_t rest = cap > s.part_bytes + 1024 ? cap - s.part_bytes - 1024 : 0;
    if ((size_t)k_all * per_src > rest) kc = std::max<size_t>(4 * kFoldSrc, rest / per_src / 4 * 4);
    s.kc_pad = (int)std::min<size_t>(kc, (size_t)k_all);
    s.z_bytes = (size_t)s.kc_pad * s.na_pad * csz;
    s.c_bytes = (size_t)s.kc_pad * rsz;
    return s;
}

size_t zz_work_bytes(int n_ant, int n_src, int prec_bits, size_t cap) {
    const ZZShape s = zz_shape(n_ant, n_src, prec_bits, cap);
    return (s.z_bytes + 255) / 256 * 256 + (s.c_bytes + 255) / 256 * 256 + s.part_bytes + 256;
}

int frontend_blocks(int n_src) { return (n_src + kFeBlock - 1) / kFeBlock; }

DriftSizing drift_sizing(int n_ant, int n_src, int n_freq, int n_time, size_t budget) {
    // per-time workspace: packed directions and strengths of the visible
    // sources, block offsets (at least 256 bytes, so that an empty sky still
    // divides)
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const int nb = frontend_blocks(n_src);
    DriftSizing z;
    z.per_time = std::max<size_t>(256, al(24 * (size_t)n_src) + al(8 * (size_t)n_freq * n_src) + al(4 * (size_t)nb));
    z.fixed = al(24 * (size_t)n_ant) + al(8 * (size_t)n_freq) * 2 + al(4 * (size_t)nb);
    const size_t cap = std::max<size_t>(budget / 4, z.per_time + z.fixed);
    z.group = (int)std::max<size_t>(1, std::min<size_t>({(size_t)std::max(n_time, 1), (cap - z.fixed) / z.per_time,
                                                         65535}));
    return z;
}

size_t footprint_bytes(const fv_problem &p, const GeomPlan &g, int dim, int prec, size_t cap) {
    const long long np = (long long)p.n_ant * (p.n_ant + 1) / 2;
    const size_t fs = 8 * (size_t)p.n_src * p.n_freq;
    size_t bytes = 24 * (size_t)p.n_ant + 24 * (size_t)p.n_src + fs * (p.beam ? 2 : 1) + 16 * (size_t)np * p.n_freq;
    if (p.n_src == 0) return bytes;
    const unsigned method = p.flags & FV_METHOD_MASK;
    if (method == FV_METHOD_DIRECT) return bytes;
    if (method == FV_METHOD_MFMA) return bytes + zz_work_bytes(p.n_ant, p.n_src, prec, cap);
    TargetTable tt;  // sizes only
    tt.n_tgt = np;
    tt.dim = dim;
    size_t ws = 0, ws_max = 0;
    for (int f = 0; f < p.n_freq; ++f) {
        SnapJob j;
        j.plan = plan_snapshot(g, p.freq_hz[f]);
        j.src = p.src_lmn;
        j.n_src = p.n_src;
        j.tt = &tt;
        const size_t b = nufft_workspace_bytes(std::vector<SnapJob>{j}, dim, prec, g.w,
                                               (p.flags & FV_DETERMINISTIC) != 0);
        ws += b;
        ws_max = std::max(ws_max, b);
    }
    ws = std::min(ws, std::max(cap, ws_max));  // frequencies run in groups of at most `cap`
    return bytes + ws + (size_t)np * (16 * (size_t)dim + 4);
}

static int env_or(const char *name, int dflt) {
    const char *e = std::getenv(name);
    return e ? std::atoi(e) : dflt;
}

Tuning Tuning::defaults() {
    static const Tuning t = [] {
        Tuning d;
        d.rows = std::max(1, std::min(16, env_or("FV_FFT_ROWS", d.rows)));
        d.lines = std::max(1, std::min(64, env_or("FV_FFT_MAX_LINES", d.lines)));
        d.tpb1 = env_or("FV_FFT_TPB1", d.tpb1);
        d.tpbm = env_or("FV_FFT_TPBM", d.tpbm);
        d.split = env_or("FV_FFT_SPLIT", d.split) ? 1 : 0;
        return d;
    }();
    return t;
}

int Tuning::tpb(int line_len, bool multi) const {
    int t = multi ? tpbm : tpb1;
    if (t != 128 && t != 256 && t != 512 && t != 1024) t = 0;
    if (t == 0) t = line_len <= 2048 ? 256 : (line_len <= 4096 ? 512 : 1024);
    return t;
}

}  // namespace fv
