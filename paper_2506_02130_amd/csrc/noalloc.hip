// Allocation-free variant of the device entry point for the matrix-core
// direct form V = Z diag(c) Z^H (paper section 5.1).  Every device buffer the
// call needs beyond the caller's inputs and output -- the input check's
// partials and planning scalars, the Z chunk, the strengths and the per-split
// partial tiles -- lives in one file-scope device array, so the call makes no
// device or pinned allocation.  Each device holds its own copy of the array
// (at its own address) until the process ends; calls on one device share it,
// so calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "fv.h"
#include "fv_internal.h"

namespace fv {
namespace {

constexpr size_t kScratchBytes = 64ull << 20;  // per device
constexpr int kMaxDevices = 64;
constexpr int kNoAllocMaxAnt = 1024;
constexpr int kNoAllocMaxFreq = 1024;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device with that device current (in host code the array's name is not a
// device address).
char *scratch_ptr(int dev) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        FV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(FV_EDEVICE, "no device address for the scratch array");
        g_ptr[dev] = p;
    }
    return (char *)g_ptr[dev];
}

// Host copy of the planning scalars: [check 8][freq][ant], per thread.
thread_local double t_scal[8 + kNoAllocMaxFreq + 3 * kNoAllocMaxAnt];

}  // namespace
}  // namespace fv

extern "C" fv_status fv_simulate_mfma_noalloc(const fv_problem *p, double *vis, void *stream) {
    try {
        if (!p || !vis) fv::fail(FV_EINVAL, "null argument");
        if ((uintptr_t)vis & 15) fv::fail(FV_EINVAL, "the output must be 16-byte aligned");
        if (p->n_ant < 1 || p->n_src < 0 || p->n_freq < 1) fv::fail(FV_EINVAL, "bad sizes");
        if (p->n_ant > fv::kNoAllocMaxAnt || p->n_freq > fv::kNoAllocMaxFreq)
            fv::fail(FV_EINVAL, "n_ant or n_freq above the allocation-free maximum (1024 each)");
        if (!p->ant_enu || !p->freq_hz || (p->n_src > 0 && (!p->src_lmn || !p->flux)))
            fv::fail(FV_EINVAL, "null device array");
        if (!(p->eps >= 1e-14 && p->eps <= 1e-1)) fv::fail(FV_EINVAL, "eps out of [1e-14, 1e-1]");
        const unsigned method = p->flags & FV_METHOD_MASK;
        if (method != FV_METHOD_MFMA) fv::fail(FV_EINVAL, "the allocation-free call runs FV_METHOD_MFMA only");
        if ((p->flags & FV_PREC_MASK) == FV_PREC_FP32 && p->eps < 1e-6)
            fv::fail(FV_EUNSUPPORTED, "FP32 needs eps >= 1e-6");
        int dev = 0;
        FV_HIP(hipGetDevice(&dev));
        if (dev < 0 || dev >= fv::kMaxDevices) fv::fail(FV_EDEVICE, "device index out of range");
        char *base = fv::scratch_ptr(dev);
        hipStream_t st = (hipStream_t)stream;
        // region 1: the input check (partials, then the planning scalars)
        const size_t nval = fv::validate_doubles(p->n_ant, p->n_freq);
        const size_t val_bytes = (nval * sizeof(double) + 255) / 256 * 256;
        double *val = (double *)base;
        fv::launch_validate(p->src_lmn, p->n_src, p->flux, p->beam, p->n_freq, p->ant_enu, p->n_ant, p->freq_hz, val,
                            st);
        const size_t nscal = 8 + (size_t)p->n_freq + 3 * (size_t)p->n_ant;
        double *h = fv::t_scal;
        FV_HIP(hipMemcpyAsync(h, val, nscal * sizeof(double), hipMemcpyDeviceToHost, st));
        FV_HIP(hipStreamSynchronize(st));
        const double *freq = h + 8, *ant = freq + p->n_freq;
        for (size_t i = 0; i < 3 * (size_t)p->n_ant; ++i)
            if (!std::isfinite(ant[i])) fv::fail(FV_EINVAL, "non-finite antenna position");
        for (int f = 0; f < p->n_freq; ++f)
            if (!(std::isfinite(freq[f]) && freq[f] > 0)) fv::fail(FV_EINVAL, "frequency must be finite and > 0");
        if (p->n_src > 0 && (h[6] != 0.0 || h[7] != 0.0)) fv::fail(FV_EINVAL, "invalid source directions or strengths");
        const long long n_pairs = (long long)p->n_ant * (p->n_ant + 1) / 2;
        if (p->n_src == 0) {
            fv::launch_zero_c128(vis, n_pairs * p->n_freq, st);
            return FV_OK;
        }
        const int dim = fv::choose_dim(ant, p->n_ant, p->eps, freq, p->n_freq, p->flags);
        const int prec = fv::choose_prec(p->eps, p->flags);
        // region 2: the Z chunk, its strengths and the partial tiles, chunked
        // over the sources to fit what is left of the array
        const size_t cap = fv::kScratchBytes - val_bytes;
        if (fv::zz_work_bytes(p->n_ant, p->n_src, prec, cap) > cap)
            fv::fail(FV_EINVAL, "the problem's partial tiles exceed the allocation-free scratch");
        fv::launch_zz(p->ant_enu, p->n_ant, p->src_lmn, p->n_src, freq, p->n_freq, p->flux, p->beam, dim, prec, vis,
                      base + val_bytes, cap, st, nullptr);
        return FV_OK;
    } catch (const fv::Error &e) {
        fv::set_last_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        fv::set_last_error(e.what());
        return FV_EDEVICE;
    }
}
