// Launch of the planned FFT passes (fft_reg.h): one kernel per orientation
// (rows here, columns in fft_reg_cols.hip, which includes this file with
// FV_FFT_COLS 1, so that the two compile in parallel), whose workgroups pick
// their snapshot's compile-time plan by line length.
#include <hip/hip_ext.h>

#include "fft_reg.h"

#ifndef FV_FFT_COLS
#define FV_FFT_COLS 0
#endif
// the two orientations carry their own kernel names (so that profiles tell
// the passes apart)
#if FV_FFT_COLS
#define FV_FFT_KERNEL k_fft_cols
#define FV_FFT_TPB fftr::kTpbCols
#define FV_FFT_WAVES __attribute__((amdgpu_waves_per_eu(4)))
#else
#define FV_FFT_KERNEL k_fft_rows
#define FV_FFT_TPB fftr::kTpbRows
#define FV_FFT_WAVES
#endif

namespace fv {
namespace {

// Physical workgroup b runs on XCD b mod 8 (round-robin dispatch); logical
// workgroups are handed out so that each XCD gets one contiguous range (nblk a
// multiple of 8), and neighbouring line groups share an L2.
__device__ __forceinline__ long long xcd_order_reg(long long b, long long nblk) {
    return (b & 7) * (nblk >> 3) + (b >> 3);
}

// One workgroup per line group of one snapshot, numbered snapshot by snapshot
// (reg_base); the snapshot of a workgroup is found by binary search.
__global__ __launch_bounds__(FV_FFT_TPB) FV_FFT_WAVES void FV_FFT_KERNEL(const SnapDev *snaps, int n_snap, int a, float2 *grid,
                                                             long long n_wg) {
    extern __shared__ __align__(16) char smem[];
    const long long wl = xcd_order_reg((long long)blockIdx.x, (long long)gridDim.x);
    if (wl >= n_wg) return;
    int lo = 0, hi = n_snap - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (snaps[mid].reg_base[a] <= wl) lo = mid;
        else hi = mid - 1;
    }
    const SnapDev &S = snaps[lo];
    const long long w = wl - S.reg_base[a];
    switch (S.n1[a]) {
#define FV_FFT_PLAN(L, NL, LP, F1, F2, F3, F4, F5, F6)                                                 \
    case L:                                                                                           \
        fftr::run_plan<fftr::Plan<L, NL, LP, F1, F2, F3, F4, F5, F6, FV_FFT_TPB>, FV_FFT_COLS != 0>(S, a, w, grid, smem); \
        break;
#if FV_FFT_COLS
#include "fft_plans_cols.inc"
#else
#include "fft_plans_rows.inc"
#endif
#undef FV_FFT_PLAN
        default:
            break;
    }
}

}  // namespace

#if FV_FFT_COLS
void launch_fft_reg_cols(const SnapDev *snaps, int n_snap, int a, void *grid, long long n_wg, size_t lds,
                         hipStream_t st, hipEvent_t ea, hipEvent_t eb)
#else
void launch_fft_reg_rows(const SnapDev *snaps, int n_snap, int a, void *grid, long long n_wg, size_t lds,
                         hipStream_t st, hipEvent_t ea, hipEvent_t eb)
#endif
{
    static bool raised = false;
    if (!raised) {
        FV_HIP(hipFuncSetAttribute((const void *)FV_FFT_KERNEL, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
        raised = true;
    }
    if (n_wg <= 0) return;
    // a multiple of 8 workgroups, so that the XCD of workgroup b is b mod 8
    const unsigned gx = (unsigned)((n_wg + 7) / 8 * 8);
    float2 *g = (float2 *)grid;
    if (ea)
        hipExtLaunchKernelGGL(FV_FFT_KERNEL, dim3(gx), dim3(FV_FFT_TPB), (uint32_t)lds, st, ea, eb, 0u, snaps, n_snap,
                              a, g, n_wg);
    else
        hipLaunchKernelGGL(FV_FFT_KERNEL, dim3(gx), dim3(FV_FFT_TPB), lds, st, snaps, n_snap, a, g, n_wg);
    FV_HIP(hipGetLastError());
}

}  // namespace fv
