// Host table of the planned FFT passes: which line lengths have a plan, its
// lines per workgroup and LDS bytes (from fft_plans_rows.inc and
// fft_plans_cols.inc, the same tables the kernels are built from).
#include "fft_plan_math.h"
#include "fv_internal.h"

namespace fv {
namespace {
struct PlanInfo {
    int L, NL;
    size_t lds;
};
#define FV_FFT_PLAN(L, NL, LP, F1, F2, F3, F4, F5, F6) \
    {L, NL, fftr::plan_lds_bytes(NL, LP, (const int[6]){F1, F2, F3, F4, F5, F6})},
const PlanInfo kRows[] = {
#include "fft_plans_rows.inc"
};
const PlanInfo kCols[] = {
#include "fft_plans_cols.inc"
};
#undef FV_FFT_PLAN

template <size_t N>
bool lookup(const PlanInfo (&t)[N], int L, int *nl, size_t *lds) {
    for (const PlanInfo &p : t)
        if (p.L == L) {
            *nl = p.NL;
            *lds = p.lds;
            return true;
        }
    return false;
}
}  // namespace

bool fft_reg_info(int L, bool cols, int *lines_per_wg, size_t *lds_bytes) {
    return cols ? lookup(kCols, L, lines_per_wg, lds_bytes) : lookup(kRows, L, lines_per_wg, lds_bytes);
}

}  // namespace fv
