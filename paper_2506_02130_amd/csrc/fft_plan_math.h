// Sizes of a planned FFT pass (fft_reg.h) that the host needs too: the
// entries of a plan's twiddle rows and the LDS a workgroup of the plan holds.
// One definition for the kernels and the host table (fft_plans.cpp).
#pragma once
#include <cstddef>

namespace fv {
namespace fftr {

// Radices F[0..5] (1 past the last group): a middle group g has one row per
// k < p_g of F_g - 1 entries, the last group one row per butterfly of F
// entries; rows are padded to an odd stride.
constexpr int plan_groups(const int *F) {
    int G = 0;
    for (int g = 0; g < 6; ++g) G += F[g] > 1;
    return G;
}
constexpr long long plan_twiddle_entries(const int *F) {
    const int G = plan_groups(F);
    long long tot = 0, p = F[0];
    for (int g = 1; g < G; ++g) {
        const int W = g == G - 1 ? F[g] : F[g] - 1;
        const int S = W % 2 == 1 ? W : W + 1;
        tot += p * S;
        p *= F[g];
    }
    return tot;
}
// NL lines of stride LP (complex) and the twiddle rows, complex FP32
constexpr size_t plan_lds_bytes(int NL, int LP, const int *F) {
    return (size_t)((long long)NL * LP + plan_twiddle_entries(F)) * 8;
}

}  // namespace fftr
}  // namespace fv
