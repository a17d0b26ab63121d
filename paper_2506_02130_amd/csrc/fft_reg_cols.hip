// The column (non-contiguous) orientation of the planned FFT pass; see fft_reg.hip.
#define FV_FFT_COLS 1
#include "fft_reg.hip"
