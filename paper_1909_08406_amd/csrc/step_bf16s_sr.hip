// Step kernels and launcher for BF16-shifted storage, stochastic rounding.
#include "step_tu.hpp"

LBM_DEFINE_STEP_LAUNCHER(enqueue_step_bf16s_sr, StoreBF16S, true)
