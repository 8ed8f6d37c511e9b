// Step kernels and launcher for FP16-shifted storage, stochastic rounding.
#include "step_tu.hpp"

LBM_DEFINE_STEP_LAUNCHER(enqueue_step_f16s_sr, StoreF16S, true)
