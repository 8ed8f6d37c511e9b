// Step kernels and launcher for FP32 storage, stochastic rounding.
#include "step_tu.hpp"

LBM_DEFINE_STEP_LAUNCHER(enqueue_step_f32_sr, StoreF32, true)
