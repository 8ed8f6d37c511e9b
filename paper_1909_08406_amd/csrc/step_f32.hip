// Step kernels and launcher for FP32 storage, round to nearest.
#include "step_tu.hpp"

LBM_DEFINE_STEP_LAUNCHER(enqueue_step_f32, StoreF32, false)
