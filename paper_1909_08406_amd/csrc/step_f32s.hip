// Step kernels and launcher for FP32-shifted storage.
#include "step_tu.hpp"

LBM_DEFINE_STEP_LAUNCHER(enqueue_step_f32s, StoreF32S, false)
