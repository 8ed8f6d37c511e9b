// Step kernels and launcher for FP64 storage.
#include "step_tu.hpp"

LBM_DEFINE_STEP_LAUNCHER(enqueue_step_f64, StoreF64, false)
