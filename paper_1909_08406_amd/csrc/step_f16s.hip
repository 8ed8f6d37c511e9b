// Step kernels and launcher for FP16-shifted storage, round to nearest.
#include "step_tu.hpp"

LBM_DEFINE_STEP_LAUNCHER(enqueue_step_f16s, StoreF16S, false)
