// Step kernels and launcher for BF16-shifted storage, round to nearest.
#include "step_tu.hpp"

LBM_DEFINE_STEP_LAUNCHER(enqueue_step_bf16s, StoreBF16S, false)
