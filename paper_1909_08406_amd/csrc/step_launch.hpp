// Launch description of one collide-and-stream step and the launchers of
// the step kernels, one per storage form and rounding mode. Each launcher
// lives in its own translation unit (step_*.hip), so the many template
// instances of the step kernel compile in parallel; the host side of the
// library (lbm.hip) fills a StepLaunch and calls the launcher of its form.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"

namespace lbm {

// Block sizes of the step-kernel variants; the batched launch keeps one
// (box, tile) list per block size.
constexpr int NBLK = 4;
constexpr int BLK_SIZES[NBLK] = {128, 256, 512, 1024};
constexpr int blk_index(int blk) { return blk == 128 ? 0 : blk == 256 ? 1 : blk == 512 ? 2 : 3; }

// Cache-policy hints of a variant.
constexpr int FL_NT_LOAD = 1;   // non-temporal loads (streamed once)
constexpr int FL_NT_STORE = 2;  // non-temporal stores
// Stage each tile's source rows in LDS (k_step_lds): 16-bit storage, per-box
// launches of boxes whose x-rows hold whole tiles; elsewhere the variant
// runs the plain kernel of its block size.
constexpr int FL_LDS = 4;

// Step-kernel launch variants: block size and cache-policy hints. Every
// variant computes the same per-node arithmetic.
struct VariantDesc {
    int blk;
    int fl;
};
constexpr VariantDesc VARIANTS[] = {
    {256, 0}, {256, FL_NT_LOAD | FL_NT_STORE}, {512, 0}, {128, 0}, {256, FL_NT_STORE}, {1024, 0}, {256, FL_LDS},
};
constexpr int NVARIANTS = int(sizeof(VARIANTS) / sizeof(VARIANTS[0]));

struct BatchBox;

// Everything one step launch needs. Pointers are device pointers unless
// noted; the per-box arrays are host arrays of nboxes entries.
struct StepLaunch {
    const void* in;          // current population buffer (all boxes)
    void* out;               // the other buffer
    int newton;              // Newton steps of the equilibrium solve, 1..4
    int schedule;            // LBM_SCHEDULE_PER_BOX (0) or LBM_SCHEDULE_BATCHED (1)
    int variant;             // 0 .. NVARIANTS-1 (energy-conserving model only)
    uint32_t model;          // MODEL_* bits
    uint32_t xcd_remap;      // group consecutive tiles per XCD
    uint32_t step;           // step count seeding the stochastic rounding
    const uint32_t* step_base;  // device counter added to step (graph replays), or null
    hipStream_t stream;
    // batched schedule
    const BatchBox* table;   // per-box parameters
    const uint2* tiles[NBLK];  // (box, tile) lists per block size
    uint64_t ntiles[NBLK];
    // per-box schedule (host arrays)
    int nboxes;
    const StepParams* params;  // kernel parameters of each box (step fields set by the launcher)
    const uint64_t* offset;    // element offset of each box in a buffer
    const uint64_t* nodes;     // nodes of each box
};

// Launchers: queue one step and return 0, or a negative lbm_error.
int enqueue_step_f64(const StepLaunch& L);
int enqueue_step_f32(const StepLaunch& L);
int enqueue_step_f32_sr(const StepLaunch& L);
int enqueue_step_f32s(const StepLaunch& L);
int enqueue_step_f16s(const StepLaunch& L);
int enqueue_step_f16s_sr(const StepLaunch& L);
int enqueue_step_bf16s(const StepLaunch& L);
int enqueue_step_bf16s_sr(const StepLaunch& L);

}  // namespace lbm
