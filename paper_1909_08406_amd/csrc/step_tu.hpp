// Body of a step launcher (included by the step_*.hip translation units):
// picks the kernel instance for the launch's Newton count, equilibrium
// model, launch variant and schedule, for storage ST and rounding SR.
#pragma once

#include <type_traits>

#include "kernels.hpp"
#include "step_launch.hpp"

namespace lbm {

template <class F>
inline int step_with_variant(int v, F&& f)
{
    using std::integral_constant;
    switch (v) {
        case 0: f(integral_constant<int, 256>{}, integral_constant<int, 0>{}); break;
        case 1: f(integral_constant<int, 256>{}, integral_constant<int, FL_NT_LOAD | FL_NT_STORE>{}); break;
        case 2: f(integral_constant<int, 512>{}, integral_constant<int, 0>{}); break;
        case 3: f(integral_constant<int, 128>{}, integral_constant<int, 0>{}); break;
        case 4: f(integral_constant<int, 256>{}, integral_constant<int, FL_NT_STORE>{}); break;
        case 5: f(integral_constant<int, 1024>{}, integral_constant<int, 0>{}); break;
        case 6: f(integral_constant<int, 256>{}, integral_constant<int, FL_LDS>{}); break;
        default: return -1;
    }
    return 0;
}

template <class F>
inline int step_with_newton(int n, F&& f)
{
    using std::integral_constant;
    switch (n) {
        case 1: return f(integral_constant<int, 1>{});
        case 2: return f(integral_constant<int, 2>{});
        case 3: return f(integral_constant<int, 3>{});
        case 4: return f(integral_constant<int, 4>{});
        default: return -1;
    }
}

template <class ST, bool SR>
int enqueue_step_impl(const StepLaunch& L)
{
    using T = typename ST::T;
    const T* in = reinterpret_cast<const T*>(L.in);
    T* out = reinterpret_cast<T*>(L.out);
    return step_with_newton(L.newton, [&](auto nw) -> int {
        constexpr int NEWTON = decltype(nw)::value;
        auto launch = [&](auto model, auto blk, auto fl) {
            constexpr int MODEL = decltype(model)::value;
            constexpr int BLK = decltype(blk)::value;
            constexpr int FL = decltype(fl)::value;
            constexpr int FLP = FL & ~FL_LDS;  // the plain kernel's hints
            if (L.schedule == 1) {
                const int i = blk_index(BLK);
                hipLaunchKernelGGL((k_step_batch<ST, NEWTON, BLK, FLP, SR, MODEL>), dim3(uint32_t(L.ntiles[i])),
                                   dim3(BLK), 0, L.stream, in, out, L.table, L.tiles[i], L.xcd_remap, L.step,
                                   L.step_base);
            } else {
                for (int b = 0; b < L.nboxes; ++b) {
                    StepParams p = L.params[b];
                    p.step = L.step;
                    p.step_base = L.step_base;
                    p.xcd_remap = L.xcd_remap;
                    const dim3 grid(uint32_t((L.nodes[b] + BLK - 1) / BLK));
                    if constexpr ((FL & FL_LDS) != 0 && sizeof(T) == 2 && (MODEL & MODEL_WALLS) == 0) {
                        // whole tiles per x-row (the grid then has no ragged tile)
                        if (p.g.nx % BLK == 0) {
                            hipLaunchKernelGGL((k_step_lds<ST, NEWTON, BLK, FL, SR, MODEL>), grid, dim3(BLK), 0,
                                               L.stream, in + L.offset[b], out + L.offset[b], p);
                            continue;
                        }
                    }
                    hipLaunchKernelGGL((k_step<ST, NEWTON, BLK, FLP, SR, MODEL>), grid, dim3(BLK), 0, L.stream,
                                       in + L.offset[b], out + L.offset[b], p);
                }
            }
        };
        using std::integral_constant;
        if (L.model != MODEL_E2) {
            // the other models run the default launch shape
            const integral_constant<int, 256> blk;
            const integral_constant<int, 0> fl;
            switch (L.model) {
                case MODEL_ISO: launch(integral_constant<int, MODEL_ISO>{}, blk, fl); break;
                case MODEL_SERIES: launch(integral_constant<int, MODEL_SERIES>{}, blk, fl); break;
                case MODEL_E2 | MODEL_ENTROPIC: launch(integral_constant<int, MODEL_E2 | MODEL_ENTROPIC>{}, blk, fl); break;
                case MODEL_ISO | MODEL_ENTROPIC:
                    launch(integral_constant<int, MODEL_ISO | MODEL_ENTROPIC>{}, blk, fl);
                    break;
                case MODEL_E2 | MODEL_WALLS: launch(integral_constant<int, MODEL_E2 | MODEL_WALLS>{}, blk, fl); break;
                case MODEL_ISO | MODEL_WALLS: launch(integral_constant<int, MODEL_ISO | MODEL_WALLS>{}, blk, fl); break;
                case MODEL_E2 | MODEL_ENTROPIC | MODEL_WALLS:
                    launch(integral_constant<int, MODEL_E2 | MODEL_ENTROPIC | MODEL_WALLS>{}, blk, fl);
                    break;
                case MODEL_ISO | MODEL_ENTROPIC | MODEL_WALLS:
                    launch(integral_constant<int, MODEL_ISO | MODEL_ENTROPIC | MODEL_WALLS>{}, blk, fl);
                    break;
                default: return -1;  // LBM_E_ARG
            }
        } else if (step_with_variant(L.variant, [&](auto blk, auto fl) {
                       launch(integral_constant<int, MODEL_E2>{}, blk, fl);
                   }) != 0) {
            return -1;  // LBM_E_ARG
        }
        return hipGetLastError() == hipSuccess ? 0 : -5;  // LBM_E_HIP
    });
}

}  // namespace lbm

// One launcher definition per translation unit.
#define LBM_DEFINE_STEP_LAUNCHER(NAME, STORE, SR) \
    namespace lbm {                               \
    int NAME(const StepLaunch& L) { return enqueue_step_impl<STORE, SR>(L); } \
    }
