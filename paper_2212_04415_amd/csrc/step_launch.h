// Launches of the step kernel for each launch shape.  The kernel
// instantiations are spread over several translation units (one per
// precision / accumulation / micromodulus combination) so they compile in
// parallel; each defines one of the functions declared at the end.
#pragma once

#include <hip/hip_runtime.h>

#include "pd_internal.h"
#include "step_kernels.h"

namespace pdmi {

#ifdef PD_STEP_LAUNCH_IMPL
// Every step launch goes through these two helpers: the block has one thread
// per node of the brick (BR::N), and it must have at least kStencil threads,
// since a block copies the stencil's slot table into LDS one entry per
// thread; with fewer, the exception pass would decode unset entries into
// offsets outside the padded grid.
template <typename T, bool KAHAN, bool HAS_C, bool LDS, typename BR>
static void launch_step(dim3 grid, hipStream_t st, const StepParams<T> &a)
{
    static_assert(BR::N >= kStencil, "a launch shape's block is smaller than the slot table it fills");
    step_kernel<T, KAHAN, HAS_C, LDS, BR><<<grid, BR::N, 0, st>>>(a);
}

template <bool HAS_C, bool LDS, typename BR>
static void launch_tick(dim3 grid, hipStream_t st, const TickParams<float> &m)
{
    static_assert(BR::N >= kStencil, "a launch shape's block is smaller than the slot table it fills");
    step_kernel_tick<float, true, HAS_C, LDS, BR><<<grid, BR::N, 0, st>>>(m);
}

template <typename T, bool KAHAN, bool HAS_C>
static void launch_shape(int shape, bool plane, dim3 grid, hipStream_t st, const StepParams<T> &a)
{
    if (plane) {
        if constexpr (sizeof(T) == 4 && KAHAN) {
            switch (shape) {
            case PD_SHAPE_LDS_16x4x4: launch_step<T, KAHAN, HAS_C, true, PlaneBrick<64, 4>>(grid, st, a); return;
            case PD_SHAPE_LDS_8x8x4: launch_step<T, KAHAN, HAS_C, true, PlaneBrick<32, 8>>(grid, st, a); return;
            case PD_SHAPE_LDS_12x4x4: launch_step<T, KAHAN, HAS_C, true, PlaneBrick<32, 4>>(grid, st, a); return;
            default: break;
            }
        } else if constexpr (sizeof(T) == 4) {
            if (shape == PD_SHAPE_LDS_16x4x4) {
                launch_step<T, KAHAN, HAS_C, true, PlaneBrick<64, 4>>(grid, st, a);
                return;
            }
        }
        launch_step<T, KAHAN, HAS_C, false, PlaneBrick<256, 1>>(grid, st, a);
        return;
    }
    if constexpr (sizeof(T) == 4 && KAHAN) {
        switch (shape) {
        case PD_SHAPE_LDS_16x4x4: launch_step<T, KAHAN, HAS_C, true, Brick<16, 4, 4, 2>>(grid, st, a); return;
        case PD_SHAPE_LDS_8x8x4: launch_step<T, KAHAN, HAS_C, true, Brick<8, 8, 4>>(grid, st, a); return;
        case PD_SHAPE_LDS_12x4x4: launch_step<T, KAHAN, HAS_C, true, Brick<12, 4, 4>>(grid, st, a); return;
        default: break;
        }
    } else if constexpr (sizeof(T) == 4) {
        if (shape == PD_SHAPE_LDS_16x4x4) {
            launch_step<T, KAHAN, HAS_C, true, Brick<16, 4, 4, 2>>(grid, st, a);
            return;
        }
    }
    launch_step<T, KAHAN, HAS_C, false, Brick<256, 1, 1>>(grid, st, a);
}

// The same choice for the several-solve tick kernel (FP32 compensated
// accumulation, 3D meshes).
template <bool HAS_C>
static void launch_tick_shape(int shape, dim3 grid, hipStream_t st, const TickParams<float> &m)
{
    switch (shape) {
    case PD_SHAPE_LDS_16x4x4: launch_tick<HAS_C, true, Brick<16, 4, 4, 2>>(grid, st, m); return;
    case PD_SHAPE_LDS_8x8x4: launch_tick<HAS_C, true, Brick<8, 8, 4>>(grid, st, m); return;
    case PD_SHAPE_LDS_12x4x4: launch_tick<HAS_C, true, Brick<12, 4, 4>>(grid, st, m); return;
    default: launch_tick<HAS_C, false, Brick<256, 1, 1>>(grid, st, m); return;
    }
}
#endif

// plane: the mesh is one node thick (PlaneBrick instantiations)
void launch_f32_kahan(int shape, bool plane, dim3 grid, hipStream_t st, const StepParams<float> &a);
void launch_f32_kahan_c(int shape, bool plane, dim3 grid, hipStream_t st, const StepParams<float> &a);
void launch_f32_plain(int shape, bool plane, dim3 grid, hipStream_t st, const StepParams<float> &a);
void launch_f32_plain_c(int shape, bool plane, dim3 grid, hipStream_t st, const StepParams<float> &a);
void launch_f64(int shape, bool plane, dim3 grid, hipStream_t st, const StepParams<double> &a);
void launch_f64_c(int shape, bool plane, dim3 grid, hipStream_t st, const StepParams<double> &a);
// one tick of several FP32 compensated 3D solves that share a launch shape
void launch_tick_f32_kahan(int shape, dim3 grid, hipStream_t st, const TickParams<float> &m);
void launch_tick_f32_kahan_c(int shape, dim3 grid, hipStream_t st, const TickParams<float> &m);

}  // namespace pdmi
