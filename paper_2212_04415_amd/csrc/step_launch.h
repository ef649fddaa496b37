// Launches of the step kernel for each launch shape.  The kernel
// instantiations are spread over several translation units (one per
// precision / accumulation / micromodulus combination) so they compile in
// parallel; each defines one of the functions declared at the end.
#pragma once

#include <hip/hip_runtime.h>

#include "pd_internal.h"
#include "step_kernels.h"

namespace pdmi {

// A block copies the stencil's slot table into LDS one entry per thread, so
// every launch shape below needs at least kStencil threads per block; with
// fewer, the exception pass would decode unset entries into offsets outside
// the padded grid.
template <typename... BR>
constexpr bool blocks_fill_slot_table()
{
    return ((BR::N >= kStencil) && ...);
}
static_assert(blocks_fill_slot_table<Brick<16, 4, 4, 2>, Brick<8, 8, 4>, Brick<12, 4, 4>, Brick<256, 1, 1>,
                                     PlaneBrick<64, 4>, PlaneBrick<32, 8>, PlaneBrick<32, 4>, PlaneBrick<256, 1>>(),
              "a launch shape's block is smaller than the slot table it fills");

#ifdef PD_STEP_LAUNCH_IMPL
template <typename T, bool KAHAN, bool HAS_C>
static void launch_shape(int shape, bool plane, dim3 grid, hipStream_t st, const StepParams<T> &a)
{
    if (plane) {
        if constexpr (sizeof(T) == 4 && KAHAN) {
            switch (shape) {
            case PD_SHAPE_LDS_16x4x4: step_kernel<T, KAHAN, HAS_C, true, PlaneBrick<64, 4>><<<grid, 256, 0, st>>>(a); return;
            case PD_SHAPE_LDS_8x8x4: step_kernel<T, KAHAN, HAS_C, true, PlaneBrick<32, 8>><<<grid, 256, 0, st>>>(a); return;
            case PD_SHAPE_LDS_12x4x4: step_kernel<T, KAHAN, HAS_C, true, PlaneBrick<32, 4>><<<grid, 128, 0, st>>>(a); return;
            default: break;
            }
        } else if constexpr (sizeof(T) == 4) {
            if (shape == PD_SHAPE_LDS_16x4x4) {
                step_kernel<T, KAHAN, HAS_C, true, PlaneBrick<64, 4>><<<grid, 256, 0, st>>>(a);
                return;
            }
        }
        step_kernel<T, KAHAN, HAS_C, false, PlaneBrick<256, 1>><<<grid, 256, 0, st>>>(a);
        return;
    }
    if constexpr (sizeof(T) == 4 && KAHAN) {
        switch (shape) {
        case PD_SHAPE_LDS_16x4x4: step_kernel<T, KAHAN, HAS_C, true, Brick<16, 4, 4, 2>><<<grid, 256, 0, st>>>(a); return;
        case PD_SHAPE_LDS_8x8x4: step_kernel<T, KAHAN, HAS_C, true, Brick<8, 8, 4>><<<grid, 256, 0, st>>>(a); return;
        case PD_SHAPE_LDS_12x4x4: step_kernel<T, KAHAN, HAS_C, true, Brick<12, 4, 4>><<<grid, 192, 0, st>>>(a); return;
        default: break;
        }
    } else if constexpr (sizeof(T) == 4) {
        if (shape == PD_SHAPE_LDS_16x4x4) {
            step_kernel<T, KAHAN, HAS_C, true, Brick<16, 4, 4, 2>><<<grid, 256, 0, st>>>(a);
            return;
        }
    }
    step_kernel<T, KAHAN, HAS_C, false, Brick<256, 1, 1>><<<grid, 256, 0, st>>>(a);
}

// The same choice for the several-solve tick kernel (FP32 compensated
// accumulation, 3D meshes).
template <bool HAS_C>
static void launch_tick_shape(int shape, dim3 grid, hipStream_t st, const TickParams<float> &m)
{
    switch (shape) {
    case PD_SHAPE_LDS_16x4x4: step_kernel_tick<float, true, HAS_C, true, Brick<16, 4, 4, 2>><<<grid, 256, 0, st>>>(m); return;
    case PD_SHAPE_LDS_8x8x4: step_kernel_tick<float, true, HAS_C, true, Brick<8, 8, 4>><<<grid, 256, 0, st>>>(m); return;
    case PD_SHAPE_LDS_12x4x4: step_kernel_tick<float, true, HAS_C, true, Brick<12, 4, 4>><<<grid, 192, 0, st>>>(m); return;
    default: step_kernel_tick<float, true, HAS_C, false, Brick<256, 1, 1>><<<grid, 256, 0, st>>>(m); return;
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
