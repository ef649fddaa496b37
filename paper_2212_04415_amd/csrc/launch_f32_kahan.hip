// Step-kernel instantiations: launch_f32_kahan.
#define PD_STEP_LAUNCH_IMPL
#include "step_launch.h"

namespace pdmi {

void launch_f32_kahan(int shape, bool plane, dim3 grid, hipStream_t st, const StepParams<float> &a)
{
    launch_shape<float, true, false>(shape, plane, grid, st, a);
}

void launch_tick_f32_kahan(int shape, dim3 grid, hipStream_t st, const TickParams<float> &m)
{
    launch_tick_shape<false>(shape, grid, st, m);
}

}  // namespace pdmi
