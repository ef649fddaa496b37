// Step-kernel instantiations: launch_f32_plain, launch_f32_plain_c.
#define PD_STEP_LAUNCH_IMPL
#include "step_launch.h"

namespace pdmi {

void launch_f32_plain(int shape, bool plane, dim3 grid, hipStream_t st, const StepParams<float> &a)
{
    launch_shape<float, false, false>(shape, plane, grid, st, a);
}

void launch_f32_plain_c(int shape, bool plane, dim3 grid, hipStream_t st, const StepParams<float> &a)
{
    launch_shape<float, false, true>(shape, plane, grid, st, a);
}

}  // namespace pdmi
