// Step-kernel instantiations: launch_f64, launch_f64_c.
#define PD_STEP_LAUNCH_IMPL
#include "step_launch.h"

namespace pdmi {

void launch_f64(int shape, bool plane, dim3 grid, hipStream_t st, const StepParams<double> &a)
{
    launch_shape<double, false, false>(shape, plane, grid, st, a);
}

void launch_f64_c(int shape, bool plane, dim3 grid, hipStream_t st, const StepParams<double> &a)
{
    launch_shape<double, false, true>(shape, plane, grid, st, a);
}

}  // namespace pdmi
