// Discrete adjoint of the explicit solve (peak reaction w.r.t. the per-node
// limit-stretch and micromodulus fields).
#include <hip/hip_runtime.h>

#include "pd_internal.h"

using namespace pdmi;

extern "C" {

int pd_qoi_grad(pd_mesh m, const pd_params *p, const double *s0_dev, const double *c_dev, double *dq_ds0_dev,
                double *dq_dc_dev, double *peak_out, int64_t *peak_step_out, void *stream)
{
    (void)s0_dev; (void)c_dev; (void)dq_ds0_dev; (void)dq_dc_dev; (void)peak_out; (void)peak_step_out; (void)stream;
    if (!m || !p) return fail(PD_EINVAL, "null argument");
    return fail(PD_ESTATE, "the adjoint is not available in this build");
}

}  // extern "C"
