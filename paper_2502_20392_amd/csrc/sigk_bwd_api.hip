// sigk_bwd_api.hip -- host side of the adjoint entry point.
#include <hip/hip_runtime.h>
#include "../../include/sigk.h"
#include "sigk_internal.h"
struct sigk_plan;
int sigk_plan_backward_impl(const sigk_plan*, const double*, const double*, double*, void*,
                            size_t, void*) {
    return SIGK_EUNSUPPORTED;
}
