// sigk_bwd.hip -- adjoint (reverse wavefront) kernels.  Placeholder until the
// adjoint sweep lands: every launcher reports "not supported".
#include "sigk_strip.h"

#ifndef SIGK_P
#define SIGK_P 8
#endif
#ifndef SIGK_D
#define SIGK_D 8
#endif

namespace sigk {
#define SIGK_CAT3(a, b, c) a##b##_##c
#define SIGK_NAME(pre, P, D) SIGK_CAT3(pre, P, D)
hipError_t SIGK_NAME(launch_ckpt_, SIGK_P, SIGK_D)(const FwdArgs&, int, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t SIGK_NAME(launch_bwd_, SIGK_P, SIGK_D)(const BwdArgs&, int, hipStream_t) {
    return hipErrorNotSupported;
}
int SIGK_NAME(occupancy_bwd_, SIGK_P, SIGK_D)() { return 1; }
}  // namespace sigk
