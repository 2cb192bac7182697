// Reverse-mode derivative of the binary64 push.
#include <hip/hip_runtime.h>

#include "../../include/gcb.h"
#include "gcb_internal.h"

extern "C" int gcb_push_backward(gcb_ctx*, const gcb_particles*, const gcb_params*, int32_t,
                                 const double* const[7], double* const[7], float* const[3],
                                 float* const[3], void*) {
    return GCB_EUNSUPPORTED;
}
