// Push kernels of the mixed-precision form.
#include <hip/hip_runtime.h>

#include "gcb_internal.h"

namespace gcb {

hipError_t launch_push_mixed(const PushLaunch&, const ParticlePtrs<float>&,
                             const ParticlePtrs<float>&, const PushConst&, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace gcb
