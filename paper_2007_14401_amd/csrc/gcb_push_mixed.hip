// Push kernels of the mixed form: binary32 fields and bulk arithmetic,
// binary64 positions and the selected quantities listed in gcb_math.hpp.
#include "gcb_push_kernels.hpp"

#ifndef GCB_TILED_MIN_WAVES_MIXED
#define GCB_TILED_MIN_WAVES_MIXED 4
#endif

namespace gcb {

hipError_t launch_push_mixed(const PushLaunch& L, const ParticlePtrs<float>& in,
                             const ParticlePtrs<float>& out, const PushConst& pc,
                             hipStream_t stream) {
    return kern::launch_push<float, float, GCB_TILED_MIN_WAVES_MIXED>(L, in, out, pc, stream);
}

}  // namespace gcb
