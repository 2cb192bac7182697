// 3D push kernels of the mixed form: binary32 fields and bulk arithmetic,
// binary64 positions and the selected quantities listed in gcb_math.hpp.
#include "gcb_push3_kernels.hpp"

#ifndef GCB_TILED3_MIN_WAVES_MIXED
#define GCB_TILED3_MIN_WAVES_MIXED 4
#endif

namespace gcb {

hipError_t launch_push3_mixed(const Push3Launch& L, const ParticlePtrs3<float>& in,
                              const ParticlePtrs3<float>& out, const PushConst3& pc,
                              hipStream_t stream) {
    return kern::launch_push3<float, float, GCB_TILED3_MIN_WAVES_MIXED>(L, in, out, pc, stream);
}

}  // namespace gcb
