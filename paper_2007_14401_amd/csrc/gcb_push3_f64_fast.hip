// 3D push kernels of the production binary64 form (GCB_ARITH_FAST): the
// arithmetic of gcb_math3.hpp compiled with -ffp-contract=fast and its
// production branches (reciprocal square roots, multiplications by
// per-launch reciprocals), in namespaces of their own as in 2D.
#define GCB_ARITH_NS arith_fast
#define GCB_FAST_ARITH 1
#define GCB_KERN_NS kern_fast
#include "gcb_push3_kernels.hpp"

#ifndef GCB_TILED3_MIN_WAVES
#define GCB_TILED3_MIN_WAVES 3
#endif

namespace gcb {

hipError_t launch_push3_f64_fast(const Push3Launch& L, const ParticlePtrs3<double>& in,
                                 const ParticlePtrs3<double>& out, const PushConst3& pc,
                                 hipStream_t stream) {
    return kern_fast::launch_push3<double, double, GCB_TILED3_MIN_WAVES>(L, in, out, pc,
                                                                        stream);
}

}  // namespace gcb
