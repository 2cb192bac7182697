// Push kernels of the production binary64 form (GCB_ARITH_FAST): the
// arithmetic of gcb_math.hpp compiled with -ffp-contract=fast, so the
// compiler fuses a product into the sum that consumes it (one rounding
// instead of two), and with its production branches (reciprocal square roots
// instead of square roots that serve as divisors, multiplications by
// per-launch reciprocals).  The instances live in namespaces of their own,
// apart from those of the exact binary64 unit.
#define GCB_ARITH_NS arith_fast
#define GCB_FAST_ARITH 1
#define GCB_KERN_NS kern_fast
#include "gcb_push_kernels.hpp"

#ifndef GCB_TILED_MIN_WAVES
#define GCB_TILED_MIN_WAVES 3
#endif

namespace gcb {

hipError_t launch_push_f64_fast(const PushLaunch& L, const ParticlePtrs<double>& in,
                                const ParticlePtrs<double>& out, const PushConst& pc,
                                hipStream_t stream) {
    return kern_fast::launch_push<double, double, GCB_TILED_MIN_WAVES>(L, in, out, pc, stream);
}

}  // namespace gcb
