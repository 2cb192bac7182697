// 3D push kernels of the binary64 form (compiled with -ffp-contract=off, so
// the arithmetic is evaluated exactly as written in gcb_math3.hpp).
#include "gcb_push3_kernels.hpp"

// Minimum waves per SIMD the 3D tiled kernel is compiled for (register budget).
#ifndef GCB_TILED3_MIN_WAVES
#define GCB_TILED3_MIN_WAVES 3
#endif

namespace gcb {

size_t tiled3_lds_bytes(int window, size_t elem_bytes) {
    size_t f = (size_t)window * window * window * 6 * elem_bytes;
    f = (f + 15) & ~(size_t)15;
    return f + (size_t)kQueueMax * sizeof(uint16_t);
}

hipError_t launch_push3_f64(const Push3Launch& L, const ParticlePtrs3<double>& in,
                            const ParticlePtrs3<double>& out, const PushConst3& pc,
                            hipStream_t stream) {
    return kern::launch_push3<double, double, GCB_TILED3_MIN_WAVES>(L, in, out, pc, stream);
}

}  // namespace gcb
