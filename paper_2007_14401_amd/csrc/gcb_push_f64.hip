// Push kernels of the binary64 form (compiled with -ffp-contract=off, so the
// arithmetic is evaluated exactly as written in gcb_math.hpp).
#include "gcb_push_kernels.hpp"

// Minimum waves per SIMD the tiled kernel is compiled for (register budget).
#ifndef GCB_TILED_MIN_WAVES
#define GCB_TILED_MIN_WAVES 3
#endif

namespace gcb {

size_t tiled_lds_bytes(int window, size_t elem_bytes) {
    size_t f = (size_t)window * window * 6 * elem_bytes;
    f = (f + 15) & ~(size_t)15;
    // then the queue of a chunk
    return f + (size_t)kTiledChunk * sizeof(uint16_t);
}

hipError_t launch_push_f64(const PushLaunch& L, const ParticlePtrs<double>& in,
                           const ParticlePtrs<double>& out, const PushConst& pc,
                           hipStream_t stream) {
    return kern::launch_push<double, double, GCB_TILED_MIN_WAVES>(L, in, out, pc, stream);
}

}  // namespace gcb
