// The curved-spacetime push in the production binary64 form
// (GCB_ARITH_FAST): the arithmetic of gcb_gr.hpp compiled with
// -ffp-contract=fast, so the compiler fuses a product into the sum that
// consumes it, and with its production branches (shared reciprocals in the
// metric, reciprocal square roots for square roots that serve as divisors).
// The kernel instances live in a namespace of their own.
#define GCB_FAST_ARITH 1
#define GCB_GR_KERN_NS grk_fast
// the production step needs more registers than three waves per SIMD leave
// without spilling; two waves with all of them in registers run faster
#ifndef GCB_GR_MIN_WAVES
#define GCB_GR_MIN_WAVES 2
#endif
#include <hip/hip_runtime.h>

#include "gcb_gr_kernels.hpp"

namespace gcb {

hipError_t launch_gr_push_fast(const GrPtrs& in, const GrPtrs& out, const uint32_t* perm,
                               int64_t n, int n_steps, const double* F, const double* dl,
                               const gr::GrConst& g, uint8_t* trace, int trace_step0,
                               DevStats* stats, hipStream_t stream) {
    return grk_fast::launch<double, double>(in, out, perm, n, n_steps, F, dl, g, trace,
                                            trace_step0, stats, stream);
}

}  // namespace gcb
