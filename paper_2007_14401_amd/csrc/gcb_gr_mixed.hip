// The curved-spacetime push in the precision form: binary32 fields, metric,
// four-velocity and bulk arithmetic, binary64 positions (see gcb_gr.hpp for
// the quantities kept in binary64).  Contraction to fused multiply-add is
// allowed in this unit.
#include <hip/hip_runtime.h>

#include "gcb_gr_kernels.hpp"

namespace gcb {

hipError_t launch_gr_push_mixed(const GrPtrs& in, const GrPtrs& out, const uint32_t* perm,
                                int64_t n, int n_steps, const float* F, const double* dl,
                                const gr::GrConst& g, uint8_t* trace, int trace_step0,
                                DevStats* stats, hipStream_t stream) {
    return grk::launch<float, float>(in, out, perm, n, n_steps, F, dl, g, trace, trace_step0, stats,
                                     stream);
}

}  // namespace gcb
