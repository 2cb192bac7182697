// Kernels of the curved-spacetime push, binary64 (compiled with
// -ffp-contract=off): the proper cell-length table and the coupled step.
#include <hip/hip_runtime.h>

#include "gcb_gr_kernels.hpp"

namespace gcb {
namespace {

__global__ __launch_bounds__(256) void k_gr_cell_lengths(gr::GrConst g, double dr, double dth,
                                                         double* dl) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= (int64_t)g.nr * g.nth) return;
    const int j = (int)(c / g.nr);
    const int i = (int)(c - (int64_t)j * g.nr);
    dl[c] = gr::cell_length(g, dr, dth, i, j);
}

}  // namespace

hipError_t launch_gr_cell_lengths(const gr::GrConst& g, double dr, double dth, double* dl,
                                  hipStream_t stream) {
    const int64_t cells = (int64_t)g.nr * g.nth;
    const unsigned blocks = (unsigned)((cells + 255) / 256);
    hipLaunchKernelGGL(k_gr_cell_lengths, dim3(blocks), dim3(256), 0, stream, g, dr, dth, dl);
    return hipGetLastError();
}

hipError_t launch_gr_push_f64(const GrPtrs& in, const GrPtrs& out, const uint32_t* perm,
                              int64_t n, int n_steps, const double* F, const double* dl,
                              const gr::GrConst& g, uint8_t* trace, int trace_step0,
                              DevStats* stats, hipStream_t stream) {
    return grk::launch<double, double>(in, out, perm, n, n_steps, F, dl, g, trace, trace_step0, stats,
                                       stream);
}

}  // namespace gcb
