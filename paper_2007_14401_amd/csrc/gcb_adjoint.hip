// Reverse-mode derivative of the binary64 push: gcb_push_backward.
//
// For a segment of n_steps steps starting from a caller-owned state, the
// forward steps are recomputed (unsorted, one lane per particle, the same
// arithmetic as gcb_push) while the start state of every step and its switch
// decisions are kept; then one adjoint kernel per step, in reverse order,
// maps the cotangents of the step outputs to those of its inputs and
// scatter-adds the field cotangents into a binary32 node-interleaved grid
// (global atomics), which is finally added to the caller's dE/dB arrays.
// Compiled with -ffp-contract=off like the forward binary64 path.
#include <hip/hip_runtime.h>

#include "../../include/gcb.h"
#include "gcb_adjoint.hpp"
#include "gcb_internal.h"

namespace gcb {
namespace {

constexpr int kWG = 128;

struct AtomicSink {
    float* g;
    int nx, ny;
    __device__ void add(int k, int i, int j, double v) const {
        if (v == 0.0) return;
        const int i0 = wrap_index(i, nx);
        const int j0 = wrap_index(j, ny);
        atomicAdd(&g[((size_t)j0 * nx + i0) * 6 + k], (float)v);
    }
};

// One regime per launch: lanes whose particle took the other branch at this
// step return at once, so no wavefront executes both reverse branches.
#ifndef GCB_ADJ_MIN_WAVES
#define GCB_ADJ_MIN_WAVES 1
#endif

template <bool kYee, bool kBoris>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(GCB_ADJ_MIN_WAVES))) void
k_adjoint_step(const double* __restrict__ st,
                                                       const double* __restrict__ qm_arr,
                                                       const uint8_t* __restrict__ S,
                                                       double* lam, int64_t n,
                                                       const double* __restrict__ F,
                                                       PushConst pc, float* grad) {
    const int64_t p = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (p >= n || (S[p] != 0) != kBoris) return;
    double s[7], l[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        s[c] = st[c * n + p];
        l[c] = lam[c * n + p];
    }
    const double qm = qm_arr ? qm_arr[p] : pc.qm;
    const GlobalAcc<double> acc{F, pc.nx, pc.ny};
    AtomicSink sink{grad, pc.nx, pc.ny};
    const Consts<double> K = make_consts<double>(pc);
    if (kBoris)
        adj::boris_step_vjp<kYee>(acc, sink, pc, K, s, qm, l);
    else
        adj::gca_step_vjp<kYee>(acc, sink, pc, K, s, qm, l);
#pragma unroll
    for (int c = 0; c < 7; ++c) lam[c * n + p] = l[c];
}

}  // namespace

hipError_t launch_adjoint_step(const AdjointLaunch& L, double* lam, const PushConst& pc,
                               hipStream_t stream) {
    if (L.n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((L.n + kWG - 1) / kWG);
    if (L.yee) {
        hipLaunchKernelGGL((k_adjoint_step<true, false>), dim3(blocks), dim3(kWG), 0, stream,
                           L.state, L.qm, L.strace, lam, L.n, L.fields, pc, L.grad_fields);
        hipLaunchKernelGGL((k_adjoint_step<true, true>), dim3(blocks), dim3(kWG), 0, stream,
                           L.state, L.qm, L.strace, lam, L.n, L.fields, pc, L.grad_fields);
    } else {
        hipLaunchKernelGGL((k_adjoint_step<false, false>), dim3(blocks), dim3(kWG), 0, stream,
                           L.state, L.qm, L.strace, lam, L.n, L.fields, pc, L.grad_fields);
        hipLaunchKernelGGL((k_adjoint_step<false, true>), dim3(blocks), dim3(kWG), 0, stream,
                           L.state, L.qm, L.strace, lam, L.n, L.fields, pc, L.grad_fields);
    }
    return hipGetLastError();
}

}  // namespace gcb
