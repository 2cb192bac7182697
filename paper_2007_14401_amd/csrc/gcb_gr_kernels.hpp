// The curved-spacetime push kernel, shared by the binary64 unit
// (gcb_gr.hip, -ffp-contract=off) and the precision-form unit
// (gcb_gr_mixed.hip).
//
// One lane per particle; the particle stays in registers for a chunk of
// steps (the fields are static and the particles independent), and its
// switch decision of every step goes to the trace.  A 512^2 grid of node
// records (12.6 MB binary64) stays in the caches; the metric is evaluated
// analytically.
#pragma once

#include <hip/hip_runtime.h>

#include "gcb_gr.hpp"
#include "gcb_internal.h"

namespace gcb {
namespace grk {

constexpr int kGrWG = 256;
constexpr int kGrStepsPerLaunch = 8;

__device__ __forceinline__ double wave_max_nan(double v) {
    for (int off = 32; off > 0; off >>= 1) v = gr::max_nan(v, __shfl_xor(v, off, 64));
    return v;
}

template <typename R, typename T>
__global__ __launch_bounds__(kGrWG) __attribute__((amdgpu_waves_per_eu(2))) void
k_gr_push(GrPtrs p, int64_t n, int s0, int ns, const T* __restrict__ F,
          const double* __restrict__ dl, gr::GrConst g, uint8_t* trace, DevStats* stats) {
    const int64_t k = (int64_t)blockIdx.x * kGrWG + threadIdx.x;
    const bool active = k < n;
    unsigned cnt_g = 0, cnt_b = 0;
    double maxres = 0.0;
    if (active) {
        double x[3] = {p.r[k], p.th[k], p.ph[k]};
        R* ur = static_cast<R*>(p.ur);
        R* uth = static_cast<R*>(p.uth);
        R* uph = static_cast<R*>(p.uph);
        R u[3] = {ur[k], uth[k], uph[k]};
        const double qm = p.qm ? p.qm[k] : g.qm;
        uint8_t st = p.status[k];
        for (int s = 0; s < ns; ++s) {
            double res;
            const int S = gr::coupled_step(F, dl, g, x, u, qm, st, res);
            if (trace) trace[(size_t)(s0 + s) * n + k] = (uint8_t)S;
            cnt_g += S == 0;
            cnt_b += S == 1;
            maxres = gr::max_nan(maxres, res);
        }
        p.r[k] = x[0];
        p.th[k] = x[1];
        p.ph[k] = x[2];
        ur[k] = u[0];
        uth[k] = u[1];
        uph[k] = u[2];
        p.status[k] = st;
    }
    if (stats) {
        unsigned long long a = cnt_g, b = cnt_b;
        for (int off = 32; off > 0; off >>= 1) {
            a += __shfl_xor(a, off, 64);
            b += __shfl_xor(b, off, 64);
        }
        const double m = wave_max_nan(maxres);
        DevStats* sl = stats + blockIdx.x % kStatSlots;
        if ((threadIdx.x & 63) == 0) {
            if (a) atomicAdd(&sl->gca_steps, a);
            if (b) atomicAdd(&sl->boris_steps, b);
            if (m > 0.0)
                atomicMax(&sl->max_res_bits, (unsigned long long)__double_as_longlong(m));
        }
    }
}


template <typename R, typename T>
hipError_t launch(const GrPtrs& p, int64_t n, int n_steps, const T* F, const double* dl,
                  const gr::GrConst& g, uint8_t* trace, DevStats* stats, hipStream_t stream) {
    if (n == 0 || n_steps == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + kGrWG - 1) / kGrWG);
    for (int s0 = 0; s0 < n_steps; s0 += kGrStepsPerLaunch) {
        const int ns = n_steps - s0 < kGrStepsPerLaunch ? n_steps - s0 : kGrStepsPerLaunch;
        hipLaunchKernelGGL((k_gr_push<R, T>), dim3(blocks), dim3(kGrWG), 0, stream, p, n, s0, ns,
                           F, dl, g, trace, stats);
    }
    return hipGetLastError();
}

}  // namespace grk
}  // namespace gcb
