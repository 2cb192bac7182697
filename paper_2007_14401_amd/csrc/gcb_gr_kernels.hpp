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

// ns steps of the particle in slot perm[k] of `in` (slot k when perm is
// null), written to slot k of `out`: the same arrays, or, on the launch after
// a sort, the other buffer, which then also receives q/m and the id
template <typename R, typename T>
__global__ __launch_bounds__(kGrWG) __attribute__((amdgpu_waves_per_eu(3))) void
k_gr_push(GrPtrs in, GrPtrs out, const uint32_t* __restrict__ perm, int64_t n, int s0, int ns,
          const T* __restrict__ F, const double* __restrict__ dl, gr::GrConst g,
          uint8_t* trace, DevStats* stats) {
    const int64_t k = (int64_t)blockIdx.x * kGrWG + threadIdx.x;
    const bool active = k < n;
    unsigned cnt_g = 0, cnt_b = 0;
    double maxres = 0.0;
    if (active) {
        const int64_t src = perm ? (int64_t)perm[k] : k;
        double x[3] = {in.r[src], in.th[src], in.ph[src]};
        R u[3] = {static_cast<const R*>(in.ur)[src], static_cast<const R*>(in.uth)[src],
                  static_cast<const R*>(in.uph)[src]};
        const double qm = in.qm ? in.qm[src] : g.qm;
        const int32_t pid = in.id ? in.id[src] : (int32_t)k;
        uint8_t st = in.status[src];
        for (int s = 0; s < ns; ++s) {
            double res;
            const int S = gr::coupled_step(F, dl, g, x, u, qm, st, res);
            if (trace) trace[(size_t)(s0 + s) * n + pid] = (uint8_t)S;
            cnt_g += S == 0;
            cnt_b += S == 1;
            maxres = gr::max_nan(maxres, res);
        }
        out.r[k] = x[0];
        out.th[k] = x[1];
        out.ph[k] = x[2];
        static_cast<R*>(out.ur)[k] = u[0];
        static_cast<R*>(out.uth)[k] = u[1];
        static_cast<R*>(out.uph)[k] = u[2];
        out.status[k] = st;
        if (out.r != in.r) {
            if (in.qm) const_cast<double*>(out.qm)[k] = qm;
            if (in.id) out.id[k] = pid;
        }
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
hipError_t launch(const GrPtrs& in, const GrPtrs& out, const uint32_t* perm, int64_t n,
                  int n_steps, const T* F, const double* dl, const gr::GrConst& g,
                  uint8_t* trace, int trace_step0, DevStats* stats, hipStream_t stream) {
    if (n == 0 || n_steps == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + kGrWG - 1) / kGrWG);
    for (int s0 = 0; s0 < n_steps; s0 += kGrStepsPerLaunch) {
        const int ns = n_steps - s0 < kGrStepsPerLaunch ? n_steps - s0 : kGrStepsPerLaunch;
        hipLaunchKernelGGL((k_gr_push<R, T>), dim3(blocks), dim3(kGrWG), 0, stream,
                           s0 == 0 ? in : out, out, s0 == 0 ? perm : nullptr, n,
                           trace_step0 + s0, ns, F, dl, g, trace, stats);
    }
    return hipGetLastError();
}

}  // namespace grk
}  // namespace gcb
