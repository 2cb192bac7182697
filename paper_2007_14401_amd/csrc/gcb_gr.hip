// Kernels of the curved-spacetime push (binary64, compiled with
// -ffp-contract=off): the proper cell-length table and the coupled step.
//
// The push keeps a particle in registers for a chunk of steps (the fields
// are static and the particles independent), writing its switch decision of
// every step to the trace; a 512^2 grid of node records (12.6 MB) stays in
// the caches, and the metric is evaluated analytically.
#include <hip/hip_runtime.h>

#include "gcb_gr.hpp"
#include "gcb_internal.h"

namespace gcb {
namespace {

constexpr int kGrWG = 256;
constexpr int kGrStepsPerLaunch = 8;

__global__ __launch_bounds__(256) void k_gr_cell_lengths(gr::GrConst g, double dr, double dth,
                                                         double* dl) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= (int64_t)g.nr * g.nth) return;
    const int j = (int)(c / g.nr);
    const int i = (int)(c - (int64_t)j * g.nr);
    dl[c] = gr::cell_length(g, dr, dth, i, j);
}

__device__ __forceinline__ double wave_max_nan(double v) {
    for (int off = 32; off > 0; off >>= 1) v = gr::max_nan(v, __shfl_xor(v, off, 64));
    return v;
}

#ifndef GCB_GR_MIN_WAVES
#define GCB_GR_MIN_WAVES 2
#endif

__global__ __launch_bounds__(kGrWG) __attribute__((amdgpu_waves_per_eu(GCB_GR_MIN_WAVES))) void
k_gr_push(GrPtrs p, int64_t n, int s0, int ns,
                                                   const double* __restrict__ F,
                                                   const double* __restrict__ dl,
                                                   gr::GrConst g, uint8_t* trace,
                                                   DevStats* stats) {
    const int64_t k = (int64_t)blockIdx.x * kGrWG + threadIdx.x;
    const bool active = k < n;
    unsigned cnt_g = 0, cnt_b = 0;
    double maxres = 0.0;
    if (active) {
        double x[3] = {p.r[k], p.th[k], p.ph[k]};
        double u[3] = {p.ur[k], p.uth[k], p.uph[k]};
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
        p.ur[k] = u[0];
        p.uth[k] = u[1];
        p.uph[k] = u[2];
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

}  // namespace

hipError_t launch_gr_cell_lengths(const gr::GrConst& g, double dr, double dth, double* dl,
                                  hipStream_t stream) {
    const int64_t cells = (int64_t)g.nr * g.nth;
    const unsigned blocks = (unsigned)((cells + 255) / 256);
    hipLaunchKernelGGL(k_gr_cell_lengths, dim3(blocks), dim3(256), 0, stream, g, dr, dth, dl);
    return hipGetLastError();
}

hipError_t launch_gr_push(const GrPtrs& p, int64_t n, int n_steps, const double* F,
                          const double* dl, const gr::GrConst& g, uint8_t* trace,
                          DevStats* stats, hipStream_t stream) {
    if (n == 0 || n_steps == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + kGrWG - 1) / kGrWG);
    for (int s0 = 0; s0 < n_steps; s0 += kGrStepsPerLaunch) {
        const int ns = n_steps - s0 < kGrStepsPerLaunch ? n_steps - s0 : kGrStepsPerLaunch;
        hipLaunchKernelGGL(k_gr_push, dim3(blocks), dim3(kGrWG), 0, stream, p, n, s0, ns, F,
                           dl, g, trace, stats);
    }
    return hipGetLastError();
}

}  // namespace gcb
