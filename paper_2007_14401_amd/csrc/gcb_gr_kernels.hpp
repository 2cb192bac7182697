// The curved-spacetime push kernel, shared by the binary64 unit
// (gcb_gr.hip, -ffp-contract=off), the production binary64 unit
// (gcb_gr_fast.hip) and the precision-form unit (gcb_gr_mixed.hip).
//
// One lane per particle, taken from the block's regime queues; the particle
// stays in registers for a chunk of steps (the fields are static and the
// particles independent), and its switch decision of every step goes to the
// trace.  A 512^2 grid of node
// records (12.6 MB binary64) stays in the caches; the metric is evaluated
// analytically.
#pragma once

#include <hip/hip_runtime.h>

#include "gcb_gr.hpp"
#include "gcb_internal.h"
#include "gcb_queues.hpp"

// The kernels are compiled once per form and arithmetic; the namespace of
// their instances is set by the including unit.
#ifndef GCB_GR_KERN_NS
#define GCB_GR_KERN_NS grk
#endif

namespace gcb {
namespace GCB_GR_KERN_NS {

constexpr int kGrWG = 256;
// waves per SIMD the register allocation must allow (the kernel is bound by
// the issue of its binary64 arithmetic; three waves hide its latencies)
#ifndef GCB_GR_MIN_WAVES
#define GCB_GR_MIN_WAVES 3
#endif

constexpr int kGrStepsPerLaunch = 8;

__device__ __forceinline__ double wave_max_nan(double v) {
    for (int off = 32; off > 0; off >>= 1) v = gr::max_nan(v, __shfl_xor(v, off, 64));
    return v;
}

// ns steps of the particles of one block of kGrWG slots: the particle in
// slot perm[k] of `in` (slot k when perm is null) is written to slot k of
// `out` -- the same arrays, or, on the launch after a sort, the other buffer,
// which then also receives q/m and the id.
//
// The block's particles are first split by the branch of their first step
// into a guiding-center queue and a full-orbit queue (particles outside the
// domain join the latter), and lane t takes the particle of queue slot t for
// all ns steps, so that a wavefront runs one branch until one of its
// particles changes regime.  Each step still takes its own switch decision;
// the metric and the fields a step evaluates at its end serve the start of
// the next.
//
// Workgroup b runs on XCD b % 8; it takes block (b % 8) * per_xcd + b / 8,
// so that each XCD works through a contiguous eighth of the (tile-sorted)
// slots and its L2 holds the part of the grid those particles sample.
template <typename R, typename T>
__global__ __launch_bounds__(kGrWG) __attribute__((amdgpu_waves_per_eu(GCB_GR_MIN_WAVES))) void
k_gr_push(GrPtrs in, GrPtrs out, const uint32_t* __restrict__ perm, int64_t n, int s0, int ns,
          int per_xcd, const T* __restrict__ F, const double* __restrict__ dl, gr::GrConst g,
          uint8_t* trace, DevStats* stats) {
    __shared__ uint16_t queue[kGrWG];
    __shared__ int wave_g[kGrWG / 64];
    __shared__ int wave_b[kGrWG / 64];
    const int64_t blk = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int64_t base = blk * kGrWG;
    if (base >= n) return;   // the whole workgroup
    const int m = (int)(n - base < kGrWG ? n - base : kGrWG);
    const R* in_ur = static_cast<const R*>(in.ur);
    const R* in_uth = static_cast<const R*>(in.uth);
    const R* in_uph = static_cast<const R*>(in.uph);
    split_queues<kGrWG>(m, queue, wave_g, wave_b, [&](int q) {
        const int64_t src = perm ? (int64_t)perm[base + q] : base + q;
        const double x[3] = {in.r[src], in.th[src], 0.0};
        const R u[3] = {in_ur[src], in_uth[src], in_uph[src]};
        const double qm = in.qm ? in.qm[src] : g.qm;
        return gr::starts_gca(F, dl, g, x, u, qm, in.status[src]);
    });
    unsigned cnt_g = 0, cnt_b = 0;
    double maxres = 0.0;
    if ((int)threadIdx.x < m) {
        const int64_t k = base + queue[threadIdx.x];
        const int64_t src = perm ? (int64_t)perm[k] : k;
        double x[3] = {in.r[src], in.th[src], in.ph[src]};
        R u[3] = {in_ur[src], in_uth[src], in_uph[src]};
        const double qm = in.qm ? in.qm[src] : g.qm;
        const int32_t pid = in.id ? in.id[src] : (int32_t)k;
        uint8_t st = in.status[src];
        gr::StepStart<R> start;
        start.valid = false;
        for (int s = 0; s < ns; ++s) {
            double res;
            const int S = gr::coupled_step(F, dl, g, x, u, qm, st, res, start);
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
    const int64_t blocks = (n + kGrWG - 1) / kGrWG;
    const int per_xcd = (int)((blocks + 7) / 8);
    for (int s0 = 0; s0 < n_steps; s0 += kGrStepsPerLaunch) {
        const int ns = n_steps - s0 < kGrStepsPerLaunch ? n_steps - s0 : kGrStepsPerLaunch;
        hipLaunchKernelGGL((k_gr_push<R, T>), dim3(8 * per_xcd), dim3(kGrWG), 0, stream,
                           s0 == 0 ? in : out, out, s0 == 0 ? perm : nullptr, n,
                           trace_step0 + s0, ns, per_xcd, F, dl, g, trace, stats);
    }
    return hipGetLastError();
}

}  // namespace GCB_GR_KERN_NS
}  // namespace gcb
