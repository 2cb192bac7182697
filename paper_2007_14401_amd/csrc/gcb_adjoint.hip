// Reverse-mode derivative of the binary64 push: gcb_push_backward.
//
// For a segment of n_steps steps starting from a caller-owned state, the
// forward steps are recomputed (unsorted, one lane per particle, the same
// arithmetic as gcb_push) while the start state of every step and its switch
// decisions are kept; then, per step in reverse order, two kernels (one per
// regime) map the cotangents of the step outputs to those of its inputs and
// record every gather point with its cotangents, and a scatter kernel spreads
// the recorded cotangents over the nodes of a binary32 node-interleaved grid
// (global atomics), which is finally added to the caller's dE/dB arrays.
//
// The scatter is a kernel of its own because atomics on this hardware count
// against the same wait counter as loads: inside the register-heavy adjoint
// kernel (one wave per SIMD) every gather would wait for the atomics issued
// before it.  The scatter kernel is light, runs many waves per SIMD, and sums a
// particle's gather points of one step in a 4x4 node window per component
// before touching memory, so most of the per-point atomics merge.
// Compiled with -ffp-contract=off like the forward binary64 path.
#include <hip/hip_runtime.h>

#include "../../include/gcb.h"
#include "gcb_adjoint.hpp"
#include "gcb_internal.h"

namespace gcb {
namespace {

constexpr int kWG = 128;

// Recorded gather points of one step, structure of arrays over particles:
// X[s*n + p], Y[s*n + p] and bar[(s*12 + c)*n + p] for slot s of particle p,
// c = E_x..E_z, B_x..B_z, dB/dx (3), dB/dy (3).
struct RecordSink {
    double* X;
    double* Y;
    float* bar;
    int64_t n, p;
    int slot;
    __device__ void sample(double x, double y, const adj::SampleBar& sb) {
        const int64_t o = (int64_t)slot * n + p;
        X[o] = x;
        Y[o] = y;
        float* b = bar + (int64_t)slot * 12 * n + p;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            b[c * n] = (float)sb.E[c];
            b[(3 + c) * n] = (float)sb.B[c];
            b[(6 + c) * n] = (float)sb.dBx[c];
            b[(9 + c) * n] = (float)sb.dBy[c];
        }
        ++slot;
    }
};

// One regime per launch: lanes whose particle took the other branch at this
// step return at once, so no wavefront executes both reverse branches.
template <bool kYee, bool kBoris>
__global__ __launch_bounds__(kWG) void k_adjoint_step(const double* __restrict__ st,
                                                      const double* __restrict__ qm_arr,
                                                      const uint8_t* __restrict__ S,
                                                      double* lam, int64_t n,
                                                      const double* __restrict__ F,
                                                      PushConst pc, RecordSink rec) {
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
    rec.p = p;
    rec.slot = 0;
    const Consts<double> K = make_consts<double>(pc);
    if (kBoris)
        adj::boris_step_vjp<kYee>(acc, rec, pc, K, s, qm, l);
    else
        adj::gca_step_vjp<kYee>(acc, rec, pc, K, s, qm, l);
#pragma unroll
    for (int c = 0; c < 7; ++c) lam[c * n + p] = l[c];
}

constexpr int kScatterWG = 256;

__device__ __forceinline__ void node_atomic(float* g, int nx, int ny, int k, int i, int j,
                                            double v) {
    if (v == 0.0) return;
    const int i0 = wrap_index(i, nx);
    const int j0 = wrap_index(j, ny);
    atomicAdd(&g[((size_t)j0 * nx + i0) * 6 + k], (float)v);
}

// Node cotangents of the recorded gather points (one Boris point, or
// gca_slots guiding-center points, per particle).  Per component the points'
// 2x2 stencils are summed in a 4x4 window around the first point's cell and
// the window is written with one atomic per non-zero node; a stencil outside
// the window (a point more than one cell away, or across the periodic seam)
// goes straight to memory.
template <bool kYee>
__global__ __launch_bounds__(kScatterWG) void k_scatter_samples(
    const double* __restrict__ X, const double* __restrict__ Y, const float* __restrict__ bar,
    const uint8_t* __restrict__ S, int64_t n, int gca_slots, PushConst pc, float* grad) {
    const int64_t p = (int64_t)blockIdx.x * kScatterWG + threadIdx.x;
    if (p >= n) return;
    const int ns = S[p] ? 1 : gca_slots;
    const double idx = pc.inv_dx, idy = pc.inv_dy;
    for (int k = 0; k < 6; ++k) {
        const double sx = kYee ? kYeeStagger[k][0] : pc.stagger[k][0];
        const double sy = kYee ? kYeeStagger[k][1] : pc.stagger[k][1];
        int i0 = 0, j0 = 0;
        double w[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) w[a][b] = 0.0;
        for (int q = 0; q < ns; ++q) {
            const int64_t o = (int64_t)q * n + p;
            const float* bq = bar + (int64_t)q * 12 * n + p;
            const double vb = (double)bq[k * n];
            const double dxb = k < 3 ? 0.0 : (double)bq[(3 + k) * n];
            const double dyb = k < 3 ? 0.0 : (double)bq[(6 + k) * n];
            const double xi = X[o] * idx - sx, eta = Y[o] * idy - sy;
            const double fi = floor(xi), fj = floor(eta);
            const int i = (int)fi, j = (int)fj;
            if (q == 0) {
                i0 = i;
                j0 = j;
            }
            if (vb == 0.0 && dxb == 0.0 && dyb == 0.0) continue;
            const double wx = xi - fi, wy = eta - fj;
            const double ax = 1.0 - wx, ay = 1.0 - wy;
            const double c00 = vb * (ax * ay) - dxb * (ay * idx) - dyb * (ax * idy);
            const double c10 = vb * (wx * ay) + dxb * (ay * idx) - dyb * (wx * idy);
            const double c01 = vb * (ax * wy) - dxb * (wy * idx) + dyb * (ax * idy);
            const double c11 = vb * (wx * wy) + dxb * (wy * idx) + dyb * (wx * idy);
            const int di = i - i0, dj = j - j0;
            if (di >= -1 && di <= 1 && dj >= -1 && dj <= 1) {
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int ra = a - 1 - di;
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int rb = b - 1 - dj;
                        const double v = ra == 0 ? (rb == 0 ? c00 : rb == 1 ? c01 : 0.0)
                                       : ra == 1 ? (rb == 0 ? c10 : rb == 1 ? c11 : 0.0)
                                                 : 0.0;
                        w[a][b] += v;
                    }
                }
            } else {
                node_atomic(grad, pc.nx, pc.ny, k, i, j, c00);
                node_atomic(grad, pc.nx, pc.ny, k, i + 1, j, c10);
                node_atomic(grad, pc.nx, pc.ny, k, i, j + 1, c01);
                node_atomic(grad, pc.nx, pc.ny, k, i + 1, j + 1, c11);
            }
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) node_atomic(grad, pc.nx, pc.ny, k, i0 - 1 + a, j0 - 1 + b, w[a][b]);
    }
}

}  // namespace

size_t adjoint_sample_bytes(int64_t n, int n_iter) {
    return (size_t)adj::gca_vjp_samples(n_iter) * (size_t)n * (2 * sizeof(double) + 12 * sizeof(float));
}

hipError_t launch_adjoint_step(const AdjointLaunch& L, double* lam, const PushConst& pc,
                               hipStream_t stream) {
    if (L.n == 0) return hipSuccess;
    const int slots = adj::gca_vjp_samples(pc.n_iter);
    double* X = static_cast<double*>(L.samples);
    double* Y = X + (size_t)slots * L.n;
    float* bar = reinterpret_cast<float*>(Y + (size_t)slots * L.n);
    const RecordSink rec{X, Y, bar, L.n, 0, 0};
    const unsigned blocks = (unsigned)((L.n + kWG - 1) / kWG);
    const unsigned sblocks = (unsigned)((L.n + kScatterWG - 1) / kScatterWG);
    if (L.yee) {
        hipLaunchKernelGGL((k_adjoint_step<true, false>), dim3(blocks), dim3(kWG), 0, stream,
                           L.state, L.qm, L.strace, lam, L.n, L.fields, pc, rec);
        hipLaunchKernelGGL((k_adjoint_step<true, true>), dim3(blocks), dim3(kWG), 0, stream,
                           L.state, L.qm, L.strace, lam, L.n, L.fields, pc, rec);
        hipLaunchKernelGGL((k_scatter_samples<true>), dim3(sblocks), dim3(kScatterWG), 0,
                           stream, X, Y, bar, L.strace, L.n, slots, pc, L.grad_fields);
    } else {
        hipLaunchKernelGGL((k_adjoint_step<false, false>), dim3(blocks), dim3(kWG), 0, stream,
                           L.state, L.qm, L.strace, lam, L.n, L.fields, pc, rec);
        hipLaunchKernelGGL((k_adjoint_step<false, true>), dim3(blocks), dim3(kWG), 0, stream,
                           L.state, L.qm, L.strace, lam, L.n, L.fields, pc, rec);
        hipLaunchKernelGGL((k_scatter_samples<false>), dim3(sblocks), dim3(kScatterWG), 0,
                           stream, X, Y, bar, L.strace, L.n, slots, pc, L.grad_fields);
    }
    return hipGetLastError();
}

}  // namespace gcb
