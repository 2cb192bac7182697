// Reverse-mode derivative of the binary64 push: gcb_push_backward.
//
// For a segment of n_steps steps starting from a caller-owned state (taken,
// with its adjoint, into the tile order of the start positions), the host
// recomputes the forward steps with the push kernels (the tiled push in
// place when sorting is on, the same parity arithmetic as the forward pass),
// keeping the start state of every step and its switch decisions; the
// decisions give each step the list of its guiding-center particles; then,
// per step in reverse order, two kernels (one per regime; the
// guiding-center one with one lane per list entry) map the cotangents of the
// step outputs to those of its inputs and record every gather point with its
// cotangents.  After a batch of steps a scatter kernel spreads the recorded
// cotangents over the nodes of a binary32 node-interleaved grid (global
// atomics), which is finally added to the caller's dE/dB arrays.
//
// The scatter is a kernel of its own because atomics on this hardware count
// against the same wait counter as loads: inside the register-heavy adjoint
// kernel (one wave per SIMD) every gather would wait for the atomics issued
// before it.  The scatter kernel is light and runs several waves per SIMD; it
// sums one particle's gather points of all steps of the batch in a 4x4 node
// window per component, kept in registers, and writes a window with one
// atomic per non-zero node only when a point falls outside it (the window
// then moves) and at the end.  A guiding-center particle drifts a small
// fraction of a cell per step, so its windows seldom move and the atomics of
// a whole batch merge; atomic throughput is what bounds the scatter.
// Compiled with -ffp-contract=off like the forward binary64 path.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/gcb.h"
#include "gcb_adjoint.hpp"
#include "gcb_internal.h"

namespace gcb {
namespace {

constexpr int kWG = 128;

// Minimum waves per SIMD the step VJP kernels are compiled for (register
// budget; 1 leaves it to the compiler).
#ifndef GCB_ADJ_MIN_WAVES
#define GCB_ADJ_MIN_WAVES 1
#endif

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

// The guiding-center VJP keeps the field samples of R^{n-1/2}, R^n and the
// first iterates of its forward recomputation in LDS (one column per lane)
// and takes them again in the reverse sweep instead of a second gather.
#ifndef GCB_ADJ_KEEP_SLOTS
#define GCB_ADJ_KEEP_SLOTS 5
#endif
constexpr int kKeepSlots = GCB_ADJ_KEEP_SLOTS;
constexpr int kSampleVals = 12;   // E, B, dB/dx, dB/dy

struct LdsSamples {
    double* base;   // entry (slot*12 + c)*kWG + lane
    __device__ void put(int slot, const adj::SampleD& s) const {
        if (slot >= kKeepSlots) return;
        double* b = base + slot * kSampleVals * kWG;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            b[c * kWG] = s.E[c];
            b[(3 + c) * kWG] = s.B[c];
            b[(6 + c) * kWG] = s.dBx[c];
            b[(9 + c) * kWG] = s.dBy[c];
        }
    }
    __device__ bool get(int slot, adj::SampleD& s) const {
        if (slot >= kKeepSlots) return false;
        const double* b = base + slot * kSampleVals * kWG;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            s.E[c] = b[c * kWG];
            s.B[c] = b[(3 + c) * kWG];
            s.dBx[c] = b[(6 + c) * kWG];
            s.dBy[c] = b[(9 + c) * kWG];
        }
        return true;
    }
};

// One regime per launch.  Guiding-center branch: lane t takes entry t of the
// step's list (k_gca_lists), so every lane of a wavefront has work and waves
// past the list return at once.  Boris branch: one lane per particle, lanes
// whose particle took the other branch return at once.
template <bool kYee, bool kBoris>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(GCB_ADJ_MIN_WAVES))) void
k_adjoint_step(const double* __restrict__ st, const double* __restrict__ qm_arr,
               const uint8_t* __restrict__ S, const uint32_t* __restrict__ list,
               const unsigned* __restrict__ count, double* lam, int64_t n,
               const double* __restrict__ F, PushConst pc, RecordSink rec) {
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    int64_t p;
    if (kBoris) {
        if (t >= n || S[t] == 0) return;
        p = t;
    } else {
        if (t >= (int64_t)*count) return;
        p = list[t];
    }
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
    if constexpr (kBoris) {
        adj::boris_step_vjp<kYee>(acc, rec, pc, K, s, qm, l);
    } else {
        __shared__ double kept[kKeepSlots * kSampleVals * kWG];
        adj::gca_step_vjp<kYee>(acc, rec, pc, K, s, qm, l, LdsSamples{kept + threadIdx.x});
    }
#pragma unroll
    for (int c = 0; c < 7; ++c) lam[c * n + p] = l[c];
}

// Guiding-center lists of every step of a segment: for step s (blockIdx.y),
// the particles that took the guiding-center branch (S = 0) go to
// list + s*n, count[s] of them (the caller zeroes count).  Each workgroup
// claims its range with one atomic; inside a workgroup the entries are in
// ascending particle order.  (The Boris branch is light and reads its state
// faster in place, so it keeps one lane per particle.)
constexpr int kListWG = 256;
constexpr int kListItems = 16;   // consecutive particles per lane

__global__ __launch_bounds__(kListWG) void k_gca_lists(const uint8_t* __restrict__ S,
                                                       int64_t n, uint32_t* list,
                                                       unsigned* count) {
    const int64_t s = blockIdx.y;
    const uint8_t* Ss = S + s * n;
    uint32_t* out = list + s * n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t p0 = ((int64_t)blockIdx.x * kListWG + threadIdx.x) * kListItems;
    unsigned mask = 0, ng = 0;
#pragma unroll
    for (int k = 0; k < kListItems; ++k) {
        const int64_t p = p0 + k;
        if (p < n && Ss[p] == 0) {
            mask |= 1u << k;
            ++ng;
        }
    }
    // inclusive wave scan of the per-lane counts
    unsigned sg = ng;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned u = __shfl_up(sg, off, 64);
        if (lane >= off) sg += u;
    }
    __shared__ unsigned wg[kListWG / 64], base;
    if (lane == 63) wg[wave] = sg;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned tg = 0;
        for (int w = 0; w < kListWG / 64; ++w) tg += wg[w];
        base = tg ? atomicAdd(&count[s], tg) : 0u;
    }
    __syncthreads();
    unsigned o = base + sg - ng;
    for (int w = 0; w < wave; ++w) o += wg[w];
#pragma unroll
    for (int k = 0; k < kListItems; ++k)
        if (mask & (1u << k)) out[o++] = (uint32_t)(p0 + k);
}

constexpr int kScatterWG = 256;
constexpr int kNoOrigin = -0x40000000;   // window not placed yet

// Node cotangents of the gather points recorded over a batch of nb steps
// (per step one Boris point or `slots` guiding-center points per particle;
// step b of the batch at records (b*slots + q)).  Per component a 4x4 node
// window with origin (ox, oy) sums the points' 2x2 stencils; a stencil that
// does not fit sends the window to memory (one atomic per non-zero node) and
// moves it there.
template <bool kYee>
__global__ __launch_bounds__(kScatterWG) void k_scatter_batch(
    const double* __restrict__ X, const double* __restrict__ Y, const float* __restrict__ bar,
    const uint8_t* __restrict__ S, int64_t n, int nb, int slots, PushConst pc, float* grad) {
    const int64_t p = (int64_t)blockIdx.x * kScatterWG + threadIdx.x;
    if (p >= n) return;
    const double idx = pc.inv_dx, idy = pc.inv_dy;
    float w[6][16];
    int ox[6], oy[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        ox[k] = kNoOrigin;
        oy[k] = kNoOrigin;
#pragma unroll
        for (int e = 0; e < 16; ++e) w[k][e] = 0.0f;
    }
    auto flush = [&](int k) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            if (w[k][e] != 0.0f) {
                const int i = wrap_index((int)((unsigned)ox[k] + (unsigned)(e >> 2)), pc.nx);
                const int j = wrap_index((int)((unsigned)oy[k] + (unsigned)(e & 3)), pc.ny);
                atomicAdd(&grad[((size_t)j * pc.nx + i) * 6 + k], w[k][e]);
                w[k][e] = 0.0f;
            }
        }
    };
    for (int b = nb - 1; b >= 0; --b) {
        const int ns = S[(int64_t)b * n + p] ? 1 : slots;
        for (int q = 0; q < ns; ++q) {
            const int64_t r = (int64_t)b * slots + q;
            const double gx = X[r * n + p] * idx;
            const double gy = Y[r * n + p] * idy;
            // a runaway point's sample is a constant NaN: no node cotangent
            if (!(fabs(gx) < kFarLattice && fabs(gy) < kFarLattice)) continue;
            const float* bq = bar + r * 12 * n + p;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const double vb = (double)bq[k * n];
                const double dxb = k < 3 ? 0.0 : (double)bq[(3 + k) * n];
                const double dyb = k < 3 ? 0.0 : (double)bq[(6 + k) * n];
                if (vb == 0.0 && dxb == 0.0 && dyb == 0.0) continue;
                const double sx = kYee ? kYeeStagger[k][0] : pc.stagger[k][0];
                const double sy = kYee ? kYeeStagger[k][1] : pc.stagger[k][1];
                const double xi = gx - sx, eta = gy - sy;
                const double fi = floor(xi), fj = floor(eta);
                const int i = (int)fi, j = (int)fj;
                const double wx = xi - fi, wy = eta - fj;
                const double ax = 1.0 - wx, ay = 1.0 - wy;
                const float c00 = (float)(vb * (ax * ay) - dxb * (ay * idx) - dyb * (ax * idy));
                const float c10 = (float)(vb * (wx * ay) + dxb * (ay * idx) - dyb * (wx * idy));
                const float c01 = (float)(vb * (ax * wy) - dxb * (wy * idx) + dyb * (ax * idy));
                const float c11 = (float)(vb * (wx * wy) + dxb * (wy * idx) + dyb * (wx * idy));
                // offsets in unsigned arithmetic: any cell index is allowed
                unsigned du = (unsigned)i - (unsigned)ox[k], dv = (unsigned)j - (unsigned)oy[k];
                if (du > 2u || dv > 2u) {
                    flush(k);
                    ox[k] = (int)((unsigned)i - 1u);
                    oy[k] = (int)((unsigned)j - 1u);
                    du = 1u;
                    dv = 1u;
                }
                const int di = (int)du, dj = (int)dv;
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int ra = (e >> 2) - di, rb = (e & 3) - dj;
                    const float v = ra == 0 ? (rb == 0 ? c00 : rb == 1 ? c01 : 0.0f)
                                  : ra == 1 ? (rb == 0 ? c10 : rb == 1 ? c11 : 0.0f)
                                            : 0.0f;
                    w[k][e] += v;
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) flush(k);
}

}  // namespace

int adjoint_slots(int n_iter) { return adj::gca_vjp_samples(n_iter); }

size_t adjoint_record_bytes(int64_t n, int n_iter, int steps) {
    return (size_t)steps * adjoint_slots(n_iter) * (size_t)n *
           (2 * sizeof(double) + 12 * sizeof(float));
}

namespace {
struct RecordArrays {
    double* X;
    double* Y;
    float* bar;
};

RecordArrays record_arrays(void* records, int64_t n, int slots, int batch) {
    RecordArrays r;
    r.X = static_cast<double*>(records);
    r.Y = r.X + (size_t)batch * slots * n;
    r.bar = reinterpret_cast<float*>(r.Y + (size_t)batch * slots * n);
    return r;
}
}  // namespace

hipError_t launch_adjoint_step(const AdjointLaunch& L, double* lam, const PushConst& pc,
                               hipStream_t stream) {
    if (L.n == 0) return hipSuccess;
    const int slots = adjoint_slots(pc.n_iter);
    const RecordArrays ra = record_arrays(L.records, L.n, slots, L.batch);
    const size_t off = (size_t)L.batch_slot * slots * L.n;
    const RecordSink rec{ra.X + off, ra.Y + off, ra.bar + 12 * off, L.n, 0, 0};
    const unsigned blocks = (unsigned)((L.n + kWG - 1) / kWG);
    if (L.yee) {
        hipLaunchKernelGGL((k_adjoint_step<true, false>), dim3(blocks), dim3(kWG), 0, stream,
                           L.state, L.qm, L.strace, L.list, L.count, lam, L.n, L.fields, pc, rec);
        hipLaunchKernelGGL((k_adjoint_step<true, true>), dim3(blocks), dim3(kWG), 0, stream,
                           L.state, L.qm, L.strace, L.list, L.count, lam, L.n, L.fields, pc, rec);
    } else {
        hipLaunchKernelGGL((k_adjoint_step<false, false>), dim3(blocks), dim3(kWG), 0, stream,
                           L.state, L.qm, L.strace, L.list, L.count, lam, L.n, L.fields, pc, rec);
        hipLaunchKernelGGL((k_adjoint_step<false, true>), dim3(blocks), dim3(kWG), 0, stream,
                           L.state, L.qm, L.strace, L.list, L.count, lam, L.n, L.fields, pc, rec);
    }
    return hipGetLastError();
}

hipError_t launch_gca_lists(const uint8_t* trace, int64_t n, int n_steps, uint32_t* lists,
                            unsigned* counts, hipStream_t stream) {
    if (n == 0 || n_steps == 0) return hipSuccess;
    const int64_t per_block = (int64_t)kListWG * kListItems;
    constexpr int kMaxGridY = 65535;
    for (int s0 = 0; s0 < n_steps; s0 += kMaxGridY) {
        const int ns = std::min(kMaxGridY, n_steps - s0);
        const dim3 grid((unsigned)((n + per_block - 1) / per_block), (unsigned)ns);
        hipLaunchKernelGGL(k_gca_lists, grid, dim3(kListWG), 0, stream, trace + (size_t)s0 * n,
                           n, lists + (size_t)s0 * n, counts + s0);
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_scatter(const AdjointLaunch& L, const uint8_t* strace_first, int nb,
                                  const PushConst& pc, hipStream_t stream) {
    if (L.n == 0 || nb <= 0) return hipSuccess;
    const int slots = adjoint_slots(pc.n_iter);
    const RecordArrays ra = record_arrays(L.records, L.n, slots, L.batch);
    const unsigned blocks = (unsigned)((L.n + kScatterWG - 1) / kScatterWG);
    if (L.yee)
        hipLaunchKernelGGL((k_scatter_batch<true>), dim3(blocks), dim3(kScatterWG), 0, stream,
                           ra.X, ra.Y, ra.bar, strace_first, L.n, nb, slots, pc,
                           L.grad_fields);
    else
        hipLaunchKernelGGL((k_scatter_batch<false>), dim3(blocks), dim3(kScatterWG), 0, stream,
                           ra.X, ra.Y, ra.bar, strace_first, L.n, nb, slots, pc,
                           L.grad_fields);
    return hipGetLastError();
}

}  // namespace gcb
