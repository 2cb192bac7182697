// Reverse-mode derivative of the binary64 3D push: the kernels of
// gcb_push_backward_3d.  The organisation is the 2D one (gcb_adjoint.hip):
// the host recomputes the segment's forward steps keeping every step's start
// state and switch decisions, lists each step's guiding-center particles,
// then per step in reverse order runs one kernel per regime that maps the
// cotangents of the step outputs to those of its inputs and records every
// gather point with its cotangents; after a batch of steps a scatter kernel
// spreads the recorded cotangents over a binary32 node-interleaved grid.
// The scatter sums, per particle and component, the points of a batch in a
// 4x4x4 node window of its own in LDS and writes a window (one atomic per
// non-zero node) only when a point leaves it and at the end: a particle
// moves at most c dt per step, so most windows are written once per batch.
// Compiled with -ffp-contract=off like the forward binary64 path.
#include <hip/hip_runtime.h>

#include "../../include/gcb.h"
#include "gcb_adjoint3.hpp"
#include "gcb_internal.h"

namespace gcb {
namespace {

constexpr int kWG = 128;
constexpr int kBar3 = 15;   // cotangents per gather point: E, B, dB/dx, dB/dy, dB/dz

// Recorded gather points of one step, structure of arrays over particles:
// X[s*n + p], Y, Z likewise and bar[(s*15 + c)*n + p] for slot s of particle
// p, c = E_x..E_z, B_x..B_z, dB/dx (3), dB/dy (3), dB/dz (3).
struct RecordSink3 {
    double* X;
    double* Y;
    double* Z;
    float* bar;
    int64_t n, p;
    int slot;
    __device__ void sample(double x, double y, double z, const adj3::SampleBar3& sb) {
        const int64_t o = (int64_t)slot * n + p;
        X[o] = x;
        Y[o] = y;
        Z[o] = z;
        float* b = bar + (int64_t)slot * kBar3 * n + p;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            b[c * n] = (float)sb.E[c];
            b[(3 + c) * n] = (float)sb.B[c];
            b[(6 + c) * n] = (float)sb.dB[0][c];
            b[(9 + c) * n] = (float)sb.dB[1][c];
            b[(12 + c) * n] = (float)sb.dB[2][c];
        }
        ++slot;
    }
};

// The guiding-center VJP keeps the field samples of R^{n-1/2}, R^n and the
// first iterates of its forward recomputation in LDS (one column per lane),
// as in 2D.
constexpr int kKeepSlots3 = 4;
constexpr int kSampleVals3 = 15;   // E, B, dB/dx, dB/dy, dB/dz

struct LdsSamples3 {
    double* base;   // entry (slot*15 + c)*kWG + lane
    __device__ void put(int slot, const Sample3<double>& s) const {
        if (slot >= kKeepSlots3) return;
        double* b = base + slot * kSampleVals3 * kWG;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            b[c * kWG] = s.E[c];
            b[(3 + c) * kWG] = s.B[c];
            b[(6 + c) * kWG] = s.dBx[c];
            b[(9 + c) * kWG] = s.dBy[c];
            b[(12 + c) * kWG] = s.dBz[c];
        }
    }
    __device__ bool get(int slot, Sample3<double>& s) const {
        if (slot >= kKeepSlots3) return false;
        const double* b = base + slot * kSampleVals3 * kWG;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            s.E[c] = b[c * kWG];
            s.B[c] = b[(3 + c) * kWG];
            s.dBx[c] = b[(6 + c) * kWG];
            s.dBy[c] = b[(9 + c) * kWG];
            s.dBz[c] = b[(12 + c) * kWG];
        }
        return true;
    }
};

// One regime per launch, as in 2D: the guiding-center branch over the
// step's list (lane t takes entry t), the Boris branch one lane per particle.
template <bool kYee, bool kBoris>
__global__ __launch_bounds__(kWG) void k_adjoint3_step(
    const double* __restrict__ st, const double* __restrict__ qm_arr,
    const uint8_t* __restrict__ S, const uint32_t* __restrict__ list,
    const unsigned* __restrict__ count, double* lam, int64_t n, const double* __restrict__ F,
    PushConst3 pc, RecordSink3 rec) {
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    int64_t p;
    if (kBoris) {
        if (t >= n || S[t] == 0) return;
        p = t;
    } else {
        if (t >= (int64_t)*count) return;
        p = list[t];
    }
    double s[9], l[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        s[c] = st[c * n + p];
        l[c] = lam[c * n + p];
    }
    const double qm = qm_arr ? qm_arr[p] : pc.b.qm;
    const GlobalAcc3<double> acc{F, pc.b.nx, pc.b.ny, pc.nz};
    rec.p = p;
    rec.slot = 0;
    const Consts3<double> K = make_consts3<double>(pc);
    if constexpr (kBoris) {
        adj3::boris_step_vjp3<kYee>(acc, rec, pc, K, s, qm, l);
    } else {
        __shared__ double kept[kKeepSlots3 * kSampleVals3 * kWG];
        adj3::gca_step_vjp3<kYee>(acc, rec, pc, K, s, qm, l, LdsSamples3{kept + threadIdx.x});
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) lam[c * n + p] = l[c];
}

constexpr int kScatterWG = 128;
constexpr int kWin = 4;                        // nodes per axis of a window
constexpr int kWin3 = kWin * kWin * kWin;
constexpr int kNoOrigin = -0x40000000;         // window not placed yet

// Node cotangents of the gather points recorded over a batch of nb steps
// (per step one Boris point or `slots` guiding-center points per particle;
// step b of the batch at records (b*slots + q)).  One component at a time,
// each lane sums its particle's points in a 4x4x4 node window of its own in
// LDS (entry e of lane t at e*kScatterWG + t); the window covers the 3x3x3
// cells around the cell it was placed on, and moves (after writing its
// non-zero nodes with one atomic each) when a point's cell leaves them.
template <bool kYee>
__global__ __launch_bounds__(kScatterWG) void k_scatter3_batch(
    const double* __restrict__ X, const double* __restrict__ Y, const double* __restrict__ Z,
    const float* __restrict__ bar, const uint8_t* __restrict__ S, int64_t n, int nb, int slots,
    PushConst3 pc, float* grad) {
    __shared__ float win[kWin3 * kScatterWG];
    const int64_t p = (int64_t)blockIdx.x * kScatterWG + threadIdx.x;
    if (p >= n) return;   // no barrier below: every lane uses only its own entries
    float* mine = win + threadIdx.x;
    const double id[3] = {pc.b.inv_dx, pc.b.inv_dy, pc.inv_dz};
    const int nn[3] = {pc.b.nx, pc.b.ny, pc.nz};
    for (int e = 0; e < kWin3; ++e) mine[e * kScatterWG] = 0.0f;
    for (int k = 0; k < 6; ++k) {
        double off[3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            off[a] = kYee ? (((kYee3Set[k] >> a) & 1) ? 0.5 : 0.0)
                          : (a < 2 ? pc.b.stagger[k][a] : pc.sz[k]);
        int org[3] = {kNoOrigin, kNoOrigin, kNoOrigin};
        auto flush = [&]() {
            for (int e = 0; e < kWin3; ++e) {
                const float v = mine[e * kScatterWG];
                if (v != 0.0f) {
                    const int i = wrap_index(org[0] + (e % kWin), nn[0]);
                    const int j = wrap_index(org[1] + (e / kWin) % kWin, nn[1]);
                    const int l = wrap_index(org[2] + e / (kWin * kWin), nn[2]);
                    atomicAdd(&grad[(((size_t)l * nn[1] + j) * nn[0] + i) * 6 + k], v);
                    mine[e * kScatterWG] = 0.0f;
                }
            }
        };
        for (int b = nb - 1; b >= 0; --b) {
            const int ns = S[(int64_t)b * n + p] ? 1 : slots;
            for (int q = 0; q < ns; ++q) {
                const int64_t r = (int64_t)b * slots + q;
                const float* bq = bar + r * kBar3 * n + p;
                const double vb = (double)bq[k * n];
                double gb[3] = {0.0, 0.0, 0.0};
                if (k >= 3) {
                    gb[0] = (double)bq[(3 + k) * n];
                    gb[1] = (double)bq[(6 + k) * n];
                    gb[2] = (double)bq[(9 + k) * n];
                }
                if (vb == 0.0 && gb[0] == 0.0 && gb[1] == 0.0 && gb[2] == 0.0) continue;
                const double g[3] = {X[r * n + p] * id[0], Y[r * n + p] * id[1],
                                     Z[r * n + p] * id[2]};
                // a runaway point's sample is a constant NaN: no node cotangent
                if (!(fabs(g[0]) < kFarLattice && fabs(g[1]) < kFarLattice &&
                      fabs(g[2]) < kFarLattice))
                    continue;
                int c[3];
                double W1[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double xi = g[a] - off[a];
                    const double f = floor(xi);
                    c[a] = (int)f;
                    W1[a] = xi - f;
                }
                // offsets in unsigned arithmetic: any cell index is allowed
                unsigned d[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) d[a] = (unsigned)c[a] - (unsigned)org[a];
                if (d[0] > 2u || d[1] > 2u || d[2] > 2u) {
                    flush();
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        org[a] = (int)((unsigned)c[a] - 1u);
                        d[a] = 1u;
                    }
                }
                const int e0 = (int)d[0] + kWin * ((int)d[1] + kWin * (int)d[2]);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int ox = e & 1, oy = (e >> 1) & 1, oz = e >> 2;
                    const double wx = ox ? W1[0] : 1.0 - W1[0];
                    const double wy = oy ? W1[1] : 1.0 - W1[1];
                    const double wz = oz ? W1[2] : 1.0 - W1[2];
                    const double sx = ox ? id[0] : -id[0];
                    const double sy = oy ? id[1] : -id[1];
                    const double sz = oz ? id[2] : -id[2];
                    const float v = (float)(vb * (wx * wy * wz) + gb[0] * (sx * wy * wz) +
                                            gb[1] * (wx * sy * wz) + gb[2] * (wx * wy * sz));
                    mine[(e0 + ox + kWin * (oy + kWin * oz)) * kScatterWG] += v;
                }
            }
        }
        flush();
    }
}

struct RecordArrays3 {
    double* X;
    double* Y;
    double* Z;
    float* bar;
};

RecordArrays3 record_arrays3(void* records, int64_t n, int slots, int batch) {
    RecordArrays3 r;
    const size_t m = (size_t)batch * slots * n;
    r.X = static_cast<double*>(records);
    r.Y = r.X + m;
    r.Z = r.Y + m;
    r.bar = reinterpret_cast<float*>(r.Z + m);
    return r;
}

}  // namespace

size_t adjoint3_record_bytes(int64_t n, int n_iter, int steps) {
    return (size_t)steps * adjoint_slots(n_iter) * (size_t)n *
           (3 * sizeof(double) + kBar3 * sizeof(float));
}

hipError_t launch_adjoint3_step(const Adjoint3Launch& L, double* lam, const PushConst3& pc,
                                hipStream_t stream) {
    if (L.n == 0) return hipSuccess;
    const int slots = adjoint_slots(pc.b.n_iter);
    const RecordArrays3 ra = record_arrays3(L.records, L.n, slots, L.batch);
    const size_t off = (size_t)L.batch_slot * slots * L.n;
    const RecordSink3 rec{ra.X + off, ra.Y + off, ra.Z + off, ra.bar + kBar3 * off, L.n, 0, 0};
    const unsigned blocks = (unsigned)((L.n + kWG - 1) / kWG);
    if (L.yee) {
        hipLaunchKernelGGL((k_adjoint3_step<true, false>), dim3(blocks), dim3(kWG), 0, stream,
                           L.state, L.qm, L.strace, L.list, L.count, lam, L.n, L.fields, pc, rec);
        hipLaunchKernelGGL((k_adjoint3_step<true, true>), dim3(blocks), dim3(kWG), 0, stream,
                           L.state, L.qm, L.strace, L.list, L.count, lam, L.n, L.fields, pc, rec);
    } else {
        hipLaunchKernelGGL((k_adjoint3_step<false, false>), dim3(blocks), dim3(kWG), 0, stream,
                           L.state, L.qm, L.strace, L.list, L.count, lam, L.n, L.fields, pc, rec);
        hipLaunchKernelGGL((k_adjoint3_step<false, true>), dim3(blocks), dim3(kWG), 0, stream,
                           L.state, L.qm, L.strace, L.list, L.count, lam, L.n, L.fields, pc, rec);
    }
    return hipGetLastError();
}

hipError_t launch_adjoint3_scatter(const Adjoint3Launch& L, const uint8_t* strace_first, int nb,
                                   const PushConst3& pc, hipStream_t stream) {
    if (L.n == 0 || nb <= 0) return hipSuccess;
    const int slots = adjoint_slots(pc.b.n_iter);
    const RecordArrays3 ra = record_arrays3(L.records, L.n, slots, L.batch);
    const unsigned blocks = (unsigned)((L.n + kScatterWG - 1) / kScatterWG);
    if (L.yee)
        hipLaunchKernelGGL((k_scatter3_batch<true>), dim3(blocks), dim3(kScatterWG), 0, stream,
                           ra.X, ra.Y, ra.Z, ra.bar, strace_first, L.n, nb, slots, pc,
                           L.grad_fields);
    else
        hipLaunchKernelGGL((k_scatter3_batch<false>), dim3(blocks), dim3(kScatterWG), 0, stream,
                           ra.X, ra.Y, ra.Z, ra.bar, strace_first, L.n, nb, slots, pc,
                           L.grad_fields);
    return hipGetLastError();
}

}  // namespace gcb
