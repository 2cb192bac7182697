// 3D push kernels, templated like the 2D ones on the bulk type R and the
// field storage type T.
//
// As in 2D, both read slot perm[p] of `in` (p when perm is null) and write
// slot p of `out`; the tiled kernel given a permutation with `out` equal to
// `in` keeps the order (keep_order: it writes each particle back to its own
// slot), and its recording instances write each step's start state.
//
// k_push3_global: one lane per particle, up to `ns` steps per launch with the
//   particle in registers, gathers through the caches.
// k_push3_tiled: one workgroup per cubic tile of cell-sorted particles for
//   all the steps of a launch (those between two sorts); the tile's field
//   window (tile + halo per side, W^3 nodes of six components) is staged once
//   in LDS, then the per-regime queues and register-resident steps of the 2D
//   kernel.
//
// Included by exactly one translation unit per form.
#pragma once

#include <hip/hip_runtime.h>

#include "gcb_access3.hpp"
#include "gcb_internal.h"
#include "gcb_math3.hpp"
#include "gcb_push_kernels.hpp"

namespace gcb {
namespace GCB_KERN_NS {

template <typename R>
__device__ __forceinline__ void load_particle3(const ParticlePtrs3<R>& in, int64_t p,
                                               double qm_default, Regs3<R>& r) {
    r.x = in.b.x[p];
    r.y = in.b.y[p];
    r.z = in.z[p];
    r.xp = in.b.xp[p];
    r.yp = in.b.yp[p];
    r.zp = in.zp[p];
    r.ux = in.b.ux[p];
    r.uy = in.b.uy[p];
    r.uz = in.b.uz[p];
    r.qm = in.b.qm ? in.b.qm[p] : qm_default;
}

template <typename R>
__device__ __forceinline__ void store_particle3(const ParticlePtrs3<R>& in,
                                                const ParticlePtrs3<R>& out, int64_t p,
                                                int64_t src, const Regs3<R>& r,
                                                uint32_t flags) {
    out.b.x[p] = r.x;
    out.b.y[p] = r.y;
    out.z[p] = r.z;
    out.b.xp[p] = r.xp;
    out.b.yp[p] = r.yp;
    out.zp[p] = r.zp;
    out.b.ux[p] = r.ux;
    out.b.uy[p] = r.uy;
    out.b.uz[p] = r.uz;
    out.b.status[p] = (uint8_t)(in.b.status[src] | flags);
    if (out.b.x != in.b.x) {   // out-of-place step after a sort: carry the rest along
        if (in.b.qm) out.b.qm[p] = r.qm;
        if (in.b.id) out.b.id[p] = in.b.id[src];
    }
}

// start state of a step into the records (x, y, z, xp, yp, zp, ux, uy, uz,
// arrays of n; the adjoint's recomputation)
template <typename R>
__device__ __forceinline__ void record_state3(double* rec, int64_t n, int64_t i,
                                              const Regs3<R>& r) {
    rec[i] = r.x;
    rec[n + i] = r.y;
    rec[2 * n + i] = r.z;
    rec[3 * n + i] = r.xp;
    rec[4 * n + i] = r.yp;
    rec[5 * n + i] = r.zp;
    rec[6 * n + i] = (double)r.ux;
    rec[7 * n + i] = (double)r.uy;
    rec[8 * n + i] = (double)r.uz;
}

template <typename R, bool kYee, int kVar, class Acc>
__device__ __forceinline__ uint32_t coupled_update3(const Acc& acc, bool gca, Regs3<R>& r,
                                                    const PushConst3& pc, const Consts3<R>& K,
                                                    double& res) {
    uint32_t fl = 0;
    res = 0.0;
    Sample3<R> s;
    if (gca) {
        gather3<R, true, kYee>(acc, pc, K, r.x, r.y, r.z, s);
        fl = gca_step3<R, kYee, var_exact(kVar), kVar == kVarMirror, kVar == kVarPhase,
                       kVar == kVarExactCurv>(
            acc, s, r, pc, K, res);
    } else {
        gather3<R, false, kYee>(acc, pc, K, r.x, r.y, r.z, s);
        boris_step3(s, r, pc, K);
    }
    return fl | finite_flag3(r);
}

template <typename R, typename T, bool kYee, int kVar>
__global__ __launch_bounds__(kWG) void k_push3_global(ParticlePtrs3<R> in,
                                                       ParticlePtrs3<R> out,
                                                       const uint32_t* __restrict__ perm,
                                                       int64_t n, int ns,
                                                       const T* __restrict__ F, PushConst3 pc,
                                                       uint8_t* trace, bool replay,
                                                       DevStats* stats) {
    const int64_t p = (int64_t)blockIdx.x * kWG + threadIdx.x;
    unsigned cnt_g = 0, cnt_b = 0;
    double maxres = 0.0;
    if (p < n) {
        const Consts3<R> K = make_consts3<R>(pc);
        GlobalAcc3<T> acc{F, pc.b.nx, pc.b.ny, pc.nz};
        const int64_t src = perm ? (int64_t)perm[p] : p;
        Regs3<R> r;
        load_particle3(in, src, pc.b.qm, r);
        const int64_t ti = in.b.id ? (int64_t)in.b.id[src] : p;
        uint32_t fl = 0;
        for (int s = 0; s < ns; ++s) {
            uint8_t* tr = trace ? trace + (size_t)s * n : nullptr;
            bool gca;
            if (replay) {
                gca = tr[ti] == 0;
            } else {
                Sample3<R> smp;
                gather3<R, false, kYee>(acc, pc, K, r.x, r.y, r.z, smp);
                gca = switch_gca(smp.E, smp.B, r.ux, r.uy, r.uz, r.qm, pc.b, K);
            }
            double res;
            fl |= coupled_update3<R, kYee, kVar>(acc, gca, r, pc, K, res);
            if (tr && !replay) tr[ti] = gca ? 0 : 1;
            if (gca) {
                ++cnt_g;
                maxres = nan_max(maxres, res);
            } else {
                ++cnt_b;
            }
        }
        store_particle3(in, out, p, src, r, fl);
    }
    if (stats) flush_stats(stats, cnt_g, cnt_b, 0, maxres);
}

// One workgroup per cubic tile of cell-sorted particles for all `steps`
// steps of a launch (those between two sorts), as the 2D kernel: the tile's
// window is staged in LDS once; each chunk of up to kQueueMax particles is
// split into the two queues by the branch of its first step, and each lane
// then keeps a particle in registers for every step of the launch,
// re-evaluating the switch at every step from the gather the update uses.
template <typename R, typename T, bool kYee, int kMinWaves, int kVar, bool kRec = false>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(kMinWaves))) void
k_push3_tiled(ParticlePtrs3<R> in_arg, ParticlePtrs3<R> out_arg,
              const uint32_t* __restrict__ perm, const int32_t* __restrict__ tile_start,
              TileGeom3 g, int chunk, const T* __restrict__ F, PushConst3 pc, uint8_t* trace,
              int64_t n, int steps, bool replay, DevStats* stats) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int wave_g[kWG / 64];
    __shared__ int wave_b[kWG / 64];
    // the state arrays' pointers are used only before and after the steps:
    // kept in LDS, not in scalar registers through the steps
    __shared__ ParticlePtrs3<R> io[2];
    if (threadIdx.x == 0) {
        io[0] = in_arg;
        io[1] = out_arg;
    }
    const ParticlePtrs3<R>& in = io[0];
    const ParticlePtrs3<R>& out = io[1];

    const int ntiles = g.ntx * g.nty * g.ntz;
    // consecutive tiles on the same XCD (workgroup b runs on XCD b % 8)
    const int tile = (int)(blockIdx.x % 8) * chunk + (int)(blockIdx.x / 8);
    if (tile >= ntiles) return;
    const int W = g.window;
    const int WWW = W * W * W;
    T* lds = reinterpret_cast<T*>(smem);
    uint16_t* queue = reinterpret_cast<uint16_t*>(
        smem + (((size_t)WWW * 6 * sizeof(T) + 15) & ~(size_t)15));

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tx = tile % g.ntx;
    const int tyz = tile / g.ntx;
    const int ty = tyz % g.nty;
    const int tz = tyz / g.nty;
    const int oi = tx * g.tile - g.halo;
    const int oj = ty * g.tile - g.halo;
    const int ol = tz * g.tile - g.halo;

    // stage the window: one (j, l) row (W records of 6 values, contiguous in
    // HBM) per wave iteration, written to the six component planes
    for (int row = wave; row < W * W; row += kWG / 64) {
        const int ll = row / W;
        const int rr = row - ll * W;
        const int gj = wrap_index(oj + rr, pc.b.ny);
        const int gl = wrap_index(ol + ll, pc.nz);
        const T* grow = F + ((size_t)gl * pc.b.ny + gj) * pc.b.nx * 6;
        for (int e = lane; e < W * 6; e += 64) {
            const int c = e / 6;
            const int k = e - c * 6;
            const int gi = wrap_index(oi + c, pc.b.nx);
            lds[((k * W + ll) * W + rr) * W + c] = grow[gi * 6 + k];
        }
    }
    __syncthreads();

    const Consts3<R> K = make_consts3<R>(pc);
    TileAcc3<T> acc{lds, GlobalAcc3<T>{F, pc.b.nx, pc.b.ny, pc.nz}, oi, oj, ol, W, false};
    const int64_t p0 = tile_start[tile];
    const int64_t p1 = tile_start[tile + 1];
    unsigned cnt_g = 0, cnt_b = 0, cnt_h = 0;
    double maxres = 0.0;

    for (int64_t base = p0; base < p1; base += kQueueMax) {
        const int m = (int)((p1 - base) < kQueueMax ? (p1 - base) : kQueueMax);
        // the branch of the launch's first step, stable split into the queues
        const int nG = split_queues<kWG>(m, queue, wave_g, wave_b, [&](int t) {
            const int64_t p = base + t;
            const int64_t src = perm ? (int64_t)perm[p] : p;
            if (replay) return trace[in.b.id ? (int64_t)in.b.id[src] : p] == 0;
            const double qm = in.b.qm ? in.b.qm[src] : pc.b.qm;
            Sample3<R> s;
            gather3<R, false, kYee>(acc, pc, K, in.b.x[src], in.b.y[src], in.z[src], s);
            return switch_gca(s.E, s.B, in.b.ux[src], in.b.uy[src], in.b.uz[src], qm, pc.b, K);
        });
        for (int q = threadIdx.x; q < m; q += kWG) {
            const int64_t p = base + queue[q];
            const int64_t src = perm ? (int64_t)perm[p] : p;
            const bool keep = perm && out.b.x == in.b.x;
            const int64_t slot = keep ? src : p;   // where the particle is written
            const int64_t tid = in.b.id ? (int64_t)in.b.id[src] : slot;   // trace column
            Regs3<R> r;
            load_particle3(in, src, pc.b.qm, r);
            uint32_t fl = 0;
            bool gca = q < nG;
            for (int st = 0; st < steps; ++st) {
                uint8_t* tr = trace ? trace + (int64_t)st * n : nullptr;
                if constexpr (kRec) record_state3(in.b.rec + (int64_t)st * 9 * n, n, tid, r);
                // the gather at x^n serves the switch and the update; the
                // gradients are formed for the branch of the previous step
                const bool prev = gca;
                Sample3<R> smp;
                acc.miss = false;
                if (prev)
                    gather3<R, true, kYee>(acc, pc, K, r.x, r.y, r.z, smp);
                else
                    gather3<R, false, kYee>(acc, pc, K, r.x, r.y, r.z, smp);
                if (st > 0) {
                    if (replay)
                        gca = tr[tid] == 0;
                    else
                        gca = switch_gca(smp.E, smp.B, r.ux, r.uy, r.uz, r.qm, pc.b, K);
                    if (gca && !prev) gather3<R, true, kYee>(acc, pc, K, r.x, r.y, r.z, smp);
                }
                double res = 0.0;
                if (gca)
                    fl |= gca_step3<R, kYee, var_exact(kVar), kVar == kVarMirror,
                                    kVar == kVarPhase, kVar == kVarExactCurv>(acc, smp, r, pc,
                                                                              K, res);
                else
                    boris_step3(smp, r, pc, K);
                fl |= finite_flag3(r);
                if (acc.miss) {
                    fl |= ST_HALO;
                    ++cnt_h;
                }
                if (tr && !replay) tr[tid] = gca ? 0 : 1;
                if (gca) {
                    ++cnt_g;
                    maxres = nan_max(maxres, res);
                } else {
                    ++cnt_b;
                }
            }
            store_particle3(in, out, slot, src, r, fl);
        }
        __syncthreads();   // the queue is rebuilt for the next chunk
    }
    if (stats) flush_stats(stats, cnt_g, cnt_b, cnt_h, maxres);
}

template <typename R, typename T, int kMinWaves, int kVar, bool kRec = false>
hipError_t launch_push3_frame(const Push3Launch& L, const ParticlePtrs3<R>& in,
                              const ParticlePtrs3<R>& out, const PushConst3& pc,
                              hipStream_t stream) {
    const T* F = static_cast<const T*>(L.fields);
    if (L.kind == PushKind::Global) {
        if (kRec) return hipErrorInvalidValue;   // records: the tiled kernel only
        const unsigned blocks = (unsigned)((L.n + kWG - 1) / kWG);
        const int ns = L.steps > 0 ? L.steps : 1;
        if (L.yee)
            hipLaunchKernelGGL((k_push3_global<R, T, true, kVar>), dim3(blocks), dim3(kWG), 0,
                               stream, in, out, L.perm, L.n, ns, F, pc, L.trace, L.replay,
                               L.stats);
        else
            hipLaunchKernelGGL((k_push3_global<R, T, false, kVar>), dim3(blocks), dim3(kWG),
                               0, stream, in, out, L.perm, L.n, ns, F, pc, L.trace, L.replay,
                               L.stats);
        return hipGetLastError();
    }
    const int ntiles = L.geom.ntx * L.geom.nty * L.geom.ntz;
    const int chunk = (ntiles + 7) / 8;
    const int ns = L.steps > 0 ? L.steps : 1;
    const size_t lds = tiled3_lds_bytes(L.geom.window, sizeof(T));
    if (L.yee) {
        auto kfn = k_push3_tiled<R, T, true, kMinWaves, kVar, kRec>;
        hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
        hipLaunchKernelGGL(kfn, dim3(8 * chunk), dim3(kWG), lds, stream, in, out, L.perm,
                           L.tile_start, L.geom, chunk, F, pc, L.trace, L.n, ns, L.replay,
                           L.stats);
    } else {
        auto kfn = k_push3_tiled<R, T, false, kMinWaves, kVar, kRec>;
        hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
        hipLaunchKernelGGL(kfn, dim3(8 * chunk), dim3(kWG), lds, stream, in, out, L.perm,
                           L.tile_start, L.geom, chunk, F, pc, L.trace, L.n, ns, L.replay,
                           L.stats);
    }
    return hipGetLastError();
}

// the exact frame exists for the binary64 form only (the host rejects the
// other combination)
template <typename R, typename T, int kMinWaves>
hipError_t launch_push3(const Push3Launch& L, const ParticlePtrs3<R>& in,
                        const ParticlePtrs3<R>& out, const PushConst3& pc, hipStream_t stream) {
    if (L.n == 0) return hipSuccess;
    // start-state records (the adjoint's recomputation): instances of their
    // own, in the binary64 parity arithmetic with the reduced frame only
    if (in.b.rec) {
        if constexpr (!kMixed<R> && GCB_FAST_ARITH == 0) {
            if (L.exact || L.mirror || L.phase) return hipErrorInvalidValue;
            return launch_push3_frame<R, T, kMinWaves, kVarReduced, true>(L, in, out, pc,
                                                                          stream);
        } else {
            return hipErrorInvalidValue;
        }
    }
    if constexpr (!kMixed<R>) {
        if (L.exact && pc.b.curvature)
            return launch_push3_frame<R, T, kMinWaves, kVarExactCurv>(L, in, out, pc, stream);
        if (L.exact) return launch_push3_frame<R, T, kMinWaves, kVarExact>(L, in, out, pc, stream);
    } else {
        if (L.exact) return hipErrorInvalidValue;
    }
    if (L.mirror) return launch_push3_frame<R, T, kMinWaves, kVarMirror>(L, in, out, pc, stream);
    if (L.phase) return launch_push3_frame<R, T, kMinWaves, kVarPhase>(L, in, out, pc, stream);
    return launch_push3_frame<R, T, kMinWaves, kVarReduced>(L, in, out, pc, stream);
}

}  // namespace GCB_KERN_NS
}  // namespace gcb
