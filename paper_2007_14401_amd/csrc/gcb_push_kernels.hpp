// Push kernels, templated on the bulk arithmetic type R (double: binary64
// form; float: mixed form) and the field storage type T.
//
// Both kernels read particle slot perm[p] of `in` (slot p when perm is null)
// and write slot p of `out`: on the step of a cell sort, perm is the sort's
// permutation and the push moves the state into tile order on the way (no
// separate permutation pass; `in` and `out` are then different buffers).
// The tiled kernel given a permutation with `out` equal to `in` keeps the
// order instead: it works through the tiles in the permutation's order and
// writes each particle back to the slot it was read from (gcb_params
// keep_order).
//
// k_push_global: one lane per particle, any particle order, gathers through
//   the cache hierarchy from the node-interleaved field array.
// k_push_tiled: one workgroup per tile of cell-sorted particles for all the
//   steps of a launch (those between two sorts).  The tile's field window
//   (tile + halo, all six components) is staged once in LDS; the particles
//   are split into two queues by the branch of their first step (so that a
//   wavefront starts on one branch of the coupled step) and each lane keeps
//   its particle in registers for all steps, re-evaluating the switch at
//   every step.
//
// Included by exactly one translation unit per form (the binary64 one is
// compiled with -ffp-contract=off).
#pragma once

#include <hip/hip_runtime.h>

#include "gcb_access.hpp"
#include "gcb_internal.h"
#include "gcb_math.hpp"
#include "gcb_queues.hpp"

// The kernels are compiled once per form and contraction setting; the
// namespace of their instances is set by the including unit.
#ifndef GCB_KERN_NS
#define GCB_KERN_NS kern
#endif

namespace gcb {
namespace GCB_KERN_NS {

constexpr int kWG = 256;

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = nan_max(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ void flush_stats(DevStats* st, unsigned gca, unsigned boris,
                                            unsigned halo, double maxres) {
    // wave-level reduction, one atomic per wave and counter
    unsigned long long g = gca, b = boris, h = halo;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        g += __shfl_xor(g, off, 64);
        b += __shfl_xor(b, off, 64);
        h += __shfl_xor(h, off, 64);
    }
    const double m = wave_max(maxres);
    st += blockIdx.x % kStatSlots;
    if ((threadIdx.x & 63) == 0) {
        if (g) atomicAdd(&st->gca_steps, g);
        if (b) atomicAdd(&st->boris_steps, b);
        if (h) atomicAdd(&st->halo_misses, h);
        if (m > 0.0) atomicMax(&st->max_res_bits, (unsigned long long)__double_as_longlong(m));
    }
}

template <typename R>
__device__ __forceinline__ void load_particle(const ParticlePtrs<R>& in, int64_t p,
                                              double qm_default, Regs<R>& r) {
    r.x = in.x[p];
    r.y = in.y[p];
    r.xp = in.xp[p];
    r.yp = in.yp[p];
    r.ux = in.ux[p];
    r.uy = in.uy[p];
    r.uz = in.uz[p];
    r.qm = in.qm ? in.qm[p] : qm_default;
}

// the start state of a step for the adjoint: slot i of the step's records
template <typename R>
__device__ __forceinline__ void record_state(double* rec, int64_t n, int64_t i,
                                             const Regs<R>& r) {
    rec[i] = r.x;
    rec[n + i] = r.y;
    rec[2 * n + i] = r.xp;
    rec[3 * n + i] = r.yp;
    rec[4 * n + i] = (double)r.ux;
    rec[5 * n + i] = (double)r.uy;
    rec[6 * n + i] = (double)r.uz;
}

template <typename R>
__device__ __forceinline__ void store_particle(const ParticlePtrs<R>& in,
                                               const ParticlePtrs<R>& out, int64_t p,
                                               int64_t src, const Regs<R>& r,
                                               uint32_t flags) {
    out.x[p] = r.x;
    out.y[p] = r.y;
    out.xp[p] = r.xp;
    out.yp[p] = r.yp;
    out.ux[p] = r.ux;
    out.uy[p] = r.uy;
    out.uz[p] = r.uz;
    out.status[p] = (uint8_t)(in.status[src] | flags);
    if (out.x != in.x) {   // out-of-place step after a sort: carry the rest along
        if (in.qm) out.qm[p] = r.qm;
        if (in.id) out.id[p] = in.id[src];
    }
}

// one coupled step for a particle already in registers (kVar: the
// guiding-center branch in the paper's reduced frame, in the exact frame of
// Sec. 2.2, or with the mirror terms)
template <typename R, bool kYee, int kVar, class Acc>
__device__ __forceinline__ uint32_t coupled_update(const Acc& acc, bool gca, Regs<R>& r,
                                                   const PushConst& pc, const Consts<R>& K,
                                                   double& res) {
    uint32_t fl = 0;
    res = 0.0;
    if (gca) {
        Sample<R> s;
        gather<R, true, kYee>(acc, pc, K, r.x, r.y, s);
        fl = gca_step<R, kYee, var_exact(kVar), kVar == kVarMirror, kVar == kVarPhase,
                      kVar == kVarExactCurv>(acc, s, r, pc, K, res);
    } else {
        Sample<R> s;
        gather<R, false, kYee>(acc, pc, K, r.x, r.y, s);
        boris_step(s, r, pc, K);
    }
    return fl | finite_flag(r);
}

// ns steps of one particle per lane (the particle stays in registers between
// them); trace (per step n bytes) is indexed by id when ids are present
template <typename R, typename T, bool kYee, int kVar, bool kRec = false>
__global__ __launch_bounds__(kWG) void k_push_global(ParticlePtrs<R> in, ParticlePtrs<R> out,
                                                      const uint32_t* __restrict__ perm,
                                                      int64_t n, int ns, const T* __restrict__ F,
                                                      PushConst pc, uint8_t* trace,
                                                      bool replay, DevStats* stats) {
    const int64_t p = (int64_t)blockIdx.x * kWG + threadIdx.x;
    const bool active = p < n;
    unsigned cnt_g = 0, cnt_b = 0;
    double maxres = 0.0;
    if (active) {
        const Consts<R> K = make_consts<R>(pc);
        GlobalAcc<T> acc{F, pc.nx, pc.ny};
        const int64_t src = perm ? (int64_t)perm[p] : p;
        Regs<R> r;
        load_particle(in, src, pc.qm, r);
        const int64_t ti = in.id ? (int64_t)in.id[src] : p;
        uint32_t fl = 0;
        for (int s = 0; s < ns; ++s) {
            uint8_t* tr = trace ? trace + (size_t)s * n : nullptr;
            if constexpr (kRec) record_state(in.rec + (int64_t)s * 7 * n, n, ti, r);
            bool gca;
            if (replay) {
                gca = tr[ti] == 0;
            } else {
                Sample<R> smp;
                gather<R, false, kYee>(acc, pc, K, r.x, r.y, smp);
                gca = switch_gca(smp.E, smp.B, r.ux, r.uy, r.uz, r.qm, pc, K);
            }
            double res;
            fl |= coupled_update<R, kYee, kVar>(acc, gca, r, pc, K, res);
            if (tr && !replay) tr[ti] = gca ? 0 : 1;
            if (gca) {
                ++cnt_g;
                maxres = nan_max(maxres, res);
            } else {
                ++cnt_b;
            }
        }
        store_particle(in, out, p, src, r, fl);
    }
    if (stats) flush_stats(stats, cnt_g, cnt_b, 0, maxres);
}

// One workgroup per tile of cell-sorted particles, for all `steps` steps of
// a launch (the steps between two cell sorts, so the particle-to-tile
// assignment of the last sort holds for all of them).  The tile's field
// window (six W x W component planes) is staged in LDS once.  Its particles
// are taken in chunks of up to kTiledChunk: the switch is evaluated for each
// at the launch's first step and the chunk is split into two queues
// (guiding center first, Boris from the back).  The queues are cut into
// slices of 64, the guiding-center slices first; each wavefront takes the
// next slice from a counter in LDS until none is left, so a wavefront starts
// with particles of one branch, and one that finishes a short Boris slice
// takes another instead of idling while the workgroup's other wavefronts
// finish theirs (the workgroup's LDS is held until its last wavefront ends).
// Each lane keeps its particle in registers for every step of the launch,
// evaluating the switch itself at every step (Sec. 4.1) from the gather at
// x^n that the update uses.  Particles seldom change branch between two
// sorts, so the wavefronts mostly stay on one branch; one that holds both
// takes both, with the same results.
template <typename R, typename T, bool kYee, int kMinWaves, int kVar, bool kRec = false>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(kMinWaves))) void
k_push_tiled(ParticlePtrs<R> in_arg, ParticlePtrs<R> out_arg, const uint32_t* __restrict__ perm,
             const int32_t* __restrict__ tile_start, TileGeom g, int chunk,
             const T* __restrict__ F, PushConst pc, uint8_t* trace, int64_t n, int steps,
             bool replay, DevStats* stats) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int wave_g[kWG / 64];
    __shared__ int wave_b[kWG / 64];
    __shared__ int next_slice;
    // The state arrays are used only before and after the steps of a chunk:
    // their twenty pointers are kept in LDS and read where they are used, so
    // that they do not occupy scalar registers through the steps.
    __shared__ ParticlePtrs<R> io[2];
    if (threadIdx.x == 0) {
        io[0] = in_arg;
        io[1] = out_arg;
    }
    const ParticlePtrs<R>& in = io[0];
    const ParticlePtrs<R>& out = io[1];

    const int ntiles = g.ntx * g.nty;
    // consecutive tiles on the same XCD: workgroups are dealt to the 8 XCDs
    // round-robin, so workgroup b runs on XCD b % 8
    const int tile = (int)(blockIdx.x % 8) * chunk + (int)(blockIdx.x / 8);
    if (tile >= ntiles) return;
    const int W = g.window;
    T* lds = reinterpret_cast<T*>(smem);
    uint16_t* queue = reinterpret_cast<uint16_t*>(
        smem + (((size_t)W * W * 6 * sizeof(T) + 15) & ~(size_t)15));

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tx = tile % g.ntx;
    const int ty = tile / g.ntx;
    const int oi = tx * g.tile - g.halo;
    const int oj = ty * g.tile - g.halo;

    // stage the window: a row of W records (6 W values, contiguous in the
    // node-interleaved array) per wave iteration, written to the six
    // component planes; a lane's columns are the same in every row, so their
    // offsets are formed once, and the loads of two rows are in flight
    // together (6 W <= 64 kCols: the host keeps W <= 64)
    {
        constexpr int kCols = 6;
        int goff[kCols], loff[kCols];
#pragma unroll
        for (int u = 0; u < kCols; ++u) {
            const int e = lane + 64 * u;
            const int c = e / 6;
            const int k = e - c * 6;
            const bool ok = e < W * 6;
            goff[u] = ok ? wrap_index(oi + c, pc.nx) * 6 + k : -1;
            loff[u] = ok ? k * W * W + c : 0;
        }
        constexpr int kRowStep = 2 * (kWG / 64);
        for (int rr = wave; rr < W; rr += kRowStep) {
            const int r2 = rr + kWG / 64;
            const bool two = r2 < W;
            const T* row0 = F + (size_t)wrap_index(oj + rr, pc.ny) * pc.nx * 6;
            const T* row1 = F + (size_t)wrap_index(oj + (two ? r2 : rr), pc.ny) * pc.nx * 6;
            T v0[kCols], v1[kCols];
#pragma unroll
            for (int u = 0; u < kCols; ++u) {
                v0[u] = goff[u] >= 0 ? row0[goff[u]] : (T)0;
                v1[u] = goff[u] >= 0 ? row1[goff[u]] : (T)0;
            }
#pragma unroll
            for (int u = 0; u < kCols; ++u) {
                if (goff[u] >= 0) {
                    lds[loff[u] + rr * W] = v0[u];
                    if (two) lds[loff[u] + r2 * W] = v1[u];
                }
            }
        }
    }
    __syncthreads();

    const Consts<R> K = make_consts<R>(pc);
    TileAcc<T> acc{lds, F, pc.nx, pc.ny, oi, oj, W, false};
    const int64_t p0 = tile_start[tile];
    const int64_t p1 = tile_start[tile + 1];
    unsigned cnt_g = 0, cnt_b = 0, cnt_h = 0;
    double maxres = 0.0;

    for (int64_t base = p0; base < p1; base += kTiledChunk) {
        const int m = (int)((p1 - base) < kTiledChunk ? (p1 - base) : kTiledChunk);
        // (the barriers of the split order this reset before any slice is
        // taken, and the barrier at the end of the previous chunk after it)
        if (threadIdx.x == 0) next_slice = 0;
        // the branch of the launch's first step per particle, split into
        // the two queues
        const int nG = split_queues<kWG>(m, queue, wave_g, wave_b, [&](int q) {
            const int64_t p = base + q;
            const int64_t src = perm ? (int64_t)perm[p] : p;
            if (replay) return trace[in.id ? (int64_t)in.id[src] : p] == 0;
            Sample<R> smp;
            gather<R, false, kYee>(acc, pc, K, in.x[src], in.y[src], smp);
            const double qm = in.qm ? in.qm[src] : pc.qm;
            return switch_gca(smp.E, smp.B, in.ux[src], in.uy[src], in.uz[src], qm, pc, K);
        });
        const int sG = (nG + 63) >> 6;                 // guiding-center slices
        const int sAll = sG + ((m - nG + 63) >> 6);   // and the Boris ones
        for (;;) {
            int sl = 0;
            if (lane == 0) sl = atomicAdd(&next_slice, 1);
            sl = __builtin_amdgcn_readfirstlane(sl);
            if (sl >= sAll) break;
            const bool gslice = sl < sG;
            const int q = gslice ? sl * 64 + lane : nG + (sl - sG) * 64 + lane;
            if (q >= (gslice ? nG : m)) continue;   // the slice's unfilled lanes
            const int64_t p = base + queue[q];
            const int64_t src = perm ? (int64_t)perm[p] : p;
            const bool keep = perm && out.x == in.x;
            const int64_t slot = keep ? src : p;   // where the particle is written
            const int64_t tid = in.id ? (int64_t)in.id[src] : slot;   // trace column
            Regs<R> r;
            load_particle(in, src, pc.qm, r);
            uint32_t fl = 0;
            bool gca = gslice;
            for (int s = 0; s < steps; ++s) {
                uint8_t* tr = trace ? trace + (int64_t)s * n : nullptr;
                if constexpr (kRec) record_state(in.rec + (int64_t)s * 7 * n, n, tid, r);
                // the gather at x^n serves the switch and the update; the
                // gradients are formed for the branch of the previous step
                const bool prev = gca;
                Sample<R> smp;
                acc.miss = false;
                if (prev)
                    gather<R, true, kYee>(acc, pc, K, r.x, r.y, smp);
                else
                    gather<R, false, kYee>(acc, pc, K, r.x, r.y, smp);
                if (s > 0) {
                    if (replay)
                        gca = tr[tid] == 0;
                    else
                        gca = switch_gca(smp.E, smp.B, r.ux, r.uy, r.uz, r.qm, pc, K);
                    if (gca && !prev) gather<R, true, kYee>(acc, pc, K, r.x, r.y, smp);
                }
                double res = 0.0;
                if (gca)
                    fl |= gca_step<R, kYee, var_exact(kVar), kVar == kVarMirror,
                                   kVar == kVarPhase, kVar == kVarExactCurv>(acc, smp, r, pc,
                                                                             K, res);
                else
                    boris_step(smp, r, pc, K);
                fl |= finite_flag(r);
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
            store_particle(in, out, slot, src, r, fl);
        }
        __syncthreads();   // the queue is rebuilt for the next chunk
    }
    if (stats) flush_stats(stats, cnt_g, cnt_b, cnt_h, maxres);
}

template <typename R, typename T, int kMinWaves, int kVar, bool kRec = false>
hipError_t launch_push_frame(const PushLaunch& L, const ParticlePtrs<R>& in,
                             const ParticlePtrs<R>& out, const PushConst& pc,
                             hipStream_t stream) {
    const T* F = static_cast<const T*>(L.fields);
    if (L.kind == PushKind::Global) {
        const unsigned blocks = (unsigned)((L.n + kWG - 1) / kWG);
        const int ns = L.steps > 0 ? L.steps : 1;
        if (L.yee)
            hipLaunchKernelGGL((k_push_global<R, T, true, kVar, kRec>), dim3(blocks), dim3(kWG), 0,
                               stream, in, out, L.perm, L.n, ns, F, pc, L.trace, L.replay,
                               L.stats);
        else
            hipLaunchKernelGGL((k_push_global<R, T, false, kVar, kRec>), dim3(blocks), dim3(kWG),
                               0,
                               stream, in, out, L.perm, L.n, ns, F, pc, L.trace, L.replay,
                               L.stats);
        return hipGetLastError();
    }
    const int ntiles = L.geom.ntx * L.geom.nty;
    const int chunk = (ntiles + 7) / 8;
    const int ns = L.steps > 0 ? L.steps : 1;
    const size_t lds = tiled_lds_bytes(L.geom.window, sizeof(T));
    if (L.yee) {
        auto kfn = k_push_tiled<R, T, true, kMinWaves, kVar, kRec>;
        hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
        hipLaunchKernelGGL(kfn, dim3(8 * chunk), dim3(kWG), lds, stream, in, out, L.perm,
                           L.tile_start, L.geom, chunk, F, pc, L.trace, L.n, ns, L.replay,
                           L.stats);
    } else {
        auto kfn = k_push_tiled<R, T, false, kMinWaves, kVar, kRec>;
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
hipError_t launch_push(const PushLaunch& L, const ParticlePtrs<R>& in,
                       const ParticlePtrs<R>& out, const PushConst& pc, hipStream_t stream) {
    if (L.n == 0) return hipSuccess;
    // start-state records (the adjoint's recomputation): instances of their
    // own, in the binary64 parity arithmetic with the paper's reduced frame
    // only (the adjoint's scope)
    if (in.rec) {
        if constexpr (!kMixed<R> && GCB_FAST_ARITH == 0) {
            if (L.exact || L.mirror || L.phase) return hipErrorInvalidValue;
            return launch_push_frame<R, T, kMinWaves, kVarReduced, true>(L, in, out, pc, stream);
        } else {
            return hipErrorInvalidValue;
        }
    }
    if constexpr (!kMixed<R>) {
        if (L.exact && pc.curvature)
            return launch_push_frame<R, T, kMinWaves, kVarExactCurv>(L, in, out, pc, stream);
        if (L.exact) return launch_push_frame<R, T, kMinWaves, kVarExact>(L, in, out, pc, stream);
    } else {
        if (L.exact) return hipErrorInvalidValue;
    }
    if (L.mirror) return launch_push_frame<R, T, kMinWaves, kVarMirror>(L, in, out, pc, stream);
    if (L.phase) return launch_push_frame<R, T, kMinWaves, kVarPhase>(L, in, out, pc, stream);
    return launch_push_frame<R, T, kMinWaves, kVarReduced>(L, in, out, pc, stream);
}

}  // namespace GCB_KERN_NS
}  // namespace gcb
