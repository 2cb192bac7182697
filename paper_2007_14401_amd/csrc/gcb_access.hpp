// Field sources for the gather: the node-interleaved device array in HBM,
// and the LDS window of a tile with a global-memory fallback.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gcb_common.hpp"

namespace gcb {

// Device layout of the fields: node-interleaved, F[(j*nx + i)*6 + k], with k
// the component (Ex, Ey, Ez, Bx, By, Bz) at that component's own node (i, j).
// The six values a node contributes sit in one 48-byte (24-byte for float)
// record, so the 2x2 stencils of all components around a point touch three
// rows of three adjacent records.
template <typename T>
struct GlobalAcc {
    const T* __restrict__ F;
    int nx, ny;

    __device__ __forceinline__ void quad(int k, int i, int j, double& f00, double& f10,
                                         double& f01, double& f11) const {
        const int i0 = wrap_index(i, nx);
        const int j0 = wrap_index(j, ny);
        const int i1 = (i0 + 1 == nx) ? 0 : i0 + 1;
        const int j1 = (j0 + 1 == ny) ? 0 : j0 + 1;
        const T* r0 = F + (size_t)j0 * nx * 6;
        const T* r1 = F + (size_t)j1 * nx * 6;
        f00 = (double)r0[i0 * 6 + k];
        f10 = (double)r0[i1 * 6 + k];
        f01 = (double)r1[i0 * 6 + k];
        f11 = (double)r1[i1 * 6 + k];
    }
};

// W x W nodes of all six components staged in LDS, covering global nodes
// [oi, oi + W) x [oj, oj + W) (periodic).  A stencil that does not fit in the
// window is read from global memory instead (same values) and noted in `miss`.
template <typename T>
struct TileAcc {
    const T* lds;
    const T* __restrict__ F;
    int nx, ny, oi, oj, W;
    mutable bool miss;

    __device__ __forceinline__ void quad(int k, int i, int j, double& f00, double& f10,
                                         double& f01, double& f11) const {
        int di = i - oi;
        int dj = j - oj;
        const unsigned lim = (unsigned)(W - 1);
        if ((unsigned)di >= lim) di += (di < 0) ? nx : -nx;
        if ((unsigned)dj >= lim) dj += (dj < 0) ? ny : -ny;
        if ((unsigned)di < lim && (unsigned)dj < lim) {
            const T* r0 = lds + (dj * W + di) * 6 + k;
            f00 = (double)r0[0];
            f10 = (double)r0[6];
            f01 = (double)r0[W * 6];
            f11 = (double)r0[W * 6 + 6];
        } else {
            miss = true;
            GlobalAcc<T> g{F, nx, ny};
            g.quad(k, i, j, f00, f10, f01, f11);
        }
    }
};

}  // namespace gcb
