// Field sources for the gather: the node-interleaved device array in HBM,
// and the LDS window of a tile with a global-memory fallback.
//
// Two interfaces:
//   quad(k, i, j, ...)   the 2x2 node values of component k around cell (i, j)
//                        (any lattice offsets; used with a runtime stagger table)
//   locate(...)/load4()  the 2D Yee lattice: the six components use four
//                        weight sets (x offset 0 or 1/2, y offset 0 or 1/2);
//                        locate() resolves the four 2x2 stencils once per
//                        gather point, load4() fetches one component.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gcb_common.hpp"

namespace gcb {

// 24-bit integer multiply (small non-negative operands)
GCB_HD int mul24(int a, int b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __mul24(a, b);
#else
    return a * b;
#endif
}

// Loader of the LDS window (component planes of W x W nodes): node (0,0) of
// each weight set at element off[set] of a plane.
template <typename T>
struct LdsLoad {
    const T* lds;
    const int* off;
    int W, WW;
    template <typename R>
    GCB_HD void load4(int set, int k, R& f00, R& f10, R& f01,
                                          R& f11) const {
        const T* p = lds + mul24(k, WW) + off[set];
        f00 = (R)p[0];
        f10 = (R)p[1];
        f01 = (R)p[W];
        f11 = (R)p[W + 1];
    }
};

// Weight-set indices of the Yee lattice: bit 0 = x offset 1/2, bit 1 = y offset 1/2.
// Ex (1/2,0) -> 1, Ey (0,1/2) -> 2, Ez (0,0) -> 0, Bx (0,1/2) -> 2, By (1/2,0) -> 1,
// Bz (1/2,1/2) -> 3.
constexpr int kYeeSet[6] = {1, 2, 0, 2, 1, 3};

// Device layout of the fields: node-interleaved, F[(j*nx + i)*6 + k], with k
// the component (Ex, Ey, Ez, Bx, By, Bz) at that component's own node (i, j).
// The six values a node contributes sit in one 48-byte (24-byte for float)
// record, so the 2x2 stencils of all components around a point touch three
// rows of three adjacent records.
template <typename T>
struct GlobalAcc {
    const T* __restrict__ F;
    int nx, ny;

    GCB_HD void quad(int k, int i, int j, double& f00, double& f10,
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

    // Yee stencils: ia/ib = floor of the x coordinate for offsets 0 and 1/2,
    // ja/jb likewise in y.
    struct Loc {
        const T* row[2][2];   // [y set][row 0/1]
        int col[2][2];        // [x set][column 0/1], in elements
    };

    GCB_HD void locate(int ia, int ib, int ja, int jb, Loc& L) const {
        const int xi[2] = {ia, ib};
        const int yj[2] = {ja, jb};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int c0 = wrap_index(xi[s], nx);
            const int c1 = (c0 + 1 == nx) ? 0 : c0 + 1;
            L.col[s][0] = c0 * 6;
            L.col[s][1] = c1 * 6;
            const int r0 = wrap_index(yj[s], ny);
            const int r1 = (r0 + 1 == ny) ? 0 : r0 + 1;
            L.row[s][0] = F + (size_t)r0 * nx * 6;
            L.row[s][1] = F + (size_t)r1 * nx * 6;
        }
    }

};

// Loader of the global array for one located gather point.
template <typename T>
struct GlobalLoad {
    const typename GlobalAcc<T>::Loc& L;
    template <typename R>
    GCB_HD void load4(int set, int k, R& f00, R& f10, R& f01,
                                          R& f11) const {
        const int sx = set & 1, sy = set >> 1;
        f00 = (R)L.row[sy][0][L.col[sx][0] + k];
        f10 = (R)L.row[sy][0][L.col[sx][1] + k];
        f01 = (R)L.row[sy][1][L.col[sx][0] + k];
        f11 = (R)L.row[sy][1][L.col[sx][1] + k];
    }
};

// W x W nodes of all six components staged in LDS, covering global nodes
// [oi, oi + W) x [oj, oj + W) (periodic), one plane per component
// (lds[(k*W + j)*W + i]): the lanes of a wavefront gather at scattered nodes,
// and in component planes neighbouring nodes sit in neighbouring banks, where
// the 6-value node records of the global layout would fold them onto a
// quarter of the banks.  A stencil that does not fit in the window is read
// from global memory instead (same values) and noted in `miss`.
template <typename T>
struct TileAcc {
    const T* lds;
    const T* __restrict__ F;
    int nx, ny, oi, oj, W;
    mutable bool miss;

    GCB_HD void quad(int k, int i, int j, double& f00, double& f10,
                                         double& f01, double& f11) const {
        int di = i - oi;
        int dj = j - oj;
        const unsigned lim = (unsigned)(W - 1);
        if ((unsigned)di >= lim) di += (di < 0) ? nx : -nx;
        if ((unsigned)dj >= lim) dj += (dj < 0) ? ny : -ny;
        if ((unsigned)di < lim && (unsigned)dj < lim) {
            const T* r0 = lds + (k * W + dj) * W + di;
            f00 = (double)r0[0];
            f10 = (double)r0[1];
            f01 = (double)r0[W];
            f11 = (double)r0[W + 1];
        } else {
            miss = true;
            GlobalAcc<T> g{F, nx, ny};
            g.quad(k, i, j, f00, f10, f01, f11);
        }
    }

    // Resolve the Yee stencils of a gather point.  Returns true and fills
    // `off` (LDS element offset of node (0,0) per weight set) when all four
    // stencils lie inside the window; otherwise fills the global fallback.
    // ib <= ia and jb <= ja (the 1/2-offset lattice's floor is never larger).
    GCB_HD bool locate(int ia, int ib, int ja, int jb, int off[4],
                                           typename GlobalAcc<T>::Loc& g) const {
        int da = ia - oi;
        int ea = ja - oj;
        if (da < 0 || da > W - 2) da += (da < 0) ? nx : -nx;
        if (ea < 0 || ea > W - 2) ea += (ea < 0) ? ny : -ny;
        const int sa = ia - ib, sb = ja - jb;   // 0 or 1 for finite coordinates
        const int db = da - sa;
        const int eb = ea - sb;
        const bool in = (unsigned)sa <= 1u && (unsigned)sb <= 1u && db >= 0 && eb >= 0 &&
                        da <= W - 2 && ea <= W - 2;
        if (in) {
            off[0] = mul24(ea, W) + da;
            off[1] = mul24(ea, W) + db;
            off[2] = mul24(eb, W) + da;
            off[3] = mul24(eb, W) + db;
        } else {
            miss = true;
            GlobalAcc<T> gl{F, nx, ny};
            gl.locate(ia, ib, ja, jb, g);
        }
        return in;
    }
};

}  // namespace gcb
