// Field sources of the 3D gather: the node-interleaved device array in HBM
// and the LDS window of a 3D tile with a global-memory fallback.
//
// Every loader fills the 2x2x2 stencil of one component in the order
// f[dz*4 + dy*2 + dx] (dx, dy, dz in {0, 1} the node offsets along x, y, z).
// On the 3D Yee lattice each component sits on its own combination of half
// offsets, so the six components use six of the eight weight sets
// (bit 0: x offset 1/2, bit 1: y offset 1/2, bit 2: z offset 1/2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gcb_access.hpp"
#include "gcb_common.hpp"

namespace gcb {

// Ex (1/2,0,0) -> 1, Ey (0,1/2,0) -> 2, Ez (0,0,1/2) -> 4, Bx (0,1/2,1/2) -> 6,
// By (1/2,0,1/2) -> 5, Bz (1/2,1/2,0) -> 3.
constexpr int kYee3Set[6] = {1, 2, 4, 6, 5, 3};

// Device layout: F[((l*ny + j)*nx + i)*6 + k], component k at its own node
// (i, j, l): the 2D layout with the rows of all z planes stacked.
template <typename T>
struct GlobalAcc3 {
    const T* __restrict__ F;
    int nx, ny, nz;

    GCB_HD const T* row(int j, int l) const {
        return F + ((size_t)l * ny + j) * nx * 6;
    }

    // stencil of component k around cell (i, j, l), any offsets
    template <typename R>
    GCB_HD void oct(int k, int i, int j, int l, R f[8]) const {
        const int i0 = wrap_index(i, nx), j0 = wrap_index(j, ny), l0 = wrap_index(l, nz);
        const int i1 = (i0 + 1 == nx) ? 0 : i0 + 1;
        const int j1 = (j0 + 1 == ny) ? 0 : j0 + 1;
        const int l1 = (l0 + 1 == nz) ? 0 : l0 + 1;
        const int c0 = i0 * 6 + k, c1 = i1 * 6 + k;
        const T* r00 = row(j0, l0);
        const T* r10 = row(j1, l0);
        const T* r01 = row(j0, l1);
        const T* r11 = row(j1, l1);
        f[0] = (R)r00[c0]; f[1] = (R)r00[c1];
        f[2] = (R)r10[c0]; f[3] = (R)r10[c1];
        f[4] = (R)r01[c0]; f[5] = (R)r01[c1];
        f[6] = (R)r11[c0]; f[7] = (R)r11[c1];
    }

    // Yee stencils of one gather point: wrapped node pairs per axis and offset
    // (a = offset 0, b = offset 1/2)
    struct Loc {
        int col[2][2];   // [x set][node], element offsets i*6
        int jj[2][2];    // [y set][node]
        int ll[2][2];    // [z set][node]
    };

    GCB_HD void locate(const int fl[3][2], Loc& L) const {
        const int n[3] = {nx, ny, nz};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int c0 = wrap_index(fl[a][s], n[a]);
                const int c1 = (c0 + 1 == n[a]) ? 0 : c0 + 1;
                int* dst = a == 0 ? L.col[s] : (a == 1 ? L.jj[s] : L.ll[s]);
                dst[0] = a == 0 ? c0 * 6 : c0;
                dst[1] = a == 0 ? c1 * 6 : c1;
            }
    }
};

template <typename T>
struct GlobalLoad3 {
    const GlobalAcc3<T>& acc;
    const typename GlobalAcc3<T>::Loc& L;
    template <typename R>
    GCB_HD void load8(int set, int k, R f[8]) const {
        const int sx = set & 1, sy = (set >> 1) & 1, sz = set >> 2;
        const int c0 = L.col[sx][0] + k, c1 = L.col[sx][1] + k;
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy) {
                const T* r = acc.row(L.jj[sy][dy], L.ll[sz][dz]);
                f[dz * 4 + dy * 2] = (R)r[c0];
                f[dz * 4 + dy * 2 + 1] = (R)r[c1];
            }
    }
};

// Loader of the LDS window (component planes of W x W x W nodes,
// lds[((k*W + l)*W + j)*W + i]): node (0,0,0) of each weight set at element
// off[set] of a plane.
template <typename T>
struct LdsLoad3 {
    const T* lds;
    const int* off;
    int W, WW, WWW;
    template <typename R>
    GCB_HD void load8(int set, int k, R f[8]) const {
        const T* p = lds + mul24(k, WWW) + off[set];
        f[0] = (R)p[0];
        f[1] = (R)p[1];
        f[2] = (R)p[W];
        f[3] = (R)p[W + 1];
        f[4] = (R)p[WW];
        f[5] = (R)p[WW + 1];
        f[6] = (R)p[WW + W];
        f[7] = (R)p[WW + W + 1];
    }
};

// W^3 nodes of all six components staged in LDS, covering global nodes
// [oi, oi+W) x [oj, oj+W) x [ol, ol+W) (periodic), one plane per component.
// A stencil outside the window is read from global memory (same values) and
// noted in `miss`.
template <typename T>
struct TileAcc3 {
    const T* lds;
    GlobalAcc3<T> g;
    int oi, oj, ol, W;
    mutable bool miss;

    // window coordinate of node index i along an axis of n nodes with window
    // origin o, or -1 if the pair (i, i+1) is not inside the window
    GCB_HD int local(int i, int o, int n) const {
        int d = i - o;
        if (d < 0 || d > W - 2) d += (d < 0) ? n : -n;
        return (d >= 0 && d <= W - 2) ? d : -1;
    }

    template <typename R>
    GCB_HD void oct(int k, int i, int j, int l, R f[8]) const {
        const int di = local(i, oi, g.nx), dj = local(j, oj, g.ny), dl = local(l, ol, g.nz);
        if (di >= 0 && dj >= 0 && dl >= 0) {
            const int off = (dl * W + dj) * W + di;
            LdsLoad3<T> ld{lds, &off, W, W * W, W * W * W};
            ld.template load8<R>(0, k, f);
        } else {
            miss = true;
            g.template oct<R>(k, i, j, l, f);
        }
    }

    // Resolve the Yee stencils of a gather point from the floors fl[axis][s]
    // (s = 0: offset 0, s = 1: offset 1/2; the second is never larger).
    // Returns true and fills off[8] when every stencil lies in the window,
    // otherwise fills the global fallback.
    GCB_HD bool locate(const int fl[3][2], int off[8],
                       typename GlobalAcc3<T>::Loc& gl) const {
        const int o[3] = {oi, oj, ol};
        const int n[3] = {g.nx, g.ny, g.nz};
        int d[3][2];
        bool in = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int da = fl[a][0] - o[a];
            if (da < 0 || da > W - 2) da += (da < 0) ? n[a] : -n[a];
            const int sa = fl[a][0] - fl[a][1];   // 0 or 1 for finite coordinates
            d[a][0] = da;
            d[a][1] = da - sa;
            in = in && (unsigned)sa <= 1u && d[a][1] >= 0 && da <= W - 2;
        }
        if (in) {
#pragma unroll
            for (int s = 0; s < 8; ++s)
                off[s] = (mul24(d[2][s >> 2], W) + d[1][(s >> 1) & 1]) * W + d[0][s & 1];
        } else {
            miss = true;
            g.locate(fl, gl);
        }
        return in;
    }
};

}  // namespace gcb
