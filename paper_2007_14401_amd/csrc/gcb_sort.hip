// Cell sort of the particle state by tile, so that the particles of a tile
// are contiguous (coalesced structure-of-arrays access) and the tiled push
// kernel can stage one field window per workgroup.
//
// Pipeline (all on the caller's stream):
//   k_tile_keys   key = tile index of (x, y); idx = slot
//   LSD radix sort of (key, idx), 8 bits per pass, stable:
//     k_radix_hist     per-block digit histogram, digit-major [256][nblocks]
//     scan             exclusive scan of the histogram (3 kernels)
//     k_radix_scatter  wave-level multisplit ranks -> stable scatter
//   k_tile_bounds tile_start from the boundaries of the sorted keys
// The push kernel of the sort's step then reads the state through idx (the
// permutation) and writes it in tile order, so there is no permutation pass
// (the same for the curved-spacetime and 3D states).
//   k_gr_tile_keys: the keys of the curved-spacetime state ((r, theta) tiles
//                 of the grid cells)
//   k_tile_keys3:   the keys of the 3D state (cubic tiles)
#include <hip/hip_runtime.h>

#include "gcb_internal.h"

namespace gcb {
namespace {

constexpr int kSortWG = 256;
constexpr int kItemsPerWave = 1024;
constexpr int kItems = kItemsPerWave * (kSortWG / 64);   // 4096 per block
constexpr int kScanWG = 256;
constexpr int kScanItems = 4096;                          // per block of the scan

__global__ __launch_bounds__(kSortWG) void k_tile_keys(const double* __restrict__ x,
                                                       const double* __restrict__ y,
                                                       int64_t n, double inv_dx,
                                                       double inv_dy, TileGeom g,
                                                       uint32_t* keys, uint32_t* idx) {
    const int64_t p = (int64_t)blockIdx.x * kSortWG + threadIdx.x;
    if (p >= n) return;
    const double gx = floor(x[p] * inv_dx);
    const double gy = floor(y[p] * inv_dy);
    // clamp into the tile range (non-finite positions land in tile 0)
    int tx = (gx >= 0.0 && gx < 2.0e9) ? (int)gx / g.tile : 0;
    int ty = (gy >= 0.0 && gy < 2.0e9) ? (int)gy / g.tile : 0;
    tx = tx < g.ntx ? tx : g.ntx - 1;
    ty = ty < g.nty ? ty : g.nty - 1;
    const uint32_t key = (uint32_t)(ty * g.ntx + tx);
    keys[p] = key;
    idx[p] = (uint32_t)p;
}

// clamped tile coordinate of one position component (non-finite -> 0)
__device__ __forceinline__ int tile_coord(double v, double inv_d, int tile, int nt) {
    const double gc = floor(v * inv_d);
    const int t = (gc >= 0.0 && gc < 2.0e9) ? (int)gc / tile : 0;
    return t < nt ? t : nt - 1;
}

__global__ __launch_bounds__(kSortWG) void k_tile_keys3(const double* __restrict__ x,
                                                        const double* __restrict__ y,
                                                        const double* __restrict__ z,
                                                        int64_t n, double inv_dx,
                                                        double inv_dy, double inv_dz,
                                                        TileGeom3 g, uint32_t* keys,
                                                        uint32_t* idx) {
    const int64_t p = (int64_t)blockIdx.x * kSortWG + threadIdx.x;
    if (p >= n) return;
    const int tx = tile_coord(x[p], inv_dx, g.tile, g.ntx);
    const int ty = tile_coord(y[p], inv_dy, g.tile, g.nty);
    const int tz = tile_coord(z[p], inv_dz, g.tile, g.ntz);
    keys[p] = (uint32_t)((tz * g.nty + ty) * g.ntx + tx);
    idx[p] = (uint32_t)p;
}

// tile_start[t] = first sorted slot whose key is >= t, for t in [0, ntiles]:
// every slot i writes the starts of the tiles in (key[i-1], key[i]].
__global__ __launch_bounds__(kSortWG) void k_tile_bounds(const uint32_t* __restrict__ keys,
                                                         int64_t n, int ntiles,
                                                         int32_t* tile_start) {
    const int64_t i = (int64_t)blockIdx.x * kSortWG + threadIdx.x;
    if (i > n) return;
    const int lo = i == 0 ? -1 : (int)keys[i - 1];
    const int hi = i == n ? ntiles : (int)keys[i];
    for (int t = lo + 1; t <= hi; ++t) tile_start[t] = (int32_t)i;
}

// key = (r, theta) tile of the particle's grid cell, row-major tiles
__global__ __launch_bounds__(kSortWG) void k_gr_tile_keys(const double* __restrict__ r,
                                                          const double* __restrict__ th,
                                                          int64_t n, gr::GrConst g, int tile,
                                                          int ntx, uint32_t* keys,
                                                          uint32_t* idx) {
    const int64_t p = (int64_t)blockIdx.x * kSortWG + threadIdx.x;
    if (p >= n) return;
    int i, j;
    double wx, wy;
    gr::grid_cell(g, r[p], th[p], i, j, wx, wy);
    keys[p] = (uint32_t)((j / tile) * ntx + i / tile);
    idx[p] = (uint32_t)p;
}

__global__ __launch_bounds__(kSortWG) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                        int64_t n, int shift,
                                                        int nblocks, uint32_t* hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * kItems;
    for (int e = threadIdx.x; e < kItems; e += kSortWG) {
        const int64_t p = b0 + e;
        if (p < n) atomicAdd(&h[(keys[p] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan, phase 1: block sums
__global__ __launch_bounds__(kScanWG) void k_scan_reduce(const uint32_t* __restrict__ in,
                                                         int64_t n, uint32_t* sums) {
    __shared__ uint32_t s[kScanWG];
    const int64_t b0 = (int64_t)blockIdx.x * kScanItems;
    uint32_t acc = 0;
    for (int e = threadIdx.x; e < kScanItems; e += kScanWG) {
        const int64_t p = b0 + e;
        if (p < n) acc += in[p];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kScanWG / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = s[0];
}

// block-wide exclusive scan of kScanWG values held one per thread
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s,
                                                         uint32_t& total) {
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kScanWG; off <<= 1) {
        const uint32_t t = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    total = s[kScanWG - 1];
    const uint32_t incl = s[threadIdx.x];
    __syncthreads();
    return incl - v;
}

// phase 2: exclusive scan of the block sums in one workgroup (any count)
__global__ __launch_bounds__(kScanWG) void k_scan_sums(uint32_t* sums, int nsums) {
    __shared__ uint32_t s[kScanWG];
    uint32_t carry = 0;
    for (int b = 0; b < nsums; b += kScanWG) {
        const int i = b + (int)threadIdx.x;
        const uint32_t v = i < nsums ? sums[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan(v, s, total);
        if (i < nsums) sums[i] = carry + ex;
        carry += total;
    }
}

// phase 3: scan within each block, offset by its block sum
__global__ __launch_bounds__(kScanWG) void k_scan_down(const uint32_t* __restrict__ in,
                                                       int64_t n,
                                                       const uint32_t* __restrict__ sums,
                                                       uint32_t* out) {
    __shared__ uint32_t s[kScanWG];
    constexpr int kPer = kScanItems / kScanWG;   // contiguous items per thread
    const int64_t b0 = (int64_t)blockIdx.x * kScanItems + (int64_t)threadIdx.x * kPer;
    uint32_t loc[kPer];
    uint32_t acc = 0;
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
        const int64_t p = b0 + e;
        loc[e] = p < n ? in[p] : 0u;
        acc += loc[e];
    }
    uint32_t total;
    uint32_t run = sums[blockIdx.x] + block_exclusive_scan(acc, s, total);
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
        const int64_t p = b0 + e;
        if (p < n) out[p] = run;
        run += loc[e];
    }
}

__global__ __launch_bounds__(kSortWG) void k_radix_scatter(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ idx, int64_t n, int shift,
    int nblocks, const uint32_t* __restrict__ offsets, uint32_t* keys_out, uint32_t* idx_out) {
    __shared__ uint32_t wcount[kSortWG / 64][256];
    __shared__ uint32_t gbase[256];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < 256 * (kSortWG / 64); d += kSortWG)
        (&wcount[0][0])[d] = 0;
    gbase[threadIdx.x] = offsets[(int64_t)threadIdx.x * nblocks + blockIdx.x];
    __syncthreads();

    const int64_t w0 = (int64_t)blockIdx.x * kItems + (int64_t)wave * kItemsPerWave;
    const unsigned long long lt = (1ull << lane) - 1ull;
    constexpr int kGroups = kItemsPerWave / 64;
    uint32_t rank[kGroups];
    uint32_t dig[kGroups];
    // pass A: ranks within this wave's sub-range, in order
#pragma unroll
    for (int gi = 0; gi < kGroups; ++gi) {
        const int64_t p = w0 + gi * 64 + lane;
        const bool valid = p < n;
        const uint32_t d = valid ? (keys[p] >> shift) & 255u : 0u;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const unsigned long long bal = __ballot(valid && ((d >> bit) & 1u));
            peers &= ((d >> bit) & 1u) ? bal : ~bal;
        }
        uint32_t before = 0;
        if (valid) before = wcount[wave][d];
        // wave-synchronous: every lane has read the counter before the leader updates it
        __builtin_amdgcn_wave_barrier();
        if (valid) {
            const int leader = __ffsll((long long)peers) - 1;
            if (lane == leader) wcount[wave][d] = before + (uint32_t)__popcll(peers);
        }
        __builtin_amdgcn_wave_barrier();
        rank[gi] = before + (uint32_t)__popcll(peers & lt);
        dig[gi] = d;
    }
    __syncthreads();
    // exclusive prefix of the per-wave counts, per digit
    {
        const int d = threadIdx.x;
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < kSortWG / 64; ++w) {
            const uint32_t c = wcount[w][d];
            wcount[w][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int gi = 0; gi < kGroups; ++gi) {
        const int64_t p = w0 + gi * 64 + lane;
        if (p < n) {
            const uint32_t d = dig[gi];
            const uint32_t dst = gbase[d] + wcount[wave][d] + rank[gi];
            keys_out[dst] = keys[p];
            idx_out[dst] = idx[p];
        }
    }
}

hipError_t scan_exclusive(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* sums,
                          hipStream_t stream) {
    const int nb = (int)((n + kScanItems - 1) / kScanItems);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanWG), 0, stream, in, n, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanWG), 0, stream, sums, nb);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kScanWG), 0, stream, in, n, sums, out);
    return hipGetLastError();
}

}  // namespace

int64_t sort_hist_elems(int64_t n) {
    const int64_t nblocks = (n + kItems - 1) / kItems;
    return 256 * (nblocks > 0 ? nblocks : 1);
}

int64_t sort_scan_tmp_elems(int64_t n_scan) { return (n_scan + kScanItems - 1) / kScanItems + 1; }

namespace {

// Stable LSD radix sort of (b.keys, b.idx) on the low nbits of the keys;
// the sorted keys end in *kfinal and the permutation in b.idx.
hipError_t radix_sort(int64_t n, int nbits, const SortBuffers& b, hipStream_t stream,
                      uint32_t** kfinal) {
    uint32_t* kin = b.keys;
    uint32_t* iin = b.idx;
    *kfinal = kin;
    if (n == 0) return hipSuccess;
    const int nblocks = (int)((n + kItems - 1) / kItems);
    const int64_t nh = 256ll * nblocks;
    uint32_t* kout = b.keys2;
    uint32_t* iout = b.idx2;
    for (int shift = 0; shift < nbits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3(nblocks), dim3(kSortWG), 0, stream, kin, n, shift,
                           nblocks, b.hist);
        hipError_t e = scan_exclusive(b.hist, b.hist, nh, b.scan_tmp, stream);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(kSortWG), 0, stream, kin, iin, n,
                           shift, nblocks, b.hist, kout, iout);
        uint32_t* t = kin; kin = kout; kout = t;
        t = iin; iin = iout; iout = t;
    }
    // the sorted permutation must end in b.idx
    if (iin != b.idx) {
        hipError_t e = hipMemcpyAsync(b.idx, iin, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice,
                                      stream);
        if (e != hipSuccess) return e;
    }
    *kfinal = kin;
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cell_sort(const double* x, const double* y, int64_t n, double inv_dx,
                            double inv_dy, const TileGeom& g, const SortBuffers& b,
                            hipStream_t stream) {
    const int ntiles = g.ntx * g.nty;
    if (n > 0) {
        const unsigned blocks = (unsigned)((n + kSortWG - 1) / kSortWG);
        hipLaunchKernelGGL(k_tile_keys, dim3(blocks), dim3(kSortWG), 0, stream, x, y, n,
                           inv_dx, inv_dy, g, b.keys, b.idx);
    }
    int nbits = 0;
    while ((1 << nbits) < ntiles) ++nbits;
    uint32_t* kin = b.keys;
    hipError_t e = radix_sort(n, nbits, b, stream, &kin);
    if (e != hipSuccess) return e;
    const unsigned blocks = (unsigned)((n + 1 + kSortWG - 1) / kSortWG);
    hipLaunchKernelGGL(k_tile_bounds, dim3(blocks), dim3(kSortWG), 0, stream, kin, n, ntiles,
                       b.tile_start);
    return hipGetLastError();
}

hipError_t launch_gr_cell_sort(const double* r, const double* th, int64_t n,
                               const gr::GrConst& g, int tile, const SortBuffers& b,
                               hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const int ntx = (g.nr + tile - 1) / tile, nty = (g.nth + tile - 1) / tile;
    const unsigned blocks = (unsigned)((n + kSortWG - 1) / kSortWG);
    hipLaunchKernelGGL(k_gr_tile_keys, dim3(blocks), dim3(kSortWG), 0, stream, r, th, n, g, tile,
                       ntx, b.keys, b.idx);
    int nbits = 0;
    while ((1 << nbits) < ntx * nty) ++nbits;
    uint32_t* kin = b.keys;
    return radix_sort(n, nbits, b, stream, &kin);
}

hipError_t launch_cell_sort3(const double* x, const double* y, const double* z, int64_t n,
                             double inv_dx, double inv_dy, double inv_dz, const TileGeom3& g,
                             const SortBuffers& b, hipStream_t stream) {
    const int ntiles = g.ntx * g.nty * g.ntz;
    if (n > 0) {
        const unsigned blocks = (unsigned)((n + kSortWG - 1) / kSortWG);
        hipLaunchKernelGGL(k_tile_keys3, dim3(blocks), dim3(kSortWG), 0, stream, x, y, z, n,
                           inv_dx, inv_dy, inv_dz, g, b.keys, b.idx);
    }
    int nbits = 0;
    while ((1 << nbits) < ntiles) ++nbits;
    uint32_t* kin = b.keys;
    hipError_t e = radix_sort(n, nbits, b, stream, &kin);
    if (e != hipSuccess) return e;
    const unsigned blocks = (unsigned)((n + 1 + kSortWG - 1) / kSortWG);
    hipLaunchKernelGGL(k_tile_bounds, dim3(blocks), dim3(kSortWG), 0, stream, kin, n, ntiles,
                       b.tile_start);
    return hipGetLastError();
}

}  // namespace gcb
