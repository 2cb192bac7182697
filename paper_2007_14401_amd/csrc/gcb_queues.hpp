// Regime compaction shared by the push kernels: a stable split of a
// workgroup's particles into a guiding-center queue and a full-orbit queue,
// so that each wavefront of the update that follows runs one branch of the
// coupled step (Sec. 3.2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gcb {

// Stable split of the m particles of one pass of a tile into two queues of
// slots in LDS: those for which decide(t) holds (guiding center) from the
// front in order, the others (Boris) from the back.  Every thread of the
// workgroup calls it; returns the length of the guiding-center queue.
template <int kThreads, class Decide>
__device__ __forceinline__ int split_queues(int m, uint16_t* queue, int* wave_g, int* wave_b,
                                            Decide&& decide) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    int nG = 0, nB = 0;
    for (int t0 = 0; t0 < m; t0 += kThreads) {
        const int t = t0 + (int)threadIdx.x;
        const bool valid = t < m;
        const bool gca = valid && decide(t);
        const unsigned long long bg = __ballot(valid && gca);
        const unsigned long long bb = __ballot(valid && !gca);
        if (lane == 0) {
            wave_g[wave] = __popcll(bg);
            wave_b[wave] = __popcll(bb);
        }
        __syncthreads();
        int offg = nG, offb = nB, totg = 0, totb = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            if (w < wave) {
                offg += wave_g[w];
                offb += wave_b[w];
            }
            totg += wave_g[w];
            totb += wave_b[w];
        }
        if (valid) {
            if (gca)
                queue[offg + __popcll(bg & lt)] = (uint16_t)t;
            else
                queue[m - 1 - (offb + __popcll(bb & lt))] = (uint16_t)t;
        }
        nG += totg;
        nB += totb;
        __syncthreads();
    }
    return nG;
}

}  // namespace gcb
