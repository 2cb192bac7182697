// Field layout conversion and reductions.
#include <hip/hip_runtime.h>

#include "gcb_internal.h"
#include "gcb_trig.hpp"

namespace gcb {
namespace {

constexpr int kWG = 256;

struct SixPtrs {
    const double* c[6];
};

template <typename T>
__global__ __launch_bounds__(kWG) void k_interleave(SixPtrs src, int64_t nodes, T* dst) {
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i >= nodes) return;
#pragma unroll
    for (int k = 0; k < 6; ++k) dst[i * 6 + k] = (T)src.c[k][i];
}

struct SixOut {
    float* c[6];
};

__global__ __launch_bounds__(kWG) void k_deinterleave_add(const float* __restrict__ g,
                                                          int64_t nodes, SixOut out) {
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i >= nodes) return;
#pragma unroll
    for (int k = 0; k < 6; ++k) out.c[k][i] += g[i * 6 + k];
}

template <typename U>
__device__ __forceinline__ double ld(const void* p, int64_t i) {
    return (double)static_cast<const U*>(p)[i];
}

// mean (Gamma - 1) c^2: per-block partial sums in a fixed order, then one
// block sums the partials (deterministic).  lam = u / (n Gamma) if requested.
template <typename U>
__global__ __launch_bounds__(kWG) void k_ke_partial(const void* ux, const void* uy,
                                                    const void* uz, int64_t n, double c,
                                                    double* lx, double* ly, double* lz,
                                                    double* partial) {
    __shared__ double s[kWG];
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        const double a = ld<U>(ux, i), b = ld<U>(uy, i), d = ld<U>(uz, i);
        const double c2 = c * c;
        const double g = sqrt(1.0 + ((a * a + b * b) + d * d) * (1.0 / c2));
        v = (g - 1.0) * c2;
        if (lx) {
            const double f = 1.0 / ((double)n * g);
            lx[i] = a * f;
            ly[i] = b * f;
            lz[i] = d * f;
        }
    }
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = kWG / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kWG) void k_ke_final(const double* partial, int64_t nparts,
                                                  int64_t n, double* out) {
    __shared__ double s[kWG];
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < nparts; i += kWG) v += partial[i];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = kWG / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = n > 0 ? s[0] / (double)n : 0.0;
}

// out[0] += particles with any status bit other than HALO; out[1 + k] +=
// particles with bit 2^k set, k = 0..6
__global__ __launch_bounds__(kWG) void k_count_flagged(const uint8_t* __restrict__ st,
                                                       int64_t n, unsigned long long* out) {
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    const uint8_t v = i < n ? st[i] : (uint8_t)0;
    const unsigned long long b = __ballot((v & ~(uint8_t)ST_HALO) != 0);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(out, (unsigned long long)__popcll(b));
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const unsigned long long m = __ballot((v >> k) & 1);
        if ((threadIdx.x & 63) == 0 && m) atomicAdd(out + 1 + k, (unsigned long long)__popcll(m));
    }
}

// zero n 8-byte words (a kernel, not a memset node, so that the clear is an
// ordinary kernel of the stream wherever the caller records it)
__global__ __launch_bounds__(kWG) void k_zero_words(unsigned long long* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// the library's sin and cos (the curved-spacetime metric's and the gyro-phase
// option's), binary64, this unit compiled without contraction like those
// instances of the parity arithmetic
__global__ __launch_bounds__(kWG) void k_sincos(const double* __restrict__ x, double* s,
                                                double* c, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i >= n) return;
    double sn, cs;
    sincos_poly<double>(x[i], sn, cs);
    s[i] = sn;
    c[i] = cs;
}

}  // namespace

// dst[s] = src[perm[s]] for n binary64 values (perm: sorted slot -> source slot)
__global__ __launch_bounds__(kWG) void k_gather_f64(const double* __restrict__ src,
                                                    const uint32_t* __restrict__ perm,
                                                    int64_t n, double* __restrict__ dst) {
    const int64_t s = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (s < n) dst[s] = src[perm[s]];
}

// dst[perm[s]] = src[s], the inverse of k_gather_f64
__global__ __launch_bounds__(kWG) void k_scatter_f64(const double* __restrict__ src,
                                                     const uint32_t* __restrict__ perm,
                                                     int64_t n, double* __restrict__ dst) {
    const int64_t s = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (s < n) dst[perm[s]] = src[s];
}

hipError_t launch_permute_f64(const double* src, const uint32_t* perm, int64_t n, double* dst,
                              bool inverse, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + kWG - 1) / kWG);
    if (inverse)
        hipLaunchKernelGGL(k_scatter_f64, dim3(blocks), dim3(kWG), 0, stream, src, perm, n, dst);
    else
        hipLaunchKernelGGL(k_gather_f64, dim3(blocks), dim3(kWG), 0, stream, src, perm, n, dst);
    return hipGetLastError();
}

hipError_t launch_sincos(const double* x, double* s, double* c, int64_t n,
                         hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + kWG - 1) / kWG);
    hipLaunchKernelGGL(k_sincos, dim3(blocks), dim3(kWG), 0, stream, x, s, c, n);
    return hipGetLastError();
}

hipError_t launch_zero_words(void* p, int64_t words, hipStream_t stream) {
    if (words <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((words + kWG - 1) / kWG);
    hipLaunchKernelGGL(k_zero_words, dim3(blocks), dim3(kWG), 0, stream,
                       static_cast<unsigned long long*>(p), words);
    return hipGetLastError();
}

hipError_t launch_interleave_fields(const double* const comps[6], int nx, int ny, void* dst,
                                    bool to_float, hipStream_t stream) {
    SixPtrs s;
    for (int k = 0; k < 6; ++k) s.c[k] = comps[k];
    const int64_t nodes = (int64_t)nx * ny;
    const unsigned blocks = (unsigned)((nodes + kWG - 1) / kWG);
    if (to_float)
        hipLaunchKernelGGL(k_interleave<float>, dim3(blocks), dim3(kWG), 0, stream, s, nodes,
                           static_cast<float*>(dst));
    else
        hipLaunchKernelGGL(k_interleave<double>, dim3(blocks), dim3(kWG), 0, stream, s, nodes,
                           static_cast<double*>(dst));
    return hipGetLastError();
}

hipError_t launch_deinterleave_add(const float* grad_fields, int nx, int ny,
                                   float* const out[6], hipStream_t stream) {
    SixOut o;
    for (int k = 0; k < 6; ++k) o.c[k] = out[k];
    const int64_t nodes = (int64_t)nx * ny;
    const unsigned blocks = (unsigned)((nodes + kWG - 1) / kWG);
    hipLaunchKernelGGL(k_deinterleave_add, dim3(blocks), dim3(kWG), 0, stream, grad_fields,
                       nodes, o);
    return hipGetLastError();
}

int64_t kinetic_partial_elems(int64_t n) { return (n + kWG - 1) / kWG + 1; }

hipError_t launch_kinetic_energy(const void* ux, const void* uy, const void* uz, bool u_float,
                                 int64_t n, double c, double* out, double* lam_x,
                                 double* lam_y, double* lam_z, double* partial,
                                 hipStream_t stream) {
    const int64_t nb = (n + kWG - 1) / kWG;
    if (nb > 0) {
        if (u_float)
            hipLaunchKernelGGL(k_ke_partial<float>, dim3((unsigned)nb), dim3(kWG), 0, stream,
                               ux, uy, uz, n, c, lam_x, lam_y, lam_z, partial);
        else
            hipLaunchKernelGGL(k_ke_partial<double>, dim3((unsigned)nb), dim3(kWG), 0, stream,
                               ux, uy, uz, n, c, lam_x, lam_y, lam_z, partial);
    }
    hipLaunchKernelGGL(k_ke_final, dim3(1), dim3(kWG), 0, stream, partial, nb, n, out);
    return hipGetLastError();
}

hipError_t launch_count_flagged(const uint8_t* status, int64_t n, unsigned long long* out,
                                hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + kWG - 1) / kWG);
    hipLaunchKernelGGL(k_count_flagged, dim3(blocks), dim3(kWG), 0, stream, status, n, out);
    return hipGetLastError();
}

}  // namespace gcb
