// Definitions shared by the device code and the host launchers of libgcb.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Per-particle arithmetic is compiled for the device and, for host-side
// checks of the same code, for the host.
#define GCB_HD __host__ __device__ __forceinline__

namespace gcb {

enum : uint32_t {
    ST_NONFINITE = 1,
    ST_KAPPA = 2,
    ST_QUAD = 4,
    ST_BZERO = 8,
    ST_FPRES = 16,
    ST_HALO = 32,
    ST_MIRROR = 128,
};

// Gyration handling of a guiding-center step (the values of
// gcb_params.gyration): mu conserved, u_perp_g held, mu = 0, mu conserved
// with the gyration phase advanced over the step.
enum : int32_t {
    GYR_MU = 0,
    GYR_UPERP = 1,
    GYR_ZERO = 2,
    GYR_PHASE = 3,
};

// Variants of the guiding-center branch, one kernel instance each: the
// paper's reduced frame, the exact frame of Sec. 2.2 with the zero-curvature
// scheme, the reduced frame with the mirror force and grad-B drift
// (gcb_params.frame and .mirror), the reduced frame with the gyration phase
// advanced (GYR_PHASE), and the exact frame with the curvature scheme.
enum : int {
    kVarReduced = 0,
    kVarExact = 1,
    kVarMirror = 2,
    kVarPhase = 3,
    kVarExactCurv = 4,
};

// the exact frame (either scheme)
constexpr bool var_exact(int v) { return v == kVarExact || v == kVarExactCurv; }

// 1 - v_E^2/c^2 is clamped to this floor where the drift reaches c.
constexpr double kKappaFloor = 1.0e-12;
// |1 - (dt/2) v_E.(b.grad)b| below this: no division in the parallel update.
constexpr double kDFloor = 1.0e-12;

// Lattice coordinates (position / cell size) of magnitude this or more, or
// NaN, have no field: a gather there returns NaN (a runaway iteration).
constexpr double kFarLattice = 1073741824.0;   // 2^30

// 1/sqrt(x) for finite x > 0 in binary64: the hardware estimate refined by
// two Newton-Raphson steps y <- y + y (1 - x y^2)/2 (each roughly doubles
// the number of correct bits; the result is within a few units in the last
// place).
GCB_HD double rsqrt_nr(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rsq(x);
#else
    double y = 1.0 / sqrt(x);
#endif
    double e = fma(-(x * y), y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-(x * y), y, 1.0);
    y = fma(0.5 * y, e, y);
    return y;
}

// 1/x for finite normal x in binary64: the hardware estimate refined by two
// Newton-Raphson steps y <- y + y (1 - x y); within a few units in the last
// place.
GCB_HD double rcp_nr(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rcp(x);
#else
    double y = 1.0 / x;
#endif
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    return y;
}

// 2D Yee lattice offsets (cells) of Ex, Ey, Ez, Bx, By, Bz.
constexpr double kYeeStagger[6][2] = {
    {0.5, 0.0}, {0.0, 0.5}, {0.0, 0.0}, {0.0, 0.5}, {0.5, 0.0}, {0.5, 0.5}};

// Per-launch constants, passed by value as a kernel argument.
struct PushConst {
    double dt, c, c2, inv_c2;
    double f_rho, f_E, inv_dl, fp_tol;
    double inv_dx, inv_dy, Lx, Ly;
    double qm;               // used when the per-particle array is absent
    double inv_Lx, inv_Ly;   // 1/Lx, 1/Ly (the production binary64 form)
    double stagger[6][2];
    int32_t nx, ny;
    int32_t curvature, n_iter;
    int32_t gyration, pad_;  // GYR_*
    double mirror_tol;       // > 0: ST_MIRROR where (v_perp_g/c)^2 exceeds it
};

// Device pointers of a structure-of-arrays particle state.
template <typename U>
struct ParticlePtrs {
    double* x;
    double* y;
    double* xp;
    double* yp;
    U* ux;
    U* uy;
    U* uz;
    double* qm;      // may be null
    int32_t* id;     // may be null
    uint8_t* status;
    // binary64 push, optional: the start state of every step of a launch,
    // recorded for the adjoint (step s at rec + 7*n*s: arrays x, y, xp, yp,
    // ux, uy, uz of n doubles, a particle at its trace column)
    double* rec;
};

// 3D lattice: the constants of a 2D launch (physics, x and y geometry, the
// x and y lattice offsets in b.stagger) plus the z geometry.
struct PushConst3 {
    PushConst b;
    double inv_dz, Lz;
    double inv_Lz;           // 1/Lz (the production binary64 form)
    double sz[6];            // z offsets of the lattices, in cells
    int32_t nz, pad_;
};

// 3D state: the 2D arrays plus z and its previous value.
template <typename U>
struct ParticlePtrs3 {
    ParticlePtrs<U> b;
    double* z;
    double* zp;
};

// Accumulators filled by the push kernels when statistics are requested:
// kStatSlots copies, one cache line each; workgroup b adds to slot
// b % kStatSlots so that the atomics of a launch spread over many L2 lines,
// and the host sums the slots.
constexpr int kStatSlots = 512;
struct alignas(64) DevStats {
    unsigned long long gca_steps;
    unsigned long long boris_steps;
    unsigned long long halo_misses;
    unsigned long long max_res_bits;   // bit pattern of a non-negative double
};

GCB_HD int wrap_index(int i, int n) {
    if ((unsigned)i < (unsigned)n) return i;
    int r = i % n;
    return r < 0 ? r + n : r;
}

}  // namespace gcb
