// Host-side interface between the C ABI (gcb_host.hip) and the kernel
// translation units.  Each launcher enqueues its kernels on `stream` and
// returns the hipError_t of the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gcb_common.hpp"
#include "gcb_gr.hpp"

namespace gcb {

// Geometry of the tiled launch.
struct TileGeom {
    int tile;       // tile edge in cells
    int halo;       // extra nodes on each side of the tile in the LDS window
    int ntx, nty;   // tiles along x and y
    int window;     // tile + 2*halo nodes per side
};

// Which kernel does the work of one step.
enum class PushKind { Global, Tiled };

struct PushLaunch {
    PushKind kind;
    bool yee;              // compile-time Yee offsets
    const void* fields;    // node-interleaved device fields (double or float)
    int64_t n;
    const uint32_t* perm = nullptr;   // read slot perm[p] of the input (sort steps)
    const int32_t* tile_start;   // tiled: ntiles + 1 offsets
    TileGeom geom;
    uint8_t* trace;        // nullable: trace row of this step
    bool replay;           // read the decisions from `trace` instead of writing them
    DevStats* stats;       // nullable
    int steps = 1;         // global kernel: steps per launch (trace: steps*n bytes)
    bool exact = false;    // guiding-center branch in the exact frame (binary64 only)
    bool mirror = false;   // guiding-center branch with the mirror terms
    bool phase = false;    // guiding-center branch with the gyration phase advanced
};

// binary64 form (fields double, u double)
hipError_t launch_push_f64(const PushLaunch& L, const ParticlePtrs<double>& in,
                           const ParticlePtrs<double>& out, const PushConst& pc,
                           hipStream_t stream);

// binary64 form with contracted multiply-adds (GCB_ARITH_FAST)
hipError_t launch_push_f64_fast(const PushLaunch& L, const ParticlePtrs<double>& in,
                                const ParticlePtrs<double>& out, const PushConst& pc,
                                hipStream_t stream);

// mixed form (fields float, u float)
hipError_t launch_push_mixed(const PushLaunch& L, const ParticlePtrs<float>& in,
                             const ParticlePtrs<float>& out, const PushConst& pc,
                             hipStream_t stream);

// LDS bytes the tiled kernel needs for a window of `window` nodes per side
// (window <= kTiledMaxWindow).
size_t tiled_lds_bytes(int window, size_t elem_bytes);
constexpr int kTiledChunk = 512;       // particles a tiled workgroup queues in LDS at once
constexpr int kTiledMaxWindow = 64;    // window edge the tiled kernel stages
constexpr int kTiledMaxSteps = 16;     // steps per tiled launch (not past the next sort)
constexpr int kQueueMax = 2048;   // particles compacted per pass in a 3D tile

// ---------------------------------------------------------------------------
// 3D push

struct TileGeom3 {
    int tile;            // cubic tile edge in cells
    int halo;            // extra nodes on each side of the tile in the LDS window
    int ntx, nty, ntz;   // tiles along x, y, z
    int window;          // tile + 2*halo nodes per side
};

struct Push3Launch {
    PushKind kind;
    bool yee;              // compile-time 3D Yee offsets
    const void* fields;    // node-interleaved device fields (double or float)
    int64_t n;
    const uint32_t* perm = nullptr;   // read slot perm[p] of the input (sort steps)
    const int32_t* tile_start;   // tiled: ntiles + 1 offsets
    TileGeom3 geom;
    uint8_t* trace;        // nullable: trace row of the launch's first step
    bool replay;
    DevStats* stats;       // nullable
    int steps = 1;         // steps per launch (trace: steps*n bytes)
    bool exact = false;    // guiding-center branch in the exact frame (binary64 only)
    bool mirror = false;   // guiding-center branch with the mirror terms
    bool phase = false;    // guiding-center branch with the gyration phase advanced
};

hipError_t launch_push3_f64(const Push3Launch& L, const ParticlePtrs3<double>& in,
                            const ParticlePtrs3<double>& out, const PushConst3& pc,
                            hipStream_t stream);
// the same with contracted multiply-adds (GCB_ARITH_FAST)
hipError_t launch_push3_f64_fast(const Push3Launch& L, const ParticlePtrs3<double>& in,
                                 const ParticlePtrs3<double>& out, const PushConst3& pc,
                                 hipStream_t stream);
hipError_t launch_push3_mixed(const Push3Launch& L, const ParticlePtrs3<float>& in,
                              const ParticlePtrs3<float>& out, const PushConst3& pc,
                              hipStream_t stream);

// LDS bytes of the 3D tiled kernel for a window of `window` nodes per side.
size_t tiled3_lds_bytes(int window, size_t elem_bytes);

// ---------------------------------------------------------------------------
// cell sort

struct SortBuffers {
    uint32_t* keys;      // n
    uint32_t* idx;       // n
    uint32_t* keys2;     // n
    uint32_t* idx2;      // n
    uint32_t* hist;      // 256 * nblocks (+ scan workspace)
    uint32_t* scan_tmp;  // scan block sums
    int32_t* tile_start; // ntiles + 1
};

int64_t sort_hist_elems(int64_t n);   // elements of `hist`
int64_t sort_scan_tmp_elems(int64_t n_scan);

// Compute tile keys from positions, sort (stable), produce tile_start and the
// permutation idx (sorted slot -> source slot).
hipError_t launch_cell_sort(const double* x, const double* y, int64_t n, double inv_dx,
                            double inv_dy, const TileGeom& g, const SortBuffers& b,
                            hipStream_t stream);

// The same for the 3D state: keys are the cubic tiles of (x, y, z), row-major
// (x fastest).
hipError_t launch_cell_sort3(const double* x, const double* y, const double* z, int64_t n,
                             double inv_dx, double inv_dy, double inv_dz, const TileGeom3& g,
                             const SortBuffers& b, hipStream_t stream);

// ---------------------------------------------------------------------------
// fields

hipError_t launch_interleave_fields(const double* const comps[6], int nx, int ny,
                                    void* dst, bool to_float, hipStream_t stream);

// ---------------------------------------------------------------------------
// reductions

hipError_t launch_kinetic_energy(const void* ux, const void* uy, const void* uz,
                                 bool u_float, int64_t n, double c, double* out,
                                 double* lam_x, double* lam_y, double* lam_z,
                                 double* partial, hipStream_t stream);
int64_t kinetic_partial_elems(int64_t n);

hipError_t launch_count_flagged(const uint8_t* status, int64_t n,
                                unsigned long long* out, hipStream_t stream);

// zero `words` 8-byte words at p (8-byte aligned) with a kernel
hipError_t launch_zero_words(void* p, int64_t words, hipStream_t stream);

// the library's binary64 sin and cos of n values (device arrays)
// dst[s] = src[perm[s]] (inverse: dst[perm[s]] = src[s]) for n binary64 values
hipError_t launch_permute_f64(const double* src, const uint32_t* perm, int64_t n, double* dst,
                              bool inverse, hipStream_t stream);

hipError_t launch_sincos(const double* x, double* s, double* c, int64_t n,
                         hipStream_t stream);

// ---------------------------------------------------------------------------
// adjoint

struct AdjointLaunch {
    bool yee;
    const double* fields;   // node-interleaved binary64
    int64_t n;
    const double* state;    // the step's saved start state: 7 arrays of n (x,y,xp,yp,ux,uy,uz)
    const double* qm;       // nullable
    const uint8_t* strace;  // per-particle S of this step (1 = Boris)
    const uint32_t* list;   // this step's guiding-center list (launch_gca_lists)
    const unsigned* count;  // its length
    float* grad_fields;     // node-interleaved float gradient accumulators
    void* records;          // adjoint_record_bytes(n, n_iter, batch) of scratch
    int batch;              // steps whose gather points the records hold
    int batch_slot;         // this step's place in the batch
};

// gather points recorded per particle and guiding-center step
int adjoint_slots(int n_iter);
size_t adjoint_record_bytes(int64_t n, int n_iter, int steps);

// One step of the reverse sweep: lam (7*n, in/out) from the cotangents of
// the step's outputs to those of its inputs; the step's gather points go to
// batch slot L.batch_slot of the records.
hipError_t launch_adjoint_step(const AdjointLaunch& L, double* lam /*7*n in/out*/,
                               const PushConst& pc, hipStream_t stream);

// Guiding-center lists of n_steps steps from their switch traces (trace:
// n_steps*n, 0 = guiding center): for step s, lists[s*n + t] for
// t < counts[s].  counts (n_steps) must be zero on entry.
hipError_t launch_gca_lists(const uint8_t* trace, int64_t n, int n_steps, uint32_t* lists,
                            unsigned* counts, hipStream_t stream);

// Node cotangents of the first nb batch slots into L.grad_fields; strace_first
// is the switch trace of the step in slot 0 (the later slots follow at
// strides of n).
hipError_t launch_adjoint_scatter(const AdjointLaunch& L, const uint8_t* strace_first, int nb,
                                  const PushConst& pc, hipStream_t stream);

hipError_t launch_deinterleave_add(const float* grad_fields, int nx, int ny,
                                   float* const out[6], hipStream_t stream);

// 3D adjoint (gcb_adjoint3.hip): the 2D organisation with 9-array states
// (x, y, z, xp, yp, zp, ux, uy, uz) and 3D gather points.
struct Adjoint3Launch {
    bool yee;               // 3D Yee offsets
    const double* fields;   // node-interleaved binary64 3D fields
    int64_t n;
    const double* state;    // the step's saved start state: 9 arrays of n
    const double* qm;       // nullable
    const uint8_t* strace;  // per-particle S of this step (1 = Boris)
    const uint32_t* list;   // this step's guiding-center list
    const unsigned* count;  // its length
    float* grad_fields;     // node-interleaved float gradient accumulators
    void* records;          // adjoint3_record_bytes(n, n_iter, batch) of scratch
    int batch;
    int batch_slot;
};

size_t adjoint3_record_bytes(int64_t n, int n_iter, int steps);
hipError_t launch_adjoint3_step(const Adjoint3Launch& L, double* lam /*9*n in/out*/,
                                const PushConst3& pc, hipStream_t stream);
hipError_t launch_adjoint3_scatter(const Adjoint3Launch& L, const uint8_t* strace_first, int nb,
                                   const PushConst3& pc, hipStream_t stream);

// curved-spacetime push (gcb_gr.hip)
struct GrPtrs {
    double *r, *th, *ph;
    void *ur, *uth, *uph;   // double (binary64 form) or float (precision form)
    const double* qm;       // nullable
    int32_t* id;            // nullable
    uint8_t* status;
};

// stable sort of the particles by (r, theta) tiles of tile x tile cells;
// the permutation ends in b.idx
hipError_t launch_gr_cell_sort(const double* r, const double* th, int64_t n,
                               const gr::GrConst& g, int tile, const SortBuffers& b,
                               hipStream_t stream);

hipError_t launch_gr_cell_lengths(const gr::GrConst& g, double dr, double dth, double* dl,
                                  hipStream_t stream);
// n_steps steps; the first launch reads slot perm[k] of `in` (k when perm is
// null) and writes slot k of `out`, later ones work in place on `out`;
// trace[step*n + (id ? id : slot)]
hipError_t launch_gr_push_f64(const GrPtrs& in, const GrPtrs& out, const uint32_t* perm,
                              int64_t n, int n_steps, const double* F, const double* dl,
                              const gr::GrConst& g, uint8_t* trace, int trace_step0,
                              DevStats* stats, hipStream_t stream);
hipError_t launch_gr_push_mixed(const GrPtrs& in, const GrPtrs& out, const uint32_t* perm,
                                int64_t n, int n_steps, const float* F, const double* dl,
                                const gr::GrConst& g, uint8_t* trace, int trace_step0,
                                DevStats* stats, hipStream_t stream);
hipError_t launch_gr_push_fast(const GrPtrs& in, const GrPtrs& out, const uint32_t* perm,
                               int64_t n, int n_steps, const double* F, const double* dl,
                               const gr::GrConst& g, uint8_t* trace, int trace_step0,
                               DevStats* stats, hipStream_t stream);

}  // namespace gcb
