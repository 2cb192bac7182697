// C ABI of libgcb (declared in include/gcb.h): argument validation, device
// memory owned by the context, the step loop and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gcb.h"
#include "gcb_internal.h"

using namespace gcb;

namespace {

struct DevBuf {
    void* ptr = nullptr;
    size_t cap = 0;
};

struct TimedLaunch {
    int cls;
    hipEvent_t start, stop;
};

}  // namespace

// The fixed scratch of gcb_push_noalloc: one copy per device, which the
// device holds until the process ends.  Host code never uses the array's
// name as an address: gcb_create looks up the device's copy once per device
// with hipGetSymbolAddress and every use goes through that pointer.
constexpr size_t kNoAllocScratchBytes = (size_t)GCB_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// address of `scratch` on `device` (the current device), looked up once
hipError_t noalloc_scratch(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace

struct gcb_ctx {
    int device = 0;
    std::string err;
    // fields
    bool have_fields = false;
    int nx = 0, ny = 0;
    double dx = 1.0, dy = 1.0;
    double stagger[6][2] = {};
    int dtype = GCB_F64;
    bool yee = false;
    DevBuf fields;
    // curved-spacetime fields
    bool have_gr = false;
    int gr_dtype = GCB_F64;
    gr::GrConst gr{};
    double gr_dr = 0.0, gr_dth = 0.0;
    DevBuf gr_fields, gr_dl, gr_pscratch;
    // 3D fields
    bool have_f3 = false;
    int n3[3] = {};
    double d3[3] = {1.0, 1.0, 1.0};
    double stagger3[6][3] = {};
    int dtype3 = GCB_F64;
    bool yee3 = false;
    DevBuf fields3;
    // scratch
    DevBuf sort_keys, sort_idx, sort_keys2, sort_idx2, sort_hist, sort_scan, tile_start;
    DevBuf pscratch;     // sorted copy of the particle state
    DevBuf stats;        // DevStats + flagged counter
    DevBuf ke_partial;
    DevBuf adj_states, adj_lam, adj_grad, adj_trace, adj_work, adj_samples, adj_lists;
    DevBuf adj_order;    // tile order of a backward segment: q/m and the permutation
    // fixed scratch of gcb_push_noalloc on this context's device (the address
    // of the file-scope array `scratch` there); while `arena` is set, every
    // piece of call scratch is carved from it instead of allocated
    char* noalloc_base = nullptr;
    char* arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    // timing
    bool timing = false;
    std::vector<TimedLaunch> launches;
    double ms[GCB_NTIMERS] = {};
    int64_t count[GCB_NTIMERS] = {};
};

namespace {

thread_local std::string g_thread_err;

int fail(gcb_ctx* ctx, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g_thread_err = buf;
    return code;
}

#define GCB_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(ctx, GCB_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

int ensure(gcb_ctx* ctx, DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (b.cap >= bytes) return GCB_OK;
    if (b.ptr) {
        hipError_t e = hipFree(b.ptr);
        b.ptr = nullptr;
        b.cap = 0;
        if (e != hipSuccess) return fail(ctx, GCB_EHIP, "hipFree: %s", hipGetErrorString(e));
    }
    hipError_t e = hipMalloc(&b.ptr, bytes);
    if (e != hipSuccess) {
        b.ptr = nullptr;
        (void)hipGetLastError();
        return fail(ctx, GCB_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes,
                    hipGetErrorString(e));
    }
    b.cap = bytes;
    return GCB_OK;
}

// Scratch of a call: from the context buffer `b` (grown with hipMalloc), or,
// inside gcb_push_noalloc, carved from the fixed array (256-byte aligned),
// failing with GCB_EINVAL when it is exhausted.
int take(gcb_ctx* ctx, DevBuf& b, size_t bytes, void** out) {
    if (ctx->arena) {
        const size_t off = (ctx->arena_used + 255) & ~(size_t)255;
        if (off > ctx->arena_cap || bytes > ctx->arena_cap - off)
            return fail(ctx, GCB_EINVAL,
                        "gcb_push_noalloc: the call needs more than the %zu bytes of its fixed "
                        "scratch (fewer particles, or gcb_push)", ctx->arena_cap);
        *out = ctx->arena + off;
        ctx->arena_used = off + bytes;
        return GCB_OK;
    }
    const int rc = ensure(ctx, b, bytes);
    if (rc) return rc;
    *out = b.ptr;
    return GCB_OK;
}

void release(DevBuf& b) {
    if (b.ptr) (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.cap = 0;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// record a timing event pair around a launch sequence
struct Timer {
    gcb_ctx* ctx;
    hipStream_t s;
    int cls;
    hipEvent_t a = nullptr, b = nullptr;
    Timer(gcb_ctx* c, hipStream_t st, int k) : ctx(c), s(st), cls(k) {
        if (!ctx->timing) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            ctx->timing = false;
            return;
        }
        (void)hipEventRecord(a, s);
    }
    void done() {
        if (!a) return;
        (void)hipEventRecord(b, s);
        ctx->launches.push_back({cls, a, b});
        a = b = nullptr;
    }
};

const double kYee[6][2] = {{0.5, 0.0}, {0.0, 0.5}, {0.0, 0.0},
                           {0.0, 0.5}, {0.5, 0.0}, {0.5, 0.5}};
const double kYee3[6][3] = {{0.5, 0.0, 0.0}, {0.0, 0.5, 0.0}, {0.0, 0.0, 0.5},
                            {0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}, {0.5, 0.5, 0.0}};

int validate_params(gcb_ctx* ctx, const gcb_params* prm) {
    if (!prm) return fail(ctx, GCB_EINVAL, "params is NULL");
    if (!finite_pos(prm->dt)) return fail(ctx, GCB_EINVAL, "dt must be finite and > 0");
    if (!finite_pos(prm->c)) return fail(ctx, GCB_EINVAL, "c must be finite and > 0");
    if (!(prm->f_rho >= 0.0) || !(prm->f_E >= 0.0))
        return fail(ctx, GCB_EINVAL, "f_rho and f_E must be >= 0");
    if (!(prm->fp_tol >= 0.0)) return fail(ctx, GCB_EINVAL, "fp_tol must be >= 0");
    if (prm->curvature != 0 && prm->curvature != 1)
        return fail(ctx, GCB_EINVAL, "curvature must be 0 or 1");
    if (prm->n_iter < 1 || prm->n_iter > 64)
        return fail(ctx, GCB_EINVAL, "n_iter must be in [1, 64]");
    if (prm->form != GCB_FORM_F64 && prm->form != GCB_FORM_MIXED)
        return fail(ctx, GCB_EINVAL, "unknown form %d", prm->form);
    if (prm->sort_every < 0) return fail(ctx, GCB_EINVAL, "sort_every must be >= 0");
    if (prm->kernel < GCB_KERNEL_AUTO || prm->kernel > GCB_KERNEL_TILED)
        return fail(ctx, GCB_EINVAL, "unknown kernel %d", prm->kernel);
    if (prm->tile < 0 || prm->tile == 1 || prm->tile > 256)
        return fail(ctx, GCB_EINVAL, "tile must be 0 or in [2, 256]");
    if (prm->replay != 0 && prm->replay != 1)
        return fail(ctx, GCB_EINVAL, "replay must be 0 or 1");
    if (prm->frame != GCB_FRAME_REDUCED && prm->frame != GCB_FRAME_EXACT)
        return fail(ctx, GCB_EINVAL, "unknown frame %d", prm->frame);
    if (prm->gyration < GCB_GYRATION_MU || prm->gyration > GCB_GYRATION_PHASE)
        return fail(ctx, GCB_EINVAL, "unknown gyration %d", prm->gyration);
    if (prm->gyration == GCB_GYRATION_PHASE && (prm->frame != GCB_FRAME_REDUCED || prm->mirror))
        return fail(ctx, GCB_EUNSUPPORTED,
                    "GCB_GYRATION_PHASE goes with the reduced frame and without the mirror terms");
    if (prm->mirror != 0 && prm->mirror != 1)
        return fail(ctx, GCB_EINVAL, "mirror must be 0 or 1");
    if (prm->mirror && prm->curvature != 1)
        return fail(ctx, GCB_EUNSUPPORTED, "the mirror terms need curvature = 1");
    if (prm->mirror && prm->frame != GCB_FRAME_REDUCED)
        return fail(ctx, GCB_EUNSUPPORTED, "the mirror terms go with the reduced frame");
    if (!(std::isfinite(prm->mirror_tol) && prm->mirror_tol >= 0.0))
        return fail(ctx, GCB_EINVAL, "mirror_tol must be finite and >= 0");
    if (prm->arith != GCB_ARITH_EXACT && prm->arith != GCB_ARITH_FAST)
        return fail(ctx, GCB_EINVAL, "unknown arith %d", prm->arith);
    if (prm->keep_order != 0 && prm->keep_order != 1)
        return fail(ctx, GCB_EINVAL, "keep_order must be 0 or 1");
    return GCB_OK;
}

// the production binary64 arithmetic is served by the binary64 pushes
// (2D, 3D, curved spacetime) only
int reject_fast_arith(gcb_ctx* ctx, const gcb_params* prm) {
    if (prm->arith != GCB_ARITH_EXACT)
        return fail(ctx, GCB_EUNSUPPORTED,
                    "GCB_ARITH_FAST is served by gcb_push, gcb_push_3d and gcb_push_gr with "
                    "GCB_FORM_F64 only");
    return GCB_OK;
}

// the exact frame (binary64), the gyration options other
// than a conserved mu and the mirror terms are served by gcb_push and
// gcb_push_3d only, the check of the mirror terms (check_ok) by the pushes,
// the production arithmetic (fast_ok) as reject_fast_arith says
int reject_push_options(gcb_ctx* ctx, const gcb_params* prm, bool check_ok = false,
                        bool fast_ok = false) {
    if (!fast_ok && reject_fast_arith(ctx, prm)) return GCB_EUNSUPPORTED;
    if (prm->frame != GCB_FRAME_REDUCED)
        return fail(ctx, GCB_EUNSUPPORTED,
                    "the exact frame is served by gcb_push and gcb_push_3d only");
    if (prm->gyration != GCB_GYRATION_MU)
        return fail(ctx, GCB_EUNSUPPORTED,
                    "gyration options other than GCB_GYRATION_MU are served by gcb_push and "
                    "gcb_push_3d only");
    if (prm->mirror != 0)
        return fail(ctx, GCB_EUNSUPPORTED,
                    "the mirror terms are served by gcb_push and gcb_push_3d only");
    if (!check_ok && prm->mirror_tol != 0.0)
        return fail(ctx, GCB_EUNSUPPORTED,
                    "the check of the mirror terms is served by the pushes only");
    return GCB_OK;
}

int validate_particles(gcb_ctx* ctx, const gcb_particles* p, const gcb_params* prm) {
    if (!p) return fail(ctx, GCB_EINVAL, "particles is NULL");
    if (p->n < 0) return fail(ctx, GCB_EINVAL, "n must be >= 0");
    if (p->n >= (int64_t)1 << 31) return fail(ctx, GCB_EINVAL, "n must be < 2^31");
    if (p->n == 0) return GCB_OK;
    if (!p->x || !p->y || !p->xp || !p->yp || !p->ux || !p->uy || !p->uz || !p->status)
        return fail(ctx, GCB_EINVAL, "particle arrays x, y, xp, yp, ux, uy, uz, status "
                                     "must be non-NULL");
    const uintptr_t m8 = (uintptr_t)p->x | (uintptr_t)p->y | (uintptr_t)p->xp |
                         (uintptr_t)p->yp | (uintptr_t)p->qm;
    if (m8 & 7) return fail(ctx, GCB_EINVAL, "double arrays must be 8-byte aligned");
    const size_t ua = prm->form == GCB_FORM_F64 ? 8 : 4;
    if (((uintptr_t)p->ux | (uintptr_t)p->uy | (uintptr_t)p->uz) & (ua - 1))
        return fail(ctx, GCB_EINVAL, "u arrays misaligned for their element type");
    if ((uintptr_t)p->id & 3) return fail(ctx, GCB_EINVAL, "id array misaligned");
    if (!p->qm && !(std::isfinite(prm->qm) && prm->qm != 0.0))
        return fail(ctx, GCB_EINVAL, "params.qm must be finite and non-zero when "
                                     "particles.qm is NULL");
    return GCB_OK;
}

template <typename U>
ParticlePtrs<U> ptrs_of(const gcb_particles* p) {
    ParticlePtrs<U> r{};
    r.x = p->x;
    r.y = p->y;
    r.xp = p->xp;
    r.yp = p->yp;
    r.ux = static_cast<U*>(p->ux);
    r.uy = static_cast<U*>(p->uy);
    r.uz = static_cast<U*>(p->uz);
    r.qm = p->qm;
    r.id = p->id;
    r.status = p->status;
    return r;
}

// carve a scratch copy of the state (same shape as `like`) out of one
// buffer, plus n_extra more double arrays of n
template <typename U>
int scratch_state(gcb_ctx* ctx, const ParticlePtrs<U>& like, int64_t n, ParticlePtrs<U>& out,
                  int n_extra = 0, double** extra = nullptr) {
    const size_t nd = (size_t)n * sizeof(double), nu = (size_t)n * sizeof(U);
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t bytes = (4 + n_extra) * up(nd) + 3 * up(nu) + up(n) + (like.qm ? up(nd) : 0) +
                   (like.id ? up((size_t)n * 4) : 0);
    void* base;
    int rc = take(ctx, ctx->pscratch, bytes, &base);
    if (rc) return rc;
    char* b = static_cast<char*>(base);
    auto take = [&](size_t s) {
        char* r = b;
        b += up(s);
        return r;
    };
    out.x = reinterpret_cast<double*>(take(nd));
    out.y = reinterpret_cast<double*>(take(nd));
    out.xp = reinterpret_cast<double*>(take(nd));
    out.yp = reinterpret_cast<double*>(take(nd));
    out.ux = reinterpret_cast<U*>(take(nu));
    out.uy = reinterpret_cast<U*>(take(nu));
    out.uz = reinterpret_cast<U*>(take(nu));
    out.status = reinterpret_cast<uint8_t*>(take(n));
    out.qm = like.qm ? reinterpret_cast<double*>(take(nd)) : nullptr;
    out.id = like.id ? reinterpret_cast<int32_t*>(take((size_t)n * 4)) : nullptr;
    for (int e = 0; e < n_extra; ++e) extra[e] = reinterpret_cast<double*>(take(nd));
    return GCB_OK;
}

// copy every array of a state (same shape) from a to b
template <typename U>
hipError_t copy_state(const ParticlePtrs<U>& a, const ParticlePtrs<U>& b, int64_t n,
                      hipStream_t stream) {
    const size_t nd = (size_t)n * sizeof(double), nu = (size_t)n * sizeof(U);
    const hipMemcpyKind k = hipMemcpyDeviceToDevice;
    hipError_t e = hipSuccess;
    auto cp = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess && src) e = hipMemcpyAsync(dst, src, bytes, k, stream);
    };
    cp(b.x, a.x, nd);
    cp(b.y, a.y, nd);
    cp(b.xp, a.xp, nd);
    cp(b.yp, a.yp, nd);
    cp(b.ux, a.ux, nu);
    cp(b.uy, a.uy, nu);
    cp(b.uz, a.uz, nu);
    cp(b.status, a.status, (size_t)n);
    cp(b.qm, a.qm, nd);
    cp(b.id, a.id, (size_t)n * sizeof(int32_t));
    return e;
}

// the physics constants of a launch (geometry left to the caller)
PushConst physics_const(const gcb_params* prm) {
    PushConst pc{};
    pc.dt = prm->dt;
    pc.c = prm->c;
    pc.c2 = prm->c * prm->c;
    pc.inv_c2 = 1.0 / (prm->c * prm->c);
    pc.f_rho = prm->f_rho;
    pc.f_E = prm->f_E;
    pc.fp_tol = prm->fp_tol;
    pc.qm = prm->qm;
    pc.curvature = prm->curvature;
    pc.n_iter = prm->n_iter;
    pc.gyration = prm->gyration;
    pc.mirror_tol = prm->mirror_tol;
    return pc;
}

PushConst make_const(const gcb_ctx* ctx, const gcb_params* prm) {
    PushConst pc = physics_const(prm);
    pc.inv_dl = 1.0 / std::sqrt(ctx->dx * ctx->dy);
    pc.inv_dx = 1.0 / ctx->dx;
    pc.inv_dy = 1.0 / ctx->dy;
    pc.Lx = ctx->nx * ctx->dx;
    pc.Ly = ctx->ny * ctx->dy;
    pc.inv_Lx = 1.0 / pc.Lx;
    pc.inv_Ly = 1.0 / pc.Ly;
    std::memcpy(pc.stagger, ctx->stagger, sizeof(pc.stagger));
    pc.nx = ctx->nx;
    pc.ny = ctx->ny;
    return pc;
}

// 3D: the effective cell size of the switch is (dx dy dz)^(1/3) (Sec. 3)
PushConst3 make_const3(const gcb_ctx* ctx, const gcb_params* prm) {
    PushConst3 pc{};
    pc.b = physics_const(prm);
    pc.b.inv_dl = 1.0 / std::cbrt((ctx->d3[0] * ctx->d3[1]) * ctx->d3[2]);
    pc.b.inv_dx = 1.0 / ctx->d3[0];
    pc.b.inv_dy = 1.0 / ctx->d3[1];
    pc.inv_dz = 1.0 / ctx->d3[2];
    pc.b.Lx = ctx->n3[0] * ctx->d3[0];
    pc.b.Ly = ctx->n3[1] * ctx->d3[1];
    pc.Lz = ctx->n3[2] * ctx->d3[2];
    pc.b.inv_Lx = 1.0 / pc.b.Lx;
    pc.b.inv_Ly = 1.0 / pc.b.Ly;
    pc.inv_Lz = 1.0 / pc.Lz;
    for (int k = 0; k < 6; ++k) {
        pc.b.stagger[k][0] = ctx->stagger3[k][0];
        pc.b.stagger[k][1] = ctx->stagger3[k][1];
        pc.sz[k] = ctx->stagger3[k][2];
    }
    pc.b.nx = ctx->n3[0];
    pc.b.ny = ctx->n3[1];
    pc.nz = ctx->n3[2];
    return pc;
}

// Steps whose gather-point records one adjoint scatter takes: more steps
// merge more of a particle's points per atomic (2D: 13.2 ms per step backward
// at 1e7 particles with 8, 12.5 ms with 32), within a budget of record bytes
// (at most half the device memory free when the backward starts).  The 3D
// scatter's windows move more often over long batches (24.9 ms per step with
// 6 steps, 26.6 with 27), so 3D keeps short ones.
constexpr int kAdjMaxBatch = 32;
constexpr size_t kAdjRecordBudget = 128ull << 30;
// Tile edge (cells) of the order a 2D backward segment runs its particles in.
#ifndef GCB_ADJ_ORDER_TILE
#define GCB_ADJ_ORDER_TILE 32
#endif
constexpr int kAdjOrderTile = GCB_ADJ_ORDER_TILE;
// The same for the 3D backward (cubic tiles).
#ifndef GCB_ADJ3_ORDER_TILE
#define GCB_ADJ3_ORDER_TILE 8
#endif
constexpr int kAdj3OrderTile = GCB_ADJ3_ORDER_TILE;
constexpr int kAdj3MaxBatch = 8;
constexpr size_t kAdj3RecordBudget = 32ull << 30;

// the record budget of a backward call: the fixed one, capped by half the
// free device memory
size_t record_budget(size_t fixed) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return fixed;
    return std::min(fixed, free_b / 2);
}

// Halo of the LDS window in nodes: the drift bound c dt per step over the
// steps between sorts, plus one node for the stencil.  Formed in binary64;
// 0 when it exceeds kMaxHalo (no window that large fits in LDS, and the int
// arithmetic of the window origin stays far from overflow).  A window of 0
// marks the tiled kernel as unavailable.
constexpr double kMaxHalo = 256.0;
int window_halo(const gcb_params* prm, double inv_min_cell) {
    const int se = prm->sort_every > 0 ? prm->sort_every : 1;
    const double h = std::ceil(((double)se * prm->c) * prm->dt * inv_min_cell) + 1.0;
    return (h <= kMaxHalo) ? (int)h : 0;
}

TileGeom3 make_geom3(const gcb_ctx* ctx, const gcb_params* prm) {
    TileGeom3 g;
    g.tile = prm->tile ? prm->tile : 6;
    const double inv_min =
        std::max(1.0 / ctx->d3[0], std::max(1.0 / ctx->d3[1], 1.0 / ctx->d3[2]));
    g.halo = window_halo(prm, inv_min);
    g.ntx = (ctx->n3[0] + g.tile - 1) / g.tile;
    g.nty = (ctx->n3[1] + g.tile - 1) / g.tile;
    g.ntz = (ctx->n3[2] + g.tile - 1) / g.tile;
    g.window = g.halo > 0 ? g.tile + 2 * g.halo : 0;
    return g;
}

TileGeom make_geom(const gcb_ctx* ctx, const gcb_params* prm) {
    TileGeom g;
    g.tile = prm->tile ? prm->tile : 24;
    const double inv_min = std::max(1.0 / ctx->dx, 1.0 / ctx->dy);
    g.halo = window_halo(prm, inv_min);
    g.ntx = (ctx->nx + g.tile - 1) / g.tile;
    g.nty = (ctx->ny + g.tile - 1) / g.tile;
    g.window = g.halo > 0 ? g.tile + 2 * g.halo : 0;
    return g;
}

constexpr size_t kMaxLds = 160 * 1024;

int prepare_sort(gcb_ctx* ctx, int64_t n, int ntiles, SortBuffers& sb) {
    int rc;
    void *k, *i, *k2, *i2, *h, *sc, *ts;
    if ((rc = take(ctx, ctx->sort_keys, (size_t)n * 4, &k))) return rc;
    if ((rc = take(ctx, ctx->sort_idx, (size_t)n * 4, &i))) return rc;
    if ((rc = take(ctx, ctx->sort_keys2, (size_t)n * 4, &k2))) return rc;
    if ((rc = take(ctx, ctx->sort_idx2, (size_t)n * 4, &i2))) return rc;
    const int64_t nh = sort_hist_elems(n);
    if ((rc = take(ctx, ctx->sort_hist, (size_t)nh * 4, &h))) return rc;
    const int64_t ns = std::max(sort_scan_tmp_elems(nh), sort_scan_tmp_elems(ntiles + 1));
    if ((rc = take(ctx, ctx->sort_scan, (size_t)ns * 4, &sc))) return rc;
    if ((rc = take(ctx, ctx->tile_start, (size_t)(ntiles + 1) * 4, &ts))) return rc;
    sb.keys = static_cast<uint32_t*>(k);
    sb.idx = static_cast<uint32_t*>(i);
    sb.keys2 = static_cast<uint32_t*>(k2);
    sb.idx2 = static_cast<uint32_t*>(i2);
    sb.hist = static_cast<uint32_t*>(h);
    sb.scan_tmp = static_cast<uint32_t*>(sc);
    sb.tile_start = static_cast<int32_t*>(ts);
    return GCB_OK;
}

// the slots, then the flagged count and eight status-bit counts
constexpr size_t kStatBytes = kStatSlots * sizeof(DevStats) + 9 * sizeof(unsigned long long);

// the device accumulators of a push that reports statistics (not cleared)
int stats_take(gcb_ctx* ctx, const gcb_stats* stats, DevStats** dstats) {
    *dstats = nullptr;
    if (!stats) return GCB_OK;
    void* p;
    const int rc = take(ctx, ctx->stats, kStatBytes, &p);
    if (rc) return rc;
    *dstats = static_cast<DevStats*>(p);
    return GCB_OK;
}

// clear them (a kernel on the stream)
int stats_zero(gcb_ctx* ctx, DevStats* dstats, hipStream_t stream) {
    if (dstats) GCB_HIP(launch_zero_words(dstats, (int64_t)(kStatBytes / 8), stream));
    return GCB_OK;
}

int stats_begin(gcb_ctx* ctx, const gcb_stats* stats, hipStream_t stream, DevStats** dstats) {
    const int rc = stats_take(ctx, stats, dstats);
    return rc ? rc : stats_zero(ctx, *dstats, stream);
}

// count the flagged particles, copy the accumulators back and sum the slots
int stats_end(gcb_ctx* ctx, DevStats* dstats, const uint8_t* status, int64_t n,
              gcb_stats* stats, hipStream_t stream) {
    if (!stats) return GCB_OK;
    // the flagged count and the eight status-bit counts go to the nine words
    // after the slots
    unsigned long long* flagged = reinterpret_cast<unsigned long long*>(dstats + kStatSlots);
    GCB_HIP(launch_count_flagged(status, n, flagged, stream));
    DevStats host[kStatSlots + 2];   // 33 kB on the host stack: no allocation
    GCB_HIP(hipMemcpyAsync(host, dstats, kStatBytes, hipMemcpyDeviceToHost, stream));
    GCB_HIP(hipStreamSynchronize(stream));
    unsigned long long g = 0, b = 0, h = 0, mbits = 0;
    for (int s = 0; s < kStatSlots; ++s) {
        g += host[s].gca_steps;
        b += host[s].boris_steps;
        h += host[s].halo_misses;
        // non-negative doubles order like their bit patterns
        mbits = host[s].max_res_bits > mbits ? host[s].max_res_bits : mbits;
    }
    stats->gca_steps = (int64_t)g;
    stats->boris_steps = (int64_t)b;
    stats->halo_misses = (int64_t)h;
    double m;
    std::memcpy(&m, &mbits, sizeof(m));
    stats->max_fp_residual = m;
    unsigned long long extra[9];
    std::memcpy(extra, &host[kStatSlots], sizeof(extra));
    stats->flagged = (int64_t)extra[0];
    for (int k = 0; k < 8; ++k) stats->status_counts[k] = (int64_t)extra[1 + k];
    return GCB_OK;
}

// Copy six field components of rows*row_len nodes each (host or device
// arrays of doubles) into `dst`, node-interleaved, as float if requested.
int upload_interleaved(gcb_ctx* ctx, const double* const comps[6], int row_len, int rows,
                       DevBuf& dst, bool to_float, int32_t src, hipStream_t stream) {
    const int64_t nodes = (int64_t)row_len * rows;
    int rc = ensure(ctx, dst, (size_t)nodes * 6 * (to_float ? sizeof(float) : sizeof(double)));
    if (rc) return rc;
    if (src == GCB_DEVICE) {
        GCB_HIP(launch_interleave_fields(comps, row_len, rows, dst.ptr, to_float, stream));
        return GCB_OK;
    }
    DevBuf tmp;
    rc = ensure(ctx, tmp, (size_t)nodes * 6 * sizeof(double));
    if (rc) return rc;
    const double* dcomps[6];
    hipError_t e = hipSuccess;
    for (int k = 0; k < 6 && e == hipSuccess; ++k) {
        double* d = static_cast<double*>(tmp.ptr) + k * nodes;
        e = hipMemcpyAsync(d, comps[k], nodes * sizeof(double), hipMemcpyHostToDevice, stream);
        dcomps[k] = d;
    }
    if (e == hipSuccess)
        e = launch_interleave_fields(dcomps, row_len, rows, dst.ptr, to_float, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    release(tmp);
    if (e != hipSuccess) return fail(ctx, GCB_EHIP, "field conversion: %s", hipGetErrorString(e));
    return GCB_OK;
}

// kind of kernel for a request (tiled needs sorting and a window that fits)
int choose_kind(gcb_ctx* ctx, const gcb_params* prm, bool tiled_ok, int window,
                PushKind* kind) {
    if (prm->kernel == GCB_KERNEL_TILED) {
        if (!tiled_ok)
            return fail(ctx, GCB_EUNSUPPORTED,
                        "tiled kernel needs sort_every > 0 and a tile window that fits in "
                        "LDS (window %d nodes)", window);
        *kind = PushKind::Tiled;
    } else if (prm->kernel == GCB_KERNEL_GLOBAL) {
        *kind = PushKind::Global;
    } else {
        *kind = tiled_ok ? PushKind::Tiled : PushKind::Global;
    }
    return GCB_OK;
}

// record (binary64, keep_order or no sorting): the start state of every
// step, 7 arrays of n doubles per step (the adjoint's recomputation)
template <typename U>
int run_push(gcb_ctx* ctx, gcb_particles* p, const gcb_params* prm, int32_t n_steps,
             uint8_t* s_trace, DevStats* dstats, hipStream_t stream,
             double* record = nullptr) {
    const int64_t n = p->n;
    const PushConst pc = make_const(ctx, prm);
    const TileGeom g = make_geom(ctx, prm);
    const size_t esz = prm->form == GCB_FORM_F64 ? sizeof(double) : sizeof(float);
    const bool tiled_ok = prm->sort_every > 0 && g.window > 0 && g.window <= kTiledMaxWindow &&
                          tiled_lds_bytes(g.window, esz) <= kMaxLds;
    PushKind kind;
    int rc;
    if ((rc = choose_kind(ctx, prm, tiled_ok, g.window, &kind))) return rc;
    ParticlePtrs<U> user = ptrs_of<U>(p);
    ParticlePtrs<U> scr{};
    SortBuffers sb{};
    // keep_order: the tiled kernel works through the tiles of each sort in
    // place (the arrays keep their order); the global kernel needs no sort
    const bool keep = prm->keep_order != 0;
    const bool sorting = prm->sort_every > 0 && n > 0 && !(keep && kind == PushKind::Global);
    if (sorting) {
        if ((rc = prepare_sort(ctx, n, g.ntx * g.nty, sb))) return rc;
        if (!keep && (rc = scratch_state<U>(ctx, user, n, scr))) return rc;
    }
    // all scratch is in place: the first device work of the call
    if ((rc = stats_zero(ctx, dstats, stream))) return rc;
    // On a sort step the push reads the state through the sort's permutation
    // and writes it in tile order into the other of two buffers (the caller's
    // arrays and a library copy); the other steps work in place.  A state
    // that ends in the library copy is copied back.  The global kernel keeps a
    // particle in registers, the tiled kernel a tile's particles in LDS, for
    // up to 16 steps per launch (not past the next sort).
    constexpr int32_t kGlobalStepsPerLaunch = 16;
    ParticlePtrs<U> cur = user, other = scr;
    for (int32_t step = 0; step < n_steps;) {
        int32_t ns = std::min(kind == PushKind::Global ? kGlobalStepsPerLaunch : kTiledMaxSteps,
                              n_steps - step);
        if (sorting) ns = std::min(ns, prm->sort_every - step % prm->sort_every);
        ParticlePtrs<U> dst = cur;
        const uint32_t* perm = nullptr;
        if (sorting && step % prm->sort_every == 0) {
            Timer t(ctx, stream, GCB_TIMER_SORT);
            GCB_HIP(launch_cell_sort(cur.x, cur.y, n, pc.inv_dx, pc.inv_dy, g, sb, stream));
            t.done();
            perm = sb.idx;
            if (!keep) dst = other;
        }
        // in place, the sort's permutation serves every launch until the next
        if (sorting && keep) perm = sb.idx;
        cur.rec = record ? record + (size_t)step * 7 * n : nullptr;
        dst.rec = cur.rec;
        PushLaunch L;
        L.perm = perm;
        L.kind = kind;
        L.yee = ctx->yee;
        L.fields = ctx->fields.ptr;
        L.n = n;
        L.tile_start = sb.tile_start;
        L.geom = g;
        L.trace = s_trace ? s_trace + (int64_t)step * n : nullptr;
        L.replay = prm->replay != 0;
        L.stats = dstats;
        L.steps = ns;
        L.exact = prm->frame == GCB_FRAME_EXACT;
        L.mirror = prm->mirror != 0;
        L.phase = prm->gyration == GCB_GYRATION_PHASE;
        Timer t(ctx, stream, GCB_TIMER_PUSH);
        hipError_t e;
        if constexpr (sizeof(U) == sizeof(double))
            e = prm->arith == GCB_ARITH_FAST ? launch_push_f64_fast(L, cur, dst, pc, stream)
                                             : launch_push_f64(L, cur, dst, pc, stream);
        else
            e = launch_push_mixed(L, cur, dst, pc, stream);
        if (e != hipSuccess)
            return fail(ctx, GCB_EHIP, "push kernel launch failed: %s", hipGetErrorString(e));
        t.done();
        if (perm && !keep) std::swap(cur, other);
        step += ns;
    }
    if (cur.x != user.x) {
        Timer t(ctx, stream, GCB_TIMER_OTHER);
        GCB_HIP(copy_state<U>(cur, user, n, stream));
        t.done();
    }
    return GCB_OK;
}

template <typename U>
ParticlePtrs3<U> ptrs3_of(const gcb_particles3* p) {
    ParticlePtrs3<U> r{};
    r.b.x = p->x;
    r.b.y = p->y;
    r.b.xp = p->xp;
    r.b.yp = p->yp;
    r.b.ux = static_cast<U*>(p->ux);
    r.b.uy = static_cast<U*>(p->uy);
    r.b.uz = static_cast<U*>(p->uz);
    r.b.qm = p->qm;
    r.b.id = p->id;
    r.b.status = p->status;
    r.z = p->z;
    r.zp = p->zp;
    return r;
}

// record (binary64, keep_order, tiled kernel): the start state of every
// step, 9 arrays of n doubles per step (the adjoint's recomputation)
template <typename U>
int run_push3(gcb_ctx* ctx, gcb_particles3* p, const gcb_params* prm, int32_t n_steps,
              uint8_t* s_trace, DevStats* dstats, hipStream_t stream,
              double* record = nullptr) {
    const int64_t n = p->n;
    const PushConst3 pc = make_const3(ctx, prm);
    const TileGeom3 g = make_geom3(ctx, prm);
    const size_t esz = prm->form == GCB_FORM_F64 ? sizeof(double) : sizeof(float);
    const bool tiled_ok =
        prm->sort_every > 0 && g.window > 0 && tiled3_lds_bytes(g.window, esz) <= kMaxLds;
    PushKind kind;
    int rc;
    if ((rc = choose_kind(ctx, prm, tiled_ok, g.window, &kind))) return rc;
    if (record && kind != PushKind::Tiled)
        return fail(ctx, GCB_EUNSUPPORTED, "start-state records need the tiled kernel");
    ParticlePtrs3<U> user = ptrs3_of<U>(p);
    ParticlePtrs3<U> scr{};
    SortBuffers sb{};
    // keep_order: the tiled kernel works through the tiles of each sort in
    // place (the arrays keep their order); the global kernel needs no sort
    const bool keep = prm->keep_order != 0;
    const bool sorting = prm->sort_every > 0 && n > 0 && !(keep && kind == PushKind::Global);
    if (sorting) {
        if ((rc = prepare_sort(ctx, n, g.ntx * g.nty * g.ntz, sb))) return rc;
        if (!keep) {
            double* zz[2];
            if ((rc = scratch_state<U>(ctx, user.b, n, scr.b, 2, zz))) return rc;
            scr.z = zz[0];
            scr.zp = zz[1];
        }
    }
    // sort steps move the state into the other buffer, as in 2D
    constexpr int32_t kGlobalStepsPerLaunch = 16;
    ParticlePtrs3<U> cur = user, other = scr;
    for (int32_t step = 0; step < n_steps;) {
        int32_t ns = std::min(kind == PushKind::Global ? kGlobalStepsPerLaunch : kTiledMaxSteps,
                              n_steps - step);
        if (sorting) ns = std::min(ns, prm->sort_every - step % prm->sort_every);
        ParticlePtrs3<U> dst = cur;
        const uint32_t* perm = nullptr;
        if (sorting && step % prm->sort_every == 0) {
            Timer t(ctx, stream, GCB_TIMER_SORT);
            GCB_HIP(launch_cell_sort3(cur.b.x, cur.b.y, cur.z, n, pc.b.inv_dx, pc.b.inv_dy,
                                      pc.inv_dz, g, sb, stream));
            t.done();
            perm = sb.idx;
            if (!keep) dst = other;
        }
        // in place, the sort's permutation serves every launch until the next
        if (sorting && keep) perm = sb.idx;
        cur.b.rec = record ? record + (size_t)step * 9 * n : nullptr;
        dst.b.rec = cur.b.rec;
        Push3Launch L;
        L.perm = perm;
        L.kind = kind;
        L.yee = ctx->yee3;
        L.fields = ctx->fields3.ptr;
        L.n = n;
        L.tile_start = sb.tile_start;
        L.geom = g;
        L.trace = s_trace ? s_trace + (int64_t)step * n : nullptr;
        L.replay = prm->replay != 0;
        L.stats = dstats;
        L.steps = ns;
        L.exact = prm->frame == GCB_FRAME_EXACT;
        L.mirror = prm->mirror != 0;
        L.phase = prm->gyration == GCB_GYRATION_PHASE;
        Timer t(ctx, stream, GCB_TIMER_PUSH);
        hipError_t e;
        if constexpr (sizeof(U) == sizeof(double))
            e = prm->arith == GCB_ARITH_FAST ? launch_push3_f64_fast(L, cur, dst, pc, stream)
                                             : launch_push3_f64(L, cur, dst, pc, stream);
        else
            e = launch_push3_mixed(L, cur, dst, pc, stream);
        if (e != hipSuccess)
            return fail(ctx, GCB_EHIP, "push kernel launch failed: %s", hipGetErrorString(e));
        t.done();
        if (perm && !keep) std::swap(cur, other);
        step += ns;
    }
    if (cur.b.x != user.b.x) {
        Timer t(ctx, stream, GCB_TIMER_OTHER);
        hipError_t e = copy_state<U>(cur.b, user.b, n, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(user.z, cur.z, (size_t)n * sizeof(double),
                               hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(user.zp, cur.zp, (size_t)n * sizeof(double),
                               hipMemcpyDeviceToDevice, stream);
        if (e != hipSuccess) return fail(ctx, GCB_EHIP, "state copy: %s", hipGetErrorString(e));
        t.done();
    }
    return GCB_OK;
}

}  // namespace

extern "C" {

int gcb_create(gcb_ctx** out, int device) {
    if (!out) return fail(nullptr, GCB_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return fail(nullptr, GCB_EHIP, "no HIP device available (%s)",
                    e == hipSuccess ? "count 0" : hipGetErrorString(e));
    }
    if (device < 0 || device >= ndev)
        return fail(nullptr, GCB_EINVAL, "device %d out of range [0, %d)", device, ndev);
    e = hipSetDevice(device);
    if (e != hipSuccess)
        return fail(nullptr, GCB_EHIP, "hipSetDevice(%d): %s", device, hipGetErrorString(e));
    void* base = nullptr;
    e = noalloc_scratch(device, &base);
    if (e != hipSuccess)
        return fail(nullptr, GCB_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                    hipGetErrorString(e));
    gcb_ctx* c = new (std::nothrow) gcb_ctx();
    if (!c) return fail(nullptr, GCB_ENOMEM, "out of host memory");
    c->device = device;
    c->noalloc_base = static_cast<char*>(base);
    *out = c;
    return GCB_OK;
}

void gcb_destroy(gcb_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    for (auto& l : ctx->launches) {
        (void)hipEventDestroy(l.start);
        (void)hipEventDestroy(l.stop);
    }
    DevBuf* bufs[] = {&ctx->fields,     &ctx->sort_keys,  &ctx->sort_idx,  &ctx->sort_keys2,
                      &ctx->sort_idx2,  &ctx->sort_hist,  &ctx->sort_scan,
                      &ctx->tile_start, &ctx->pscratch,   &ctx->stats,     &ctx->ke_partial,
                      &ctx->adj_states, &ctx->adj_lam,    &ctx->adj_grad,  &ctx->adj_trace,
                      &ctx->adj_work,   &ctx->adj_samples, &ctx->adj_lists, &ctx->adj_order,
                      &ctx->gr_fields,
                      &ctx->gr_dl,
                      &ctx->gr_pscratch, &ctx->fields3};
    for (DevBuf* b : bufs) release(*b);
    delete ctx;
}

const char* gcb_last_error(const gcb_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_thread_err.c_str();
}

int gcb_load_fields(gcb_ctx* ctx, const gcb_grid_desc* d, const double* const E[3],
                    const double* const B[3], int32_t src, void* stream_) {
    if (!ctx) return fail(nullptr, GCB_EINVAL, "ctx is NULL");
    if (!d || !E || !B) return fail(ctx, GCB_EINVAL, "desc, E and B must be non-NULL");
    if (d->nx < 2 || d->ny < 2) return fail(ctx, GCB_EINVAL, "nx and ny must be >= 2");
    if ((int64_t)d->nx * d->ny * 6 >= ((int64_t)1 << 34))
        return fail(ctx, GCB_EINVAL, "grid too large");
    if (!finite_pos(d->dx) || !finite_pos(d->dy))
        return fail(ctx, GCB_EINVAL, "dx and dy must be finite and > 0");
    for (int k = 0; k < 6; ++k)
        for (int a = 0; a < 2; ++a)
            if (!(d->stagger[k][a] >= 0.0 && d->stagger[k][a] < 1.0))
                return fail(ctx, GCB_EINVAL, "stagger offsets must be in [0, 1)");
    if (d->dtype != GCB_F64 && d->dtype != GCB_F32)
        return fail(ctx, GCB_EINVAL, "unknown dtype %d", d->dtype);
    if (src != GCB_HOST && src != GCB_DEVICE)
        return fail(ctx, GCB_EINVAL, "src must be GCB_HOST or GCB_DEVICE");
    const double* comps[6] = {E[0], E[1], E[2], B[0], B[1], B[2]};
    for (int k = 0; k < 6; ++k)
        if (!comps[k]) return fail(ctx, GCB_EINVAL, "field component %d is NULL", k);
    GCB_HIP(hipSetDevice(ctx->device));
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    ctx->have_fields = false;
    int rc = upload_interleaved(ctx, comps, d->nx, d->ny, ctx->fields, d->dtype == GCB_F32, src,
                                stream);
    if (rc) return rc;
    ctx->nx = d->nx;
    ctx->ny = d->ny;
    ctx->dx = d->dx;
    ctx->dy = d->dy;
    std::memcpy(ctx->stagger, d->stagger, sizeof(ctx->stagger));
    ctx->dtype = d->dtype;
    ctx->yee = std::memcmp(d->stagger, kYee, sizeof(kYee)) == 0;
    ctx->have_fields = true;
    return GCB_OK;
}

int gcb_push(gcb_ctx* ctx, gcb_particles* p, const gcb_params* prm, int32_t n_steps,
             uint8_t* s_trace, gcb_stats* stats, void* stream_) {
    if (!ctx) return fail(nullptr, GCB_EINVAL, "ctx is NULL");
    int rc;
    if ((rc = validate_params(ctx, prm))) return rc;
    if ((rc = validate_particles(ctx, p, prm))) return rc;
    if (n_steps < 0) return fail(ctx, GCB_EINVAL, "n_steps must be >= 0");
    if (prm->frame == GCB_FRAME_EXACT && prm->form != GCB_FORM_F64)
        return fail(ctx, GCB_EUNSUPPORTED, "the exact frame needs GCB_FORM_F64");
    if (prm->arith == GCB_ARITH_FAST && prm->form != GCB_FORM_F64)
        return fail(ctx, GCB_EUNSUPPORTED, "GCB_ARITH_FAST needs GCB_FORM_F64");
    if (!ctx->have_fields) return fail(ctx, GCB_ENOFIELDS, "gcb_load_fields was not called");
    if (prm->form == GCB_FORM_F64 && ctx->dtype != GCB_F64)
        return fail(ctx, GCB_EINVAL, "GCB_FORM_F64 needs fields loaded as GCB_F64");
    if (prm->form == GCB_FORM_MIXED && ctx->dtype != GCB_F32)
        return fail(ctx, GCB_EINVAL, "GCB_FORM_MIXED needs fields loaded as GCB_F32");
    if (s_trace && p->n > 0 && !p->id && prm->sort_every > 0 && !prm->keep_order)
        return fail(ctx, GCB_EINVAL, "a switch trace with sorting needs particle ids");
    if (prm->replay && !s_trace && p->n > 0 && n_steps > 0)
        return fail(ctx, GCB_EINVAL, "replay needs the switch trace s_trace");
    GCB_HIP(hipSetDevice(ctx->device));
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    DevStats* dstats;
    if ((rc = stats_take(ctx, stats, &dstats))) return rc;
    if (prm->form == GCB_FORM_F64)
        rc = run_push<double>(ctx, p, prm, n_steps, s_trace, dstats, stream);
    else
        rc = run_push<float>(ctx, p, prm, n_steps, s_trace, dstats, stream);
    if (rc) return rc;
    return stats_end(ctx, dstats, p->status, p->n, stats, stream);
}

int gcb_push_noalloc(gcb_ctx* ctx, gcb_particles* p, const gcb_params* prm, int32_t n_steps,
                     uint8_t* s_trace, gcb_stats* stats, void* stream) {
    if (!ctx) return fail(nullptr, GCB_EINVAL, "ctx is NULL");
    if (!ctx->noalloc_base)
        return fail(ctx, GCB_EHIP, "the fixed scratch of device %d is not available",
                    ctx->device);
    // every piece of scratch below is carved from the device's fixed array;
    // timing records (a growing host list) are not kept for this call
    const bool timing = ctx->timing;
    ctx->timing = false;
    ctx->arena = ctx->noalloc_base;
    ctx->arena_cap = kNoAllocScratchBytes;
    ctx->arena_used = 0;
    const int rc = gcb_push(ctx, p, prm, n_steps, s_trace, stats, stream);
    ctx->arena = nullptr;
    ctx->arena_cap = ctx->arena_used = 0;
    ctx->timing = timing;
    return rc;
}

int gcb_push_backward(gcb_ctx* ctx, const gcb_particles* start, const gcb_params* prm,
                      int32_t n_steps, const double* const lam_end[7],
                      double* const lam_start[7], float* const dE[3], float* const dB[3],
                      void* stream_) {
    if (!ctx) return fail(nullptr, GCB_EINVAL, "ctx is NULL");
    int rc;
    if ((rc = validate_params(ctx, prm))) return rc;
    if ((rc = validate_particles(ctx, start, prm))) return rc;
    if (n_steps < 0) return fail(ctx, GCB_EINVAL, "n_steps must be >= 0");
    if (!lam_end || !lam_start || !dE || !dB)
        return fail(ctx, GCB_EINVAL, "lam_end, lam_start, dE and dB must be non-NULL");
    const int64_t n = start->n;
    for (int c = 0; c < 7; ++c)
        if (n > 0 && (!lam_end[c] || !lam_start[c]))
            return fail(ctx, GCB_EINVAL, "adjoint array %d is NULL", c);
    for (int c = 0; c < 3; ++c)
        if (!dE[c] || !dB[c]) return fail(ctx, GCB_EINVAL, "dE/dB component %d is NULL", c);
    if (!ctx->have_fields) return fail(ctx, GCB_ENOFIELDS, "gcb_load_fields was not called");
    if (prm->form != GCB_FORM_F64 || ctx->dtype != GCB_F64)
        return fail(ctx, GCB_EUNSUPPORTED, "the adjoint needs GCB_FORM_F64 and binary64 fields");
    if (prm->n_iter > 8)
        return fail(ctx, GCB_EUNSUPPORTED, "the adjoint supports n_iter <= 8");
    if ((rc = reject_push_options(ctx, prm))) return rc;
    GCB_HIP(hipSetDevice(ctx->device));
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const size_t nd = (size_t)n * sizeof(double);
    const size_t nodes = (size_t)ctx->nx * ctx->ny;
    if ((rc = ensure(ctx, ctx->adj_states, (size_t)n_steps * 7 * nd))) return rc;
    if ((rc = ensure(ctx, ctx->adj_trace, (size_t)n_steps * n))) return rc;
    // guiding-center lists of every step (uint32 per particle and step) and
    // their lengths
    if ((rc = ensure(ctx, ctx->adj_lists, (size_t)n_steps * (n + 1) * sizeof(uint32_t))))
        return rc;
    if ((rc = ensure(ctx, ctx->adj_lam, 7 * nd))) return rc;
    if ((rc = ensure(ctx, ctx->adj_work, 7 * nd + (size_t)n))) return rc;
    if ((rc = ensure(ctx, ctx->adj_grad, nodes * 6 * sizeof(float)))) return rc;
    // gather-point records of up to kMaxBatch steps, within the record budget
    constexpr int kMaxBatch = kAdjMaxBatch;
    const size_t budget = record_budget(kAdjRecordBudget);
    const size_t per_step = adjoint_record_bytes(n, prm->n_iter, 1);
    int batch = per_step > 0 ? (int)std::min<size_t>(kMaxBatch, budget / per_step) : 1;
    batch = std::max(1, std::min(batch, std::max(1, (int)n_steps)));
    if ((rc = ensure(ctx, ctx->adj_samples, adjoint_record_bytes(n, prm->n_iter, batch))))
        return rc;
    // The segment runs on its particles in the tile order of their start
    // positions (kAdjOrderTile-cell tiles): the state, q/m and the adjoint
    // are permuted on the way in and the adjoint back on the way out.  Each
    // particle's arithmetic is its own, so the order changes no value; the
    // reverse kernels' gathers of neighbouring lanes then share cache lines.
    TileGeom og{};
    og.tile = kAdjOrderTile;
    og.ntx = (ctx->nx + og.tile - 1) / og.tile;
    og.nty = (ctx->ny + og.tile - 1) / og.tile;
    const bool ordered = n > 0 && n_steps > 0;
    double* qms = nullptr;          // q/m in tile order
    uint32_t* perm = nullptr;       // tile slot -> caller's slot
    if (ordered) {
        if ((rc = ensure(ctx, ctx->adj_order, nd + (size_t)n * 4))) return rc;
        qms = static_cast<double*>(ctx->adj_order.ptr);
        perm = reinterpret_cast<uint32_t*>(qms + n);
    }
    double* work = static_cast<double*>(ctx->adj_work.ptr);
    uint8_t* wstatus = reinterpret_cast<uint8_t*>(work + 7 * (size_t)n);
    double* states = static_cast<double*>(ctx->adj_states.ptr);
    uint8_t* trace = static_cast<uint8_t*>(ctx->adj_trace.ptr);
    double* lam = static_cast<double*>(ctx->adj_lam.ptr);
    float* grad = static_cast<float*>(ctx->adj_grad.ptr);
    const double* src[7] = {start->x, start->y, start->xp, start->yp,
                            static_cast<const double*>(start->ux),
                            static_cast<const double*>(start->uy),
                            static_cast<const double*>(start->uz)};
    Timer t(ctx, stream, GCB_TIMER_BACKWARD);
    if (ordered) {
        SortBuffers ssb{};
        if ((rc = prepare_sort(ctx, n, og.ntx * og.nty, ssb))) return rc;
        GCB_HIP(launch_cell_sort(start->x, start->y, n, 1.0 / ctx->dx, 1.0 / ctx->dy, og, ssb,
                                 stream));
        // the sort's buffers serve the recomputation's sorts too: keep the
        // permutation
        GCB_HIP(hipMemcpyAsync(perm, ssb.idx, (size_t)n * 4, hipMemcpyDeviceToDevice, stream));
        if (start->qm) GCB_HIP(launch_permute_f64(start->qm, perm, n, qms, false, stream));
    }
    if (n > 0) {
        for (int c = 0; c < 7; ++c) {
            if (perm)
                GCB_HIP(launch_permute_f64(src[c], perm, n, work + c * (size_t)n, false, stream));
            else
                GCB_HIP(hipMemcpyAsync(work + c * (size_t)n, src[c], nd,
                                       hipMemcpyDeviceToDevice, stream));
        }
        GCB_HIP(hipMemsetAsync(wstatus, 0, (size_t)n, stream));
    }
    double* wqm = (perm && start->qm) ? qms : start->qm;
    ParticlePtrs<double> w{};
    w.x = work;
    w.y = work + n;
    w.xp = work + 2 * n;
    w.yp = work + 3 * n;
    w.ux = work + 4 * n;
    w.uy = work + 5 * n;
    w.uz = work + 6 * n;
    w.qm = wqm;
    w.id = nullptr;
    w.status = wstatus;
    const PushConst pc = make_const(ctx, prm);
    // forward recomputation, keeping each step's start state and decisions:
    // the push of the segment in place (keep_order; with sort_every > 0 the
    // tiled kernel), which records the start state of every step inside its
    // launches.  The parity arithmetic makes it the forward pass bit for bit,
    // whichever kernel ran that.
    if (n > 0 && n_steps > 0) {
        gcb_params rp = *prm;
        rp.keep_order = 1;
        rp.replay = 0;
        gcb_particles wp{n, w.x, w.y, w.xp, w.yp, w.ux, w.uy, w.uz, wqm, nullptr, wstatus};
        const bool timing = ctx->timing;   // timed as part of the backward pass
        ctx->timing = false;
        rc = run_push<double>(ctx, &wp, &rp, n_steps, trace, nullptr, stream, states);
        ctx->timing = timing;
        if (rc) return rc;
    }
    // per-step guiding-center lists, so that their reverse kernel runs full
    // wavefronts
    uint32_t* lists = static_cast<uint32_t*>(ctx->adj_lists.ptr);
    unsigned* counts = reinterpret_cast<unsigned*>(lists + (size_t)n_steps * n);
    if (n > 0 && n_steps > 0) {
        GCB_HIP(hipMemsetAsync(counts, 0, (size_t)n_steps * sizeof(unsigned), stream));
        GCB_HIP(launch_gca_lists(trace, n, n_steps, lists, counts, stream));
    }
    // reverse sweep
    for (int c = 0; c < 7 && n > 0; ++c) {
        if (perm)
            GCB_HIP(launch_permute_f64(lam_end[c], perm, n, lam + c * (size_t)n, false, stream));
        else
            GCB_HIP(hipMemcpyAsync(lam + c * (size_t)n, lam_end[c], nd, hipMemcpyDeviceToDevice,
                                   stream));
    }
    GCB_HIP(hipMemsetAsync(grad, 0, nodes * 6 * sizeof(float), stream));
    // steps in reverse order, in batches [s_lo, s_hi) of at most `batch` steps:
    // the vector-Jacobian products of the batch's steps, then one scatter
    for (int32_t s_hi = n_steps; s_hi > 0 && n > 0; s_hi -= batch) {
        const int32_t s_lo = std::max<int32_t>(0, s_hi - batch);
        AdjointLaunch A;
        A.yee = ctx->yee;
        A.fields = static_cast<const double*>(ctx->fields.ptr);
        A.n = n;
        A.qm = wqm;
        A.grad_fields = grad;
        A.records = ctx->adj_samples.ptr;
        A.batch = batch;
        for (int32_t s = s_hi - 1; s >= s_lo; --s) {
            A.state = states + (size_t)s * 7 * n;
            A.strace = trace + (size_t)s * n;
            A.list = lists + (size_t)s * n;
            A.count = counts + s;
            A.batch_slot = s - s_lo;
            GCB_HIP(launch_adjoint_step(A, lam, pc, stream));
        }
        GCB_HIP(launch_adjoint_scatter(A, trace + (size_t)s_lo * n, s_hi - s_lo, pc, stream));
    }
    for (int c = 0; c < 7 && n > 0; ++c) {
        if (perm)
            GCB_HIP(launch_permute_f64(lam + c * (size_t)n, perm, n, lam_start[c], true,
                                       stream));
        else
            GCB_HIP(hipMemcpyAsync(lam_start[c], lam + c * (size_t)n, nd,
                                   hipMemcpyDeviceToDevice, stream));
    }
    if (n_steps == 0 && n > 0)
        for (int c = 0; c < 7; ++c)
            GCB_HIP(hipMemcpyAsync(lam_start[c], lam_end[c], nd, hipMemcpyDeviceToDevice,
                                   stream));
    float* const outs[6] = {dE[0], dE[1], dE[2], dB[0], dB[1], dB[2]};
    GCB_HIP(launch_deinterleave_add(grad, ctx->nx, ctx->ny, outs, stream));
    t.done();
    return GCB_OK;
}

int gcb_load_fields_gr(gcb_ctx* ctx, const gcb_gr_desc* d, const double* const D[3],
                       const double* const B[3], int32_t src, void* stream_) {
    if (!ctx) return fail(nullptr, GCB_EINVAL, "ctx is NULL");
    if (!d || !D || !B) return fail(ctx, GCB_EINVAL, "desc, D and B must be non-NULL");
    if (d->nr < 1 || d->nth < 1) return fail(ctx, GCB_EINVAL, "nr and nth must be >= 1");
    if ((int64_t)(d->nr + 1) * (d->nth + 1) * 6 >= ((int64_t)1 << 34))
        return fail(ctx, GCB_EINVAL, "grid too large");
    if (!(std::isfinite(d->r_min) && std::isfinite(d->r_max) && d->r_min > 0.0 &&
          d->r_max > d->r_min))
        return fail(ctx, GCB_EINVAL, "need 0 < r_min < r_max (finite)");
    if (!(std::fabs(d->spin) < 1.0)) return fail(ctx, GCB_EINVAL, "need |spin| < 1");
    if (d->dtype != GCB_F64 && d->dtype != GCB_F32)
        return fail(ctx, GCB_EINVAL, "unknown dtype %d", d->dtype);
    if (src != GCB_HOST && src != GCB_DEVICE)
        return fail(ctx, GCB_EINVAL, "src must be GCB_HOST or GCB_DEVICE");
    const double* comps[6] = {D[0], D[1], D[2], B[0], B[1], B[2]};
    for (int k = 0; k < 6; ++k)
        if (!comps[k]) return fail(ctx, GCB_EINVAL, "field component %d is NULL", k);
    GCB_HIP(hipSetDevice(ctx->device));
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const int nxn = d->nr + 1, nyn = d->nth + 1;
    ctx->have_gr = false;
    int rc = upload_interleaved(ctx, comps, nxn, nyn, ctx->gr_fields, d->dtype == GCB_F32, src,
                                stream);
    if (rc) return rc;
    if ((rc = ensure(ctx, ctx->gr_dl, (size_t)d->nr * d->nth * sizeof(double)))) return rc;
    gr::GrConst g{};
    g.a = d->spin;
    g.r_min = d->r_min;
    g.r_max = d->r_max;
    g.nr = d->nr;
    g.nth = d->nth;
    const double dr = (d->r_max - d->r_min) / d->nr;
    const double dth = gr::kPi / d->nth;
    g.inv_dr = 1.0 / dr;
    g.inv_dth = 1.0 / dth;
    GCB_HIP(launch_gr_cell_lengths(g, dr, dth, static_cast<double*>(ctx->gr_dl.ptr), stream));
    ctx->gr = g;
    ctx->gr_dtype = d->dtype;
    ctx->gr_dr = dr;
    ctx->gr_dth = dth;
    ctx->have_gr = true;
    return GCB_OK;
}

int gcb_push_gr(gcb_ctx* ctx, gcb_gr_particles* p, const gcb_params* prm, int32_t n_steps,
                uint8_t* s_trace, gcb_stats* stats, void* stream_) {
    if (!ctx) return fail(nullptr, GCB_EINVAL, "ctx is NULL");
    if (!prm) return fail(ctx, GCB_EINVAL, "params is NULL");
    if (!p) return fail(ctx, GCB_EINVAL, "particles is NULL");
    if (!finite_pos(prm->dt)) return fail(ctx, GCB_EINVAL, "dt must be finite and > 0");
    if (!(prm->f_rho >= 0.0) || !(prm->f_E >= 0.0))
        return fail(ctx, GCB_EINVAL, "f_rho and f_E must be >= 0");
    if (!(prm->fp_tol >= 0.0)) return fail(ctx, GCB_EINVAL, "fp_tol must be >= 0");
    if (prm->n_iter < 1 || prm->n_iter > 64)
        return fail(ctx, GCB_EINVAL, "n_iter must be in [1, 64]");
    if (prm->form != GCB_FORM_F64 && prm->form != GCB_FORM_MIXED)
        return fail(ctx, GCB_EINVAL, "unknown form %d", prm->form);
    if (prm->replay) return fail(ctx, GCB_EUNSUPPORTED, "replay is not supported here");
    if (!(std::isfinite(prm->mirror_tol) && prm->mirror_tol >= 0.0))
        return fail(ctx, GCB_EINVAL, "mirror_tol must be finite and >= 0");
    if (prm->arith != GCB_ARITH_EXACT && prm->arith != GCB_ARITH_FAST)
        return fail(ctx, GCB_EINVAL, "unknown arith %d", prm->arith);
    if (prm->arith == GCB_ARITH_FAST && prm->form != GCB_FORM_F64)
        return fail(ctx, GCB_EUNSUPPORTED, "GCB_ARITH_FAST needs GCB_FORM_F64");
    {
        const int rc = reject_push_options(ctx, prm, true, true);
        if (rc) return rc;
    }
    if (prm->keep_order != 0)
        return fail(ctx, GCB_EUNSUPPORTED,
                    "keep_order is served by gcb_push and gcb_push_3d only");
    if (p->n < 0) return fail(ctx, GCB_EINVAL, "n must be >= 0");
    if (n_steps < 0) return fail(ctx, GCB_EINVAL, "n_steps must be >= 0");
    if (p->n > 0 && (!p->r || !p->th || !p->ph || !p->ur || !p->uth || !p->uph || !p->status))
        return fail(ctx, GCB_EINVAL, "particle arrays must be non-NULL");
    if (p->n > 0 && !p->qm && !(std::isfinite(prm->qm) && prm->qm != 0.0))
        return fail(ctx, GCB_EINVAL, "params.qm must be finite and non-zero");
    if (prm->sort_every < 0) return fail(ctx, GCB_EINVAL, "sort_every must be >= 0");
    if (s_trace && p->n > 0 && !p->id && prm->sort_every > 0)
        return fail(ctx, GCB_EINVAL, "a switch trace with sorting needs particle ids");
    if (p->n > ((int64_t)1 << 31) - 1) return fail(ctx, GCB_EINVAL, "n too large");
    if (!ctx->have_gr) return fail(ctx, GCB_ENOFIELDS, "gcb_load_fields_gr was not called");
    if (prm->form == GCB_FORM_F64 && ctx->gr_dtype != GCB_F64)
        return fail(ctx, GCB_EINVAL, "GCB_FORM_F64 needs fields loaded as GCB_F64");
    if (prm->form == GCB_FORM_MIXED && ctx->gr_dtype != GCB_F32)
        return fail(ctx, GCB_EINVAL, "GCB_FORM_MIXED needs fields loaded as GCB_F32");
    GCB_HIP(hipSetDevice(ctx->device));
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    DevStats* dstats;
    {
        const int rc = stats_begin(ctx, stats, stream, &dstats);
        if (rc) return rc;
    }
    gr::GrConst g = ctx->gr;
    g.dt = prm->dt;
    g.qm = prm->qm;
    g.f_rho = prm->f_rho;
    g.f_E = prm->f_E;
    g.fp_tol = prm->fp_tol;
    g.mirror_tol = prm->mirror_tol;
    g.n_iter = prm->n_iter;
    GrPtrs ptrs{p->r, p->th, p->ph, p->ur, p->uth, p->uph, p->qm, p->id, p->status};
    const double* dl = static_cast<const double*>(ctx->gr_dl.ptr);
    auto push = [&](const GrPtrs& in, const GrPtrs& out, const uint32_t* perm, int ns,
                    int step0) {
        if (prm->form == GCB_FORM_F64 && prm->arith == GCB_ARITH_FAST)
            return launch_gr_push_fast(in, out, perm, p->n, ns,
                                       static_cast<const double*>(ctx->gr_fields.ptr), dl, g,
                                       s_trace, step0, dstats, stream);
        if (prm->form == GCB_FORM_F64)
            return launch_gr_push_f64(in, out, perm, p->n, ns,
                                      static_cast<const double*>(ctx->gr_fields.ptr), dl, g,
                                      s_trace, step0, dstats, stream);
        return launch_gr_push_mixed(in, out, perm, p->n, ns,
                                    static_cast<const float*>(ctx->gr_fields.ptr), dl, g, s_trace,
                                    step0, dstats, stream);
    };
    if (prm->sort_every > 0 && p->n > 0 && n_steps > 0) {
        // every sort_every steps: sort by (r, theta) tiles of kGrTile^2 cells;
        // the push reads through the permutation and writes in tile order
        // into the other of two buffers (the caller's arrays and a library
        // copy, `id` and `qm` carried along); a state that ends in the copy
        // is copied back
        constexpr int kGrTile = 16;
        const int64_t n = p->n;
        const size_t ub = prm->form == GCB_FORM_F64 ? sizeof(double) : sizeof(float);
        SortBuffers sb;
        int rc;
        if ((rc = prepare_sort(ctx, n, 1, sb))) return rc;
        const size_t bytes = (size_t)n * (3 * sizeof(double) + 3 * ub + sizeof(double) +
                                          sizeof(int32_t) + 1);
        if ((rc = ensure(ctx, ctx->gr_pscratch, bytes))) return rc;
        char* base = static_cast<char*>(ctx->gr_pscratch.ptr);
        GrPtrs sc;
        sc.r = reinterpret_cast<double*>(base);
        sc.th = sc.r + n;
        sc.ph = sc.th + n;
        sc.qm = p->qm ? sc.ph + n : nullptr;
        char* c = reinterpret_cast<char*>(sc.ph + 2 * n);
        sc.ur = c;
        sc.uth = c + n * ub;
        sc.uph = c + 2 * n * ub;
        sc.id = p->id ? reinterpret_cast<int32_t*>(c + 3 * n * ub) : nullptr;
        sc.status = reinterpret_cast<uint8_t*>(c + 3 * n * ub + n * sizeof(int32_t));
        GrPtrs cur = ptrs, other = sc;
        for (int32_t s0 = 0; s0 < n_steps; s0 += prm->sort_every) {
            const int ns = std::min<int32_t>(prm->sort_every, n_steps - s0);
            {
                Timer t(ctx, stream, GCB_TIMER_SORT);
                GCB_HIP(launch_gr_cell_sort(cur.r, cur.th, n, g, kGrTile, sb, stream));
                t.done();
            }
            Timer t(ctx, stream, GCB_TIMER_PUSH);
            GCB_HIP(push(cur, other, sb.idx, ns, s0));
            t.done();
            std::swap(cur, other);
        }
        if (cur.r != ptrs.r) {
            Timer t(ctx, stream, GCB_TIMER_OTHER);
            const hipMemcpyKind k = hipMemcpyDeviceToDevice;
            const size_t nd = (size_t)n * sizeof(double);
            GCB_HIP(hipMemcpyAsync(ptrs.r, cur.r, nd, k, stream));
            GCB_HIP(hipMemcpyAsync(ptrs.th, cur.th, nd, k, stream));
            GCB_HIP(hipMemcpyAsync(ptrs.ph, cur.ph, nd, k, stream));
            GCB_HIP(hipMemcpyAsync(ptrs.ur, cur.ur, n * ub, k, stream));
            GCB_HIP(hipMemcpyAsync(ptrs.uth, cur.uth, n * ub, k, stream));
            GCB_HIP(hipMemcpyAsync(ptrs.uph, cur.uph, n * ub, k, stream));
            GCB_HIP(hipMemcpyAsync(ptrs.status, cur.status, (size_t)n, k, stream));
            if (p->qm)
                GCB_HIP(hipMemcpyAsync(const_cast<double*>(ptrs.qm), cur.qm, nd, k, stream));
            if (p->id)
                GCB_HIP(hipMemcpyAsync(ptrs.id, cur.id, (size_t)n * sizeof(int32_t), k, stream));
            t.done();
        }
    } else {
        Timer t(ctx, stream, GCB_TIMER_PUSH);
        GCB_HIP(push(ptrs, ptrs, nullptr, n_steps, 0));
        t.done();
    }
    return stats_end(ctx, dstats, p->status, p->n, stats, stream);
}

int gcb_load_fields_3d(gcb_ctx* ctx, const gcb_grid3_desc* d, const double* const E[3],
                       const double* const B[3], int32_t src, void* stream_) {
    if (!ctx) return fail(nullptr, GCB_EINVAL, "ctx is NULL");
    if (!d || !E || !B) return fail(ctx, GCB_EINVAL, "desc, E and B must be non-NULL");
    for (int a = 0; a < 3; ++a) {
        if (d->n[a] < 2 || d->n[a] > (1 << 24))
            return fail(ctx, GCB_EINVAL, "grid sizes must be in [2, 2^24]");
        if (!finite_pos(d->d[a])) return fail(ctx, GCB_EINVAL, "cell sizes must be finite and > 0");
    }
    if ((int64_t)d->n[0] * d->n[1] * d->n[2] * 6 >= ((int64_t)1 << 34))
        return fail(ctx, GCB_EINVAL, "grid too large");
    for (int k = 0; k < 6; ++k)
        for (int a = 0; a < 3; ++a)
            if (!(d->stagger[k][a] >= 0.0 && d->stagger[k][a] < 1.0))
                return fail(ctx, GCB_EINVAL, "stagger offsets must be in [0, 1)");
    if (d->dtype != GCB_F64 && d->dtype != GCB_F32)
        return fail(ctx, GCB_EINVAL, "unknown dtype %d", d->dtype);
    if (src != GCB_HOST && src != GCB_DEVICE)
        return fail(ctx, GCB_EINVAL, "src must be GCB_HOST or GCB_DEVICE");
    const double* comps[6] = {E[0], E[1], E[2], B[0], B[1], B[2]};
    for (int k = 0; k < 6; ++k)
        if (!comps[k]) return fail(ctx, GCB_EINVAL, "field component %d is NULL", k);
    GCB_HIP(hipSetDevice(ctx->device));
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    ctx->have_f3 = false;
    // rows of nx nodes, one per (j, l), l slowest: the 2D interleave of ny*nz rows
    const int rc = upload_interleaved(ctx, comps, d->n[0], d->n[1] * d->n[2], ctx->fields3,
                                      d->dtype == GCB_F32, src, stream);
    if (rc) return rc;
    for (int a = 0; a < 3; ++a) {
        ctx->n3[a] = d->n[a];
        ctx->d3[a] = d->d[a];
    }
    std::memcpy(ctx->stagger3, d->stagger, sizeof(ctx->stagger3));
    ctx->dtype3 = d->dtype;
    ctx->yee3 = std::memcmp(d->stagger, kYee3, sizeof(kYee3)) == 0;
    ctx->have_f3 = true;
    return GCB_OK;
}

int gcb_push_3d(gcb_ctx* ctx, gcb_particles3* p, const gcb_params* prm, int32_t n_steps,
                uint8_t* s_trace, gcb_stats* stats, void* stream_) {
    if (!ctx) return fail(nullptr, GCB_EINVAL, "ctx is NULL");
    if (!p) return fail(ctx, GCB_EINVAL, "particles is NULL");
    int rc;
    if ((rc = validate_params(ctx, prm))) return rc;
    if (prm->arith == GCB_ARITH_FAST && prm->form != GCB_FORM_F64)
        return fail(ctx, GCB_EUNSUPPORTED, "GCB_ARITH_FAST needs GCB_FORM_F64");
    // the 2D checks on the x, y, u, qm, id and status arrays, then z
    gcb_particles view{p->n, p->x, p->y, p->xp, p->yp, p->ux, p->uy, p->uz, p->qm, p->id,
                       p->status};
    if ((rc = validate_particles(ctx, &view, prm))) return rc;
    if (p->n > 0 && (!p->z || !p->zp))
        return fail(ctx, GCB_EINVAL, "particle arrays z, zp must be non-NULL");
    if (((uintptr_t)p->z | (uintptr_t)p->zp) & 7)
        return fail(ctx, GCB_EINVAL, "double arrays must be 8-byte aligned");
    if (n_steps < 0) return fail(ctx, GCB_EINVAL, "n_steps must be >= 0");
    if (prm->frame == GCB_FRAME_EXACT && prm->form != GCB_FORM_F64)
        return fail(ctx, GCB_EUNSUPPORTED, "the exact frame needs GCB_FORM_F64");
    if (!ctx->have_f3) return fail(ctx, GCB_ENOFIELDS, "gcb_load_fields_3d was not called");
    if (prm->form == GCB_FORM_F64 && ctx->dtype3 != GCB_F64)
        return fail(ctx, GCB_EINVAL, "GCB_FORM_F64 needs fields loaded as GCB_F64");
    if (prm->form == GCB_FORM_MIXED && ctx->dtype3 != GCB_F32)
        return fail(ctx, GCB_EINVAL, "GCB_FORM_MIXED needs fields loaded as GCB_F32");
    if (s_trace && p->n > 0 && !p->id && prm->sort_every > 0 && !prm->keep_order)
        return fail(ctx, GCB_EINVAL, "a switch trace with sorting needs particle ids");
    if (prm->replay && !s_trace && p->n > 0 && n_steps > 0)
        return fail(ctx, GCB_EINVAL, "replay needs the switch trace s_trace");
    GCB_HIP(hipSetDevice(ctx->device));
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    DevStats* dstats;
    if ((rc = stats_begin(ctx, stats, stream, &dstats))) return rc;
    if (prm->form == GCB_FORM_F64)
        rc = run_push3<double>(ctx, p, prm, n_steps, s_trace, dstats, stream);
    else
        rc = run_push3<float>(ctx, p, prm, n_steps, s_trace, dstats, stream);
    if (rc) return rc;
    return stats_end(ctx, dstats, p->status, p->n, stats, stream);
}

int gcb_push_backward_3d(gcb_ctx* ctx, const gcb_particles3* start, const gcb_params* prm,
                         int32_t n_steps, const double* const lam_end[9],
                         double* const lam_start[9], float* const dE[3], float* const dB[3],
                         void* stream_) {
    if (!ctx) return fail(nullptr, GCB_EINVAL, "ctx is NULL");
    if (!start) return fail(ctx, GCB_EINVAL, "particles is NULL");
    int rc;
    if ((rc = validate_params(ctx, prm))) return rc;
    gcb_particles view{start->n,  start->x,  start->y,  start->xp, start->yp, start->ux,
                       start->uy, start->uz, start->qm, start->id, start->status};
    if ((rc = validate_particles(ctx, &view, prm))) return rc;
    if (start->n > 0 && (!start->z || !start->zp))
        return fail(ctx, GCB_EINVAL, "particle arrays z, zp must be non-NULL");
    if (((uintptr_t)start->z | (uintptr_t)start->zp) & 7)
        return fail(ctx, GCB_EINVAL, "double arrays must be 8-byte aligned");
    if (n_steps < 0) return fail(ctx, GCB_EINVAL, "n_steps must be >= 0");
    if (!lam_end || !lam_start || !dE || !dB)
        return fail(ctx, GCB_EINVAL, "lam_end, lam_start, dE and dB must be non-NULL");
    const int64_t n = start->n;
    for (int c = 0; c < 9; ++c)
        if (n > 0 && (!lam_end[c] || !lam_start[c]))
            return fail(ctx, GCB_EINVAL, "adjoint array %d is NULL", c);
    for (int c = 0; c < 3; ++c)
        if (!dE[c] || !dB[c]) return fail(ctx, GCB_EINVAL, "dE/dB component %d is NULL", c);
    if (!ctx->have_f3) return fail(ctx, GCB_ENOFIELDS, "gcb_load_fields_3d was not called");
    if (prm->form != GCB_FORM_F64 || ctx->dtype3 != GCB_F64)
        return fail(ctx, GCB_EUNSUPPORTED, "the adjoint needs GCB_FORM_F64 and binary64 fields");
    if (prm->n_iter > 8)
        return fail(ctx, GCB_EUNSUPPORTED, "the adjoint supports n_iter <= 8");
    if ((rc = reject_push_options(ctx, prm))) return rc;
    GCB_HIP(hipSetDevice(ctx->device));
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    constexpr int kS = 9;   // state arrays: x, y, z, xp, yp, zp, ux, uy, uz
    const size_t nd = (size_t)n * sizeof(double);
    const size_t nodes = (size_t)ctx->n3[0] * ctx->n3[1] * ctx->n3[2];
    if ((rc = ensure(ctx, ctx->adj_states, (size_t)n_steps * kS * nd))) return rc;
    if ((rc = ensure(ctx, ctx->adj_trace, (size_t)n_steps * n))) return rc;
    if ((rc = ensure(ctx, ctx->adj_lists, (size_t)n_steps * (n + 1) * sizeof(uint32_t))))
        return rc;
    if ((rc = ensure(ctx, ctx->adj_lam, kS * nd))) return rc;
    if ((rc = ensure(ctx, ctx->adj_work, kS * nd + (size_t)n))) return rc;
    if ((rc = ensure(ctx, ctx->adj_grad, nodes * 6 * sizeof(float)))) return rc;
    constexpr int kMaxBatch = kAdj3MaxBatch;
    const size_t budget = record_budget(kAdj3RecordBudget);
    const size_t per_step = adjoint3_record_bytes(n, prm->n_iter, 1);
    int batch = per_step > 0 ? (int)std::min<size_t>(kMaxBatch, budget / per_step) : 1;
    batch = std::max(1, std::min(batch, std::max(1, (int)n_steps)));
    if ((rc = ensure(ctx, ctx->adj_samples, adjoint3_record_bytes(n, prm->n_iter, batch))))
        return rc;
    // the segment's particles in the tile order of their start positions, as
    // in the 2D backward (cubic kAdj3OrderTile-cell tiles)
    TileGeom3 og{};
    og.tile = kAdj3OrderTile;
    og.ntx = (ctx->n3[0] + og.tile - 1) / og.tile;
    og.nty = (ctx->n3[1] + og.tile - 1) / og.tile;
    og.ntz = (ctx->n3[2] + og.tile - 1) / og.tile;
    const bool ordered = n > 0 && n_steps > 0;
    double* qms = nullptr;          // q/m in tile order
    uint32_t* perm = nullptr;       // tile slot -> caller's slot
    if (ordered) {
        if ((rc = ensure(ctx, ctx->adj_order, nd + (size_t)n * 4))) return rc;
        qms = static_cast<double*>(ctx->adj_order.ptr);
        perm = reinterpret_cast<uint32_t*>(qms + n);
    }
    double* work = static_cast<double*>(ctx->adj_work.ptr);
    uint8_t* wstatus = reinterpret_cast<uint8_t*>(work + kS * (size_t)n);
    double* states = static_cast<double*>(ctx->adj_states.ptr);
    uint8_t* trace = static_cast<uint8_t*>(ctx->adj_trace.ptr);
    double* lam = static_cast<double*>(ctx->adj_lam.ptr);
    float* grad = static_cast<float*>(ctx->adj_grad.ptr);
    const double* src[kS] = {start->x,  start->y,  start->z,
                             start->xp, start->yp, start->zp,
                             static_cast<const double*>(start->ux),
                             static_cast<const double*>(start->uy),
                             static_cast<const double*>(start->uz)};
    Timer t(ctx, stream, GCB_TIMER_BACKWARD);
    if (ordered) {
        SortBuffers ssb{};
        if ((rc = prepare_sort(ctx, n, og.ntx * og.nty * og.ntz, ssb))) return rc;
        GCB_HIP(launch_cell_sort3(start->x, start->y, start->z, n, 1.0 / ctx->d3[0],
                                  1.0 / ctx->d3[1], 1.0 / ctx->d3[2], og, ssb, stream));
        GCB_HIP(hipMemcpyAsync(perm, ssb.idx, (size_t)n * 4, hipMemcpyDeviceToDevice, stream));
        if (start->qm) GCB_HIP(launch_permute_f64(start->qm, perm, n, qms, false, stream));
    }
    if (n > 0) {
        for (int c = 0; c < kS; ++c) {
            if (perm)
                GCB_HIP(launch_permute_f64(src[c], perm, n, work + c * (size_t)n, false, stream));
            else
                GCB_HIP(hipMemcpyAsync(work + c * (size_t)n, src[c], nd,
                                       hipMemcpyDeviceToDevice, stream));
        }
        GCB_HIP(hipMemsetAsync(wstatus, 0, (size_t)n, stream));
    }
    double* wqm = (perm && start->qm) ? qms : start->qm;
    ParticlePtrs3<double> w{};
    w.b.x = work;
    w.b.y = work + n;
    w.z = work + 2 * n;
    w.b.xp = work + 3 * n;
    w.b.yp = work + 4 * n;
    w.zp = work + 5 * n;
    w.b.ux = work + 6 * n;
    w.b.uy = work + 7 * n;
    w.b.uz = work + 8 * n;
    w.b.qm = wqm;
    w.b.id = nullptr;
    w.b.status = wstatus;
    const PushConst3 pc = make_const3(ctx, prm);
    // forward recomputation, keeping each step's start state and decisions:
    // with sort_every > 0 and a window that fits, the tiled push in place
    // (keep_order), which records the start state of every step inside its
    // launches; otherwise one launch of the global kernel and one state copy
    // per step.  The parity arithmetic makes either the forward pass bit for
    // bit.
    gcb_params rp = *prm;
    rp.keep_order = 1;
    rp.replay = 0;
    const TileGeom3 rg = make_geom3(ctx, &rp);
    const bool tiled_rec = n > 0 && n_steps > 0 && rp.sort_every > 0 &&
                           rp.kernel != GCB_KERNEL_GLOBAL && rg.window > 0 &&
                           tiled3_lds_bytes(rg.window, sizeof(double)) <= kMaxLds;
    if (tiled_rec) {
        rp.kernel = GCB_KERNEL_TILED;
        gcb_particles3 wp{n,    w.b.x, w.b.y, w.z,  w.b.xp, w.b.yp, w.zp,
                          w.b.ux, w.b.uy, w.b.uz, wqm,  nullptr, wstatus};
        const bool timing = ctx->timing;   // timed as part of the backward pass
        ctx->timing = false;
        rc = run_push3<double>(ctx, &wp, &rp, n_steps, trace, nullptr, stream, states);
        ctx->timing = timing;
        if (rc) return rc;
    }
    for (int32_t s = 0; s < n_steps && n > 0 && !tiled_rec; ++s) {
        GCB_HIP(hipMemcpyAsync(states + (size_t)s * kS * n, work, kS * nd,
                               hipMemcpyDeviceToDevice, stream));
        Push3Launch L;
        L.kind = PushKind::Global;
        L.yee = ctx->yee3;
        L.fields = ctx->fields3.ptr;
        L.n = n;
        L.tile_start = nullptr;
        L.geom = TileGeom3{};
        L.trace = trace + (size_t)s * n;
        L.replay = false;
        L.stats = nullptr;
        L.steps = 1;
        GCB_HIP(launch_push3_f64(L, w, w, pc, stream));
    }
    uint32_t* lists = static_cast<uint32_t*>(ctx->adj_lists.ptr);
    unsigned* counts = reinterpret_cast<unsigned*>(lists + (size_t)n_steps * n);
    if (n > 0 && n_steps > 0) {
        GCB_HIP(hipMemsetAsync(counts, 0, (size_t)n_steps * sizeof(unsigned), stream));
        GCB_HIP(launch_gca_lists(trace, n, n_steps, lists, counts, stream));
    }
    // reverse sweep
    for (int c = 0; c < kS && n > 0; ++c) {
        if (perm)
            GCB_HIP(launch_permute_f64(lam_end[c], perm, n, lam + c * (size_t)n, false, stream));
        else
            GCB_HIP(hipMemcpyAsync(lam + c * (size_t)n, lam_end[c], nd, hipMemcpyDeviceToDevice,
                                   stream));
    }
    GCB_HIP(hipMemsetAsync(grad, 0, nodes * 6 * sizeof(float), stream));
    for (int32_t s_hi = n_steps; s_hi > 0 && n > 0; s_hi -= batch) {
        const int32_t s_lo = std::max<int32_t>(0, s_hi - batch);
        Adjoint3Launch A;
        A.yee = ctx->yee3;
        A.fields = static_cast<const double*>(ctx->fields3.ptr);
        A.n = n;
        A.qm = wqm;
        A.grad_fields = grad;
        A.records = ctx->adj_samples.ptr;
        A.batch = batch;
        for (int32_t s = s_hi - 1; s >= s_lo; --s) {
            A.state = states + (size_t)s * kS * n;
            A.strace = trace + (size_t)s * n;
            A.list = lists + (size_t)s * n;
            A.count = counts + s;
            A.batch_slot = s - s_lo;
            GCB_HIP(launch_adjoint3_step(A, lam, pc, stream));
        }
        GCB_HIP(launch_adjoint3_scatter(A, trace + (size_t)s_lo * n, s_hi - s_lo, pc, stream));
    }
    for (int c = 0; c < kS && n > 0; ++c) {
        if (perm)
            GCB_HIP(launch_permute_f64(lam + c * (size_t)n, perm, n, lam_start[c], true,
                                       stream));
        else
            GCB_HIP(hipMemcpyAsync(lam_start[c], lam + c * (size_t)n, nd,
                                   hipMemcpyDeviceToDevice, stream));
    }
    if (n_steps == 0 && n > 0)
        for (int c = 0; c < kS; ++c)
            GCB_HIP(hipMemcpyAsync(lam_start[c], lam_end[c], nd, hipMemcpyDeviceToDevice,
                                   stream));
    // the 3D node-interleaved layout is the 2D one with nx columns and ny*nz rows
    float* const outs[6] = {dE[0], dE[1], dE[2], dB[0], dB[1], dB[2]};
    GCB_HIP(launch_deinterleave_add(grad, ctx->n3[0], ctx->n3[1] * ctx->n3[2], outs, stream));
    t.done();
    return GCB_OK;
}

int gcb_kinetic_energy(gcb_ctx* ctx, const gcb_particles* p, const gcb_params* prm,
                       double* out, double* const lam_u[3], void* stream_) {
    if (!ctx) return fail(nullptr, GCB_EINVAL, "ctx is NULL");
    int rc;
    if ((rc = validate_params(ctx, prm))) return rc;
    if (!p || p->n < 0) return fail(ctx, GCB_EINVAL, "invalid particles");
    if (!out) return fail(ctx, GCB_EINVAL, "out is NULL");
    if (p->n > 0 && (!p->ux || !p->uy || !p->uz))
        return fail(ctx, GCB_EINVAL, "u arrays must be non-NULL");
    if (lam_u && p->n > 0 && (!lam_u[0] || !lam_u[1] || !lam_u[2]))
        return fail(ctx, GCB_EINVAL, "lam_u entries must be non-NULL");
    GCB_HIP(hipSetDevice(ctx->device));
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if ((rc = ensure(ctx, ctx->ke_partial, kinetic_partial_elems(p->n) * sizeof(double))))
        return rc;
    Timer t(ctx, stream, GCB_TIMER_OTHER);
    GCB_HIP(launch_kinetic_energy(p->ux, p->uy, p->uz, prm->form == GCB_FORM_MIXED, p->n,
                                  prm->c, out, lam_u ? lam_u[0] : nullptr,
                                  lam_u ? lam_u[1] : nullptr, lam_u ? lam_u[2] : nullptr,
                                  static_cast<double*>(ctx->ke_partial.ptr), stream));
    t.done();
    return GCB_OK;
}

int gcb_sincos(gcb_ctx* ctx, const double* x, double* s, double* c, int64_t n,
               void* stream_) {
    if (!ctx) return fail(nullptr, GCB_EINVAL, "ctx is NULL");
    if (n < 0) return fail(ctx, GCB_EINVAL, "n must be >= 0");
    if (n > 0 && (!x || !s || !c)) return fail(ctx, GCB_EINVAL, "x, s and c must be non-NULL");
    GCB_HIP(hipSetDevice(ctx->device));
    GCB_HIP(launch_sincos(x, s, c, n, static_cast<hipStream_t>(stream_)));
    return GCB_OK;
}

int gcb_set_timing(gcb_ctx* ctx, int32_t enabled) {
    if (!ctx) return fail(nullptr, GCB_EINVAL, "ctx is NULL");
    for (auto& l : ctx->launches) {
        (void)hipEventDestroy(l.start);
        (void)hipEventDestroy(l.stop);
    }
    ctx->launches.clear();
    for (int k = 0; k < GCB_NTIMERS; ++k) {
        ctx->ms[k] = 0.0;
        ctx->count[k] = 0;
    }
    ctx->timing = enabled != 0;
    return GCB_OK;
}

int gcb_get_timing(gcb_ctx* ctx, double ms[GCB_NTIMERS], int64_t launches[GCB_NTIMERS]) {
    if (!ctx || !ms || !launches) return fail(ctx, GCB_EINVAL, "NULL argument");
    GCB_HIP(hipSetDevice(ctx->device));
    for (auto& l : ctx->launches) {
        GCB_HIP(hipEventSynchronize(l.stop));
        float t = 0.f;
        GCB_HIP(hipEventElapsedTime(&t, l.start, l.stop));
        ctx->ms[l.cls] += t;
        ctx->count[l.cls] += 1;
        (void)hipEventDestroy(l.start);
        (void)hipEventDestroy(l.stop);
    }
    ctx->launches.clear();
    for (int k = 0; k < GCB_NTIMERS; ++k) {
        ms[k] = ctx->ms[k];
        launches[k] = ctx->count[k];
    }
    return GCB_OK;
}

}  // extern "C"
