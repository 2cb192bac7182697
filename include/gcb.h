/*
 * gcb.h -- C ABI of libgcb, an MI355X (gfx950) implementation of the coupled
 * guiding-center / Boris particle pusher of Bacchini, Ripperda, Philippov &
 * Parfrey, "A coupled guiding center-Boris particle pusher for magnetized
 * plasmas in compact-object magnetospheres" (arXiv:2007.14401).
 *
 * Problem (Sec. 4, opening paragraph; Sec. 3.1): test particles that do not
 * act back on the fields are advanced through static E and B given on a grid.
 * At every step each particle is tested against the switch of Sec. 4.1 and
 * advanced either with the relativistic Boris push (Sec. 2.1) or with the
 * guiding-center leapfrog (Sec. 2.2.1 without, Sec. 2.2.2 with curvature
 * terms), converting to guiding-center variables and back (Sec. 3.1).
 *
 * Conventions shared by every entry point
 *   - Gaussian units with explicit c.  u is the spatial part of the
 *     four-velocity in velocity units (u = Gamma v), Gamma = sqrt(1+u^2/c^2).
 *   - 2D3V: positions (x, y) on a periodic box [0, nx*dx) x [0, ny*dy);
 *     u, E and B have three components; nothing depends on z.
 *   - Leapfrog staggering (Sec. 2.1): x^n at integer levels, u^{n-1/2} at
 *     half levels; the state also carries the previous position x^{n-1},
 *     needed for the midpoint R^{n-1/2} of the variable conversion (Sec. 3.1).
 *   - All array arguments of gcb_push / gcb_push_backward /
 *     gcb_kinetic_energy are DEVICE pointers on the context's device, owned
 *     by the caller, 8-byte aligned.  Field arrays handed to gcb_load_fields
 *     may be host or device pointers (see `src`).
 *   - Streams are passed as `void*` holding a hipStream_t (NULL = the null
 *     stream).  Work is enqueued on that stream; calls return without a
 *     device synchronisation unless stats or timings are requested.
 *   - Every int-returning call returns GCB_OK (0) or a negative code and
 *     never aborts; gcb_last_error(ctx) gives a message.  Arguments are
 *     validated before any device work is enqueued.
 *   - One context per host thread; a context is bound to one device.
 */
#ifndef GCB_H
#define GCB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define GCB_OK            0
#define GCB_EINVAL       -1   /* invalid argument (null pointer, bad size, bad enum) */
#define GCB_ENOFIELDS    -2   /* gcb_push before gcb_load_fields */
#define GCB_ENOMEM       -3   /* device allocation failed */
#define GCB_EHIP         -4   /* a HIP runtime call failed (message has the HIP error) */
#define GCB_EUNSUPPORTED -5   /* valid request the library does not serve */

/* precision of the device copy of the fields (gcb_grid_desc.dtype) */
#define GCB_F64 0
#define GCB_F32 1

/* arithmetic form (gcb_params.form) */
#define GCB_FORM_F64   0   /* everything in binary64; state u is double */
#define GCB_FORM_MIXED 1   /* binary32 bulk arithmetic, binary64 positions and
                              selected quantities; state u is float; needs
                              fields loaded with dtype GCB_F32 */

/* binary64 arithmetic (gcb_params.arith) */
#define GCB_ARITH_EXACT 0   /* every operation of the step separately rounded, in the
                               order of the CPU definition the library is tested
                               against (no fused multiply-add): results agree with it
                               bit for bit (the parity build of the kernels) */
#define GCB_ARITH_FAST  1   /* the production build: multiply-adds fused where the
                               compiler forms them (one rounding instead of two), and
                               a square root that only serves as a divisor taken as a
                               refined hardware reciprocal square root, quotients by a
                               shared value as products with its reciprocal; a step
                               differs from GCB_ARITH_EXACT by a few units in the last
                               place (relative 1e-12 asserted per step, switch decisions
                               identical); over many steps the difference grows as the
                               orbit's own sensitivity to its initial state does */

/* guiding-center frame (gcb_params.frame) */
#define GCB_FRAME_REDUCED 0   /* the paper's schemes: b = B/B, v_E = c E x B/B^2, E_par = E.b */
#define GCB_FRAME_EXACT   1   /* the exact frame of Sec. 2.2: b*, the exact v_E and kappa,
                                 E_par = E'/kappa, and with curvature = 1 the curvature terms
                                 of b*; GCB_FORM_F64, gcb_push and gcb_push_3d only */

/* gyration handling of a guiding-center step (gcb_params.gyration), Sec. 2.2 */
#define GCB_GYRATION_MU    0   /* mu/m = u_perp_g^2/(2 B kappa) conserved (eq. dmudt): u_perp_g^2
                                  = 2 mu B kappa/m at every point of the step (the paper's choice) */
#define GCB_GYRATION_UPERP 1   /* u_perp_g held at its value at the decomposition over the step:
                                  the alternative the paper describes, which conserves the energy
                                  exactly when E = 0 and the curvature terms vanish */
#define GCB_GYRATION_ZERO  2   /* mu = 0: the gyration found at the decomposition is discarded
                                  (the paper allows it where radiation has removed it) */
#define GCB_GYRATION_PHASE 3   /* mu conserved as GCB_GYRATION_MU, and the gyration phase
                                  evolved (the extra equation Sec. 3.1 allows) instead of the
                                  gyration direction being held: over the step the direction is
                                  turned about b at R^n by -(q/m) B dt/(c kappa Gamma), Gamma of
                                  eq. lfacgca2 at R^n with the mean of u_par before and after the
                                  parallel update (the gyration frequency of a particle whose
                                  guiding center drifts with v_E); reduced frame, mirror = 0 */

/* where field arrays live (gcb_load_fields.src) */
#define GCB_HOST   0
#define GCB_DEVICE 1

/* kernel choice (gcb_params.kernel) */
#define GCB_KERNEL_AUTO   0   /* tiled when sort_every > 0 and the grid allows it */
#define GCB_KERNEL_GLOBAL 1   /* one lane per particle, gathers through the caches */
#define GCB_KERNEL_TILED  2   /* cell-sorted particles, LDS field tiles, per-regime queues */

/* sticky per-particle status bits (gcb_particles.status) */
#define GCB_ST_NONFINITE 1    /* a non-finite position or four-velocity was produced   */
#define GCB_ST_KAPPA     2    /* v_E >= c at a guiding-center evaluation; 1 - v_E^2/c^2
                                 clamped to 1e-12                                        */
#define GCB_ST_QUAD      4    /* parallel update (Sec. 2.2.2) had no admissible root     */
#define GCB_ST_BZERO     8    /* B = 0 at a guiding-center evaluation point              */
#define GCB_ST_FPRES    16    /* last fixed-point increment |R^K - R^{K-1}| > fp_tol      */
#define GCB_ST_HALO     32    /* informational: a gather fell outside the LDS tile window
                                 and was served from global memory (same values)         */
#define GCB_ST_OUT      64    /* curved-spacetime push: the particle left the (r, theta)
                                 domain and is no longer advanced                        */
#define GCB_ST_MIRROR  128    /* (v_perp_g/c)^2 = u_perp_g^2/(Gamma^2 c^2) at a guiding-center
                                 decomposition exceeded gcb_params.mirror_tol: the mirror
                                 terms the reduced equations leave out may not be
                                 negligible (the check Sec. 2.2 asks for)               */

typedef struct gcb_ctx gcb_ctx;

/* Create a context bound to HIP device `device`.  *out receives the context
   (NULL on failure).  Returns GCB_EHIP if the device cannot be used. */
int gcb_create(gcb_ctx** out, int device);

/* Free all device memory owned by the context.  NULL is accepted. */
void gcb_destroy(gcb_ctx* ctx);

/* Message for the last failed call on this context (or, for ctx == NULL, on
   this thread).  The string is owned by the library and valid until the next
   call on the same context/thread. */
const char* gcb_last_error(const gcb_ctx* ctx);

/* Grid of the static fields.  Field component k (order Ex, Ey, Ez, Bx, By,
   Bz) has its nodes at ((i + stagger[k][0]) dx, (j + stagger[k][1]) dy),
   i in [0,nx), j in [0,ny), periodic.  The paper gathers fields at a particle
   with a linear shape function from the surrounding nodes and gradients by
   differentiating it (Sec. 4, opening paragraph): bilinear interpolation on
   each component's own lattice.  The cell size of the switch is
   dl = sqrt(dx dy) (Sec. 3, effective cell size). */
typedef struct {
    int32_t nx, ny;          /* >= 2 each */
    double  dx, dy;          /* > 0 */
    double  stagger[6][2];   /* offsets in cells, each in [0, 1) */
    int32_t dtype;           /* GCB_F64 or GCB_F32: precision of the device copy */
} gcb_grid_desc;

/* Copy the six field components into context-owned device storage
   (node-interleaved, converted to desc->dtype).  E[c] and B[c] point to
   nx*ny doubles in row-major order, element [j*nx + i].  src says whether
   they are host (GCB_HOST) or device (GCB_DEVICE) pointers; the caller keeps
   ownership.  Replaces previously loaded fields.  Enqueued on `stream`;
   host sources are copied before the call returns. */
int gcb_load_fields(gcb_ctx* ctx, const gcb_grid_desc* desc,
                    const double* const E[3], const double* const B[3],
                    int32_t src, void* stream);

/* Parameters of a push (Sec. 2.2, 3, 4.1). */
typedef struct {
    double  dt;          /* time step, > 0 */
    double  c;           /* speed of light, > 0 */
    double  qm;          /* q/m used when particles.qm == NULL (signed, != 0) */
    double  f_rho;       /* switch threshold on rho~/dl (Sec. 4.1; 0.4 there) */
    double  f_E;         /* switch threshold on E/B (Sec. 4.1; 1 there) */
    double  fp_tol;      /* iteration-error threshold for GCB_ST_FPRES (1e-7, Sec. 2.2.1) */
    int32_t curvature;   /* 1: Sec. 2.2.2 scheme (curvature drift and acceleration);
                            0: Sec. 2.2.1 scheme */
    int32_t n_iter;      /* K >= 1 fixed-point iterations for R^{n+1} (3-4 in Sec. 2.2) */
    int32_t form;        /* GCB_FORM_F64 or GCB_FORM_MIXED */
    int32_t sort_every;  /* cell-sort the particles every this many steps
                            (0 = never; the tiled kernel needs > 0) */
    int32_t kernel;      /* GCB_KERNEL_* */
    int32_t tile;        /* tile edge in cells for the tiled kernel (0 = 24) */
    int32_t replay;      /* 1: take every switch decision from s_trace (written by an
                            earlier gcb_push over the same particles) instead of
                            evaluating the switch; the push is then the map that
                            gcb_push_backward differentiates, with S held fixed */
    int32_t frame;       /* GCB_FRAME_REDUCED (0) or GCB_FRAME_EXACT.  The exact frame
                            (Sec. 2.2): w_E = c E x B/(E^2 + B^2), s = sqrt(1 - 4 w_E^2/c^2),
                            v_E = 2 w_E/(1 + s), kappa = (1 - v_E^2/c^2)^(-1/2),
                            B' = sqrt((B^2 - E^2 + (E^2 + B^2) s)/2), E' = E.B/B',
                            b* = eta (Psi E_perp + B) with Psi = 2 E' B^2/(B'(E^2+B^2)(1+s)),
                            eta = 1/(B sqrt(Psi^2 E_perp^2/B^2 + 1)); the scheme
                            (Sec. 2.2.1 with curvature = 0, Sec. 2.2.2 with curvature = 1)
                            and the conversions of Sec. 3.1 then use b*, this v_E and
                            kappa, and du_par/dt = (q/m) E'/kappa; with curvature = 1,
                            (b*.grad)b* and (v_E.grad)b* in eq. curvdrift and eq. dupardt,
                            the gradient of b* by the chain rule through E and B (the
                            gather then also forms the E gradients).  Binary64 (either
                            arithmetic), gcb_push and gcb_push_3d, mirror = 0; other calls
                            and combinations return GCB_EUNSUPPORTED. */
    int32_t gyration;    /* GCB_GYRATION_* (0 = mu conserved).  Other values than
                            GCB_GYRATION_MU: gcb_push and gcb_push_3d only (both forms;
                            both frames, except GCB_GYRATION_PHASE: reduced frame and no
                            mirror terms); other calls return GCB_EUNSUPPORTED */
    int32_t mirror;      /* 1: add the mirror force and the grad-B drift that Sec. 2.2
                            names and leaves out, with the step's mu (mu/m =
                            u_perp_g^2/(2 B kappa) under GCB_GYRATION_MU):
                            du_par/dt gains -(mu/(m kappa Gamma)) b.grad|B| and the
                            bracket of the curvature drift (eq. curvdrift) gains
                            (mu/(m kappa Gamma)) grad|B| -- grad(B/kappa) is taken as
                            grad|B|/kappa, so with E = 0 these are the textbook
                            relativistic terms.  The force is time-centred by one
                            predictor-corrector pass on 1/Gamma (two solves of the
                            parallel update); the conversions of Sec. 3.1 are
                            unchanged.  Needs curvature = 1 (else GCB_EUNSUPPORTED);
                            gcb_push and gcb_push_3d only, both forms; 0 (default):
                            the paper's reduced equations */
    double  mirror_tol;  /* > 0: set GCB_ST_MIRROR where (v_perp_g/c)^2 exceeds this at a
                            guiding-center decomposition (Gamma of the full u), the
                            validity check of leaving out (or of the size of) the mirror
                            terms, whose ratio to the curvature terms grows as
                            v_perp_g^2 (Sec. 2.2); 0 (default): no check.  Finite and
                            >= 0 (else GCB_EINVAL); gcb_push, gcb_push_3d and gcb_push_gr
                            (there with c = 1 and the metric's norm of u_perp_g); the
                            adjoints return GCB_EUNSUPPORTED for a value other than 0 */
    int32_t arith;       /* GCB_ARITH_EXACT (0, default) or GCB_ARITH_FAST: how the
                            binary64 form evaluates the step (see below).
                            GCB_ARITH_FAST: gcb_push, gcb_push_noalloc, gcb_push_3d
                            and gcb_push_gr with GCB_FORM_F64 only (else
                            GCB_EUNSUPPORTED) */
    int32_t keep_order;  /* 1: with sort_every > 0 the particles are still cell-sorted
                            (the tiled kernel works through each tile's particles) but
                            every particle is written back to its own slot, so the
                            arrays keep their order and a switch trace needs no ids
                            (trace column = slot); the results are those of any other
                            order.  0 (default): sorting permutes the arrays.  Values
                            other than 0 and 1: GCB_EINVAL; gcb_push, gcb_push_noalloc,
                            gcb_push_3d and the backward passes only (else
                            GCB_EUNSUPPORTED) */
} gcb_params;

/* Particle state, structure of arrays, caller-owned device memory of length n.
   gcb_push updates it in place; when sorting is on, all arrays (including qm,
   id and status) are permuted together, so `id` is how a caller follows a
   particle. */
typedef struct {
    int64_t  n;            /* number of particles, >= 0 */
    double  *x, *y;        /* x^n, wrapped into the box */
    double  *xp, *yp;      /* x^{n-1} (any periodic image) */
    void    *ux, *uy, *uz; /* u^{n-1/2}: double (GCB_FORM_F64) or float (GCB_FORM_MIXED) */
    double  *qm;           /* optional per-particle q/m (NULL: params.qm) */
    int32_t *id;           /* optional particle ids (NULL: none); values in [0, n)
                              when a switch trace is requested */
    uint8_t *status;       /* required: sticky GCB_ST_* bits, OR-ed by every step */
} gcb_particles;

typedef struct {
    int64_t gca_steps;       /* particle-steps taken with the guiding-center system */
    int64_t boris_steps;     /* particle-steps taken with the Boris push */
    int64_t flagged;         /* particles with any status bit other than GCB_ST_HALO at the end */
    int64_t halo_misses;     /* particle-steps with a gather outside the LDS window */
    double  max_fp_residual; /* max over guiding-center steps of |R^K - R^{K-1}|_inf */
    int64_t status_counts[8];/* particles with status bit 2^k set at the end, k = 0..7
                                (GCB_ST_NONFINITE ... GCB_ST_MIRROR) */
} gcb_stats;

/* Advance the particles by n_steps steps of the coupled scheme (Sec. 3.1):
   per particle and step, decide S from the fields at x^n (Sec. 4.1), then
   Boris (S = 1) or guiding-center leapfrog (S = 0), then store x^{n+1},
   x^n (as the previous position) and u^{n+1/2}.
   s_trace (nullable, device, n_steps*n bytes): s_trace[step*n + k] = S for
   the particle with id k (or array slot k if id == NULL and sorting is off);
   written, or read when params.replay is 1 (then it must be non-NULL).
   stats (nullable, host): filled after a device synchronisation. */
int gcb_push(gcb_ctx* ctx, gcb_particles* p, const gcb_params* prm,
             int32_t n_steps, uint8_t* s_trace, gcb_stats* stats, void* stream);

/* For callers that cannot allocate device memory -- code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc: gcb_push
   (same arguments, same kernels, bit-for-bit the same results) with every
   piece of the library's call scratch (cell-sort keys and permutation, the
   tile-ordered copy of the state, statistics accumulators) carved from a
   fixed device array of GCB_NOALLOC_SCRATCH_BYTES that the library holds on
   each device it runs on until the process ends; the call performs no
   hipMalloc/hipFree and no other allocation.  With sorting on (sort_every >
   0, n > 0) a call needs about (16 + 4*8 + 3*sizeof(u) + 1 [+ 8 with qm]
   [+ 4 with id]) bytes per particle plus 32 kB for statistics: about 720,000
   binary64 particles with qm and id fit.  A call that needs more returns
   GCB_EINVAL before any device work is enqueued.  Fields must have been
   loaded (gcb_load_fields allocates).  The array keeps the last call's
   contents; what must start at zero is cleared by the call.  Every context
   on a device shares that device's array: calls that overlap in time on one
   device (other streams, other threads) race and must be serialised by the
   caller.  Timings (gcb_set_timing) are not recorded for this call. */
#define GCB_NOALLOC_SCRATCH_BYTES (64u << 20)
int gcb_push_noalloc(gcb_ctx* ctx, gcb_particles* p, const gcb_params* prm,
                     int32_t n_steps, uint8_t* s_trace, gcb_stats* stats, void* stream);

/* Reverse-mode derivative of n_steps pushes started from `start` (which is
   not modified), with every switch decision held at its forward value.
   lam_end[7]: device arrays of length n with dL/d(x, y, xp, yp, ux, uy, uz)
   at the end of the segment (double).  lam_start[7]: output, the same
   derivatives at the segment start (double, overwritten).  dE[3], dB[3]:
   device float arrays of nx*ny elements, element [j*nx+i] of component k,
   ACCUMULATED (+=) with dL/dF at every node.  Only GCB_FORM_F64 with
   fields loaded as GCB_F64.  The call works on the particles in the tile
   order of their start positions (permuted in and the adjoint permuted back;
   no result depends on the order).  The forward steps are recomputed
   internally: with params.sort_every > 0 by the tiled push in place
   (keep_order), else by the cache-served kernel; needs n_steps * n * 61 +
   n * 12 bytes of context scratch plus the gather-point records of up to 32
   steps (64 bytes per gather point, at most 128 GiB and half the device
   memory free at the call). */
int gcb_push_backward(gcb_ctx* ctx, const gcb_particles* start,
                      const gcb_params* prm, int32_t n_steps,
                      const double* const lam_end[7], double* const lam_start[7],
                      float* const dE[3], float* const dB[3], void* stream);

/* Mean kinetic energy per unit mass L = (1/n) sum (Gamma - 1) c^2 of the
   state (the loss of the differentiation workload).  out (device, 1 double)
   receives L.  lam_u (nullable, 3 device double arrays of length n) receives
   dL/du = u / (n Gamma). */
int gcb_kinetic_energy(gcb_ctx* ctx, const gcb_particles* p,
                       const gcb_params* prm, double* out,
                       double* const lam_u[3], void* stream);

/* The library's binary64 sin and cos, the ones the curved-spacetime metric
   takes of theta (Sec. 2.3) and the gyro-phase option of the phase advance
   (Sec. 3.1): Cody-Waite reduction by pi/2 (two-part constant, exact
   multiples for |x| < 1.6e6) and Taylor polynomials of degree 19 and 20 on
   [-pi/4, pi/4], within two units in the last place of the correctly rounded
   values away from their zeros, for |x| <= 1e5 at least.  x, s and c are
   device arrays of n doubles on the context's device (s[i] = sin x[i],
   c[i] = cos x[i]); caller-owned; enqueued on `stream`.  n < 0 or NULL
   arrays with n > 0: GCB_EINVAL. */
int gcb_sincos(gcb_ctx* ctx, const double* x, double* s, double* c, int64_t n,
               void* stream);

/* ---------------------------------------------------------------------------
   Curved spacetime (Sec. 2.3, 2.4, 3.2): the coupled scheme in Kerr
   spacetime (M = 1, spin a) in spherical Kerr-Schild coordinates, geometrized
   units (c = G = 1).  The fields are axisymmetric and static.

   Grid: D^i and B^i (contravariant components along r, theta, phi) on the
   nodes r = r_min + i dr, theta = j dth of a uniform grid, i in [0, nr],
   j in [0, nth], dr = (r_max - r_min)/nr, dth = pi/nth, all six components
   at the nodes, gathered with the linear shape function (bilinear in r and
   theta; points beyond the grid take the value at its nearest edge).  The
   cell length of the switch is dl = sqrt(proper area of the particle's cell)
   (Sec. 3, eq. volint over the (r, theta) 2-metric; 2 x 2 Gauss-Legendre). */
typedef struct {
    int32_t nr, nth;        /* cells along r and theta, >= 1 */
    double  r_min, r_max;   /* 0 < r_min < r_max */
    double  spin;           /* Kerr a, |a| < 1 */
    int32_t dtype;          /* GCB_F64 (plain path) or GCB_F32 (precision form) */
} gcb_gr_desc;

/* Load D[3] = (D^r, D^th, D^ph) and B[3] = (B^r, B^th, B^ph): each an array
   of (nth+1)*(nr+1) doubles, element [j*(nr+1) + i] at node (i, j), host
   (GCB_HOST) or device (GCB_DEVICE) memory, caller-owned.  Builds the
   node-interleaved device copy and the table of cell lengths.  Replaces
   earlier curved-spacetime fields; the flat-space fields are independent. */
int gcb_load_fields_gr(gcb_ctx* ctx, const gcb_gr_desc* desc,
                       const double* const D[3], const double* const B[3],
                       int32_t src, void* stream);

/* Particle state of the curved-spacetime push, structure of arrays,
   caller-owned device memory of length n: position x^i = (r, theta, phi) and
   covariant four-velocity u_i at the same time level (Sec. 3.2, not
   staggered).  Updated in place; with params.sort_every > 0 all arrays
   (including qm, id and status) are permuted together into (r, theta) tile
   order every sort_every steps, so `id` is how a caller follows a particle.
   phi is kept in [0, 2 pi). */
typedef struct {
    int64_t  n;
    double  *r, *th, *ph;
    void    *ur, *uth, *uph;  /* double (GCB_FORM_F64) or float (GCB_FORM_MIXED) */
    double  *qm;            /* optional per-particle q/m (NULL: params.qm) */
    int32_t *id;            /* optional particle ids, permuted with the sort; values in
                               [0, n) when a switch trace is requested with sorting */
    uint8_t *status;        /* required: sticky GCB_ST_* bits */
} gcb_gr_particles;

/* Advance by n_steps coupled steps (Sec. 3.2): per particle and step, the
   switch at x^n with Gamma of the full u (guiding center iff B > 0,
   Gamma/(|q/m| B dl) < f_rho and D/B < f_E), then either the full-orbit step
   of Sec. 2.3 (half Lorentz push in the local frame of the normal observer,
   implicit-midpoint geodesic update by n_iter fixed-point iterations, half
   push) or the guiding-center step of Sec. 2.4 (half parallel push,
   implicit-midpoint update of (R, u_par) by n_iter iterations, half push,
   u rebuilt at R^{n+1} with the gyration direction of the step start).
   Reads dt, qm, f_rho, f_E, fp_tol, mirror_tol, n_iter, form, arith and
   sort_every of params (c is 1 here; replay must be 0; frame, gyration and
   mirror must keep their defaults).  GCB_FORM_F64 needs fields loaded as
   GCB_F64 and takes either arith; GCB_FORM_MIXED (binary32 fields, metric,
   four-velocity and bulk arithmetic, binary64 positions, and binary64 for
   Gamma when |u|^2 > 1e6, for 1 - v_E^2 when v_E^2 > 0.81 and for a switch
   ratio within a relative 1e-4 of its threshold) needs GCB_F32 fields.
   A particle whose new position leaves r_min <= r < r_max, 0 <= theta <= pi
   gets GCB_ST_OUT and keeps its state from then on.
   s_trace (nullable, device, n_steps*n bytes): s_trace[step*n + k] = 0
   (guiding center), 1 (full orbit) or 2 (not advanced) for the particle
   with id k (or array slot k when id is NULL; sorting then needs ids).
   stats (nullable, host): as for gcb_push; max_fp_residual covers both
   branches (both iterate); flagged counts GCB_ST_OUT too. */
int gcb_push_gr(gcb_ctx* ctx, gcb_gr_particles* p, const gcb_params* prm,
                int32_t n_steps, uint8_t* s_trace, gcb_stats* stats, void* stream);

/* ---------------------------------------------------------------------------
   Three dimensions: the coupled scheme of gcb_push (same equations, switch,
   params and status bits) on a periodic 3D box [0, nx dx) x [0, ny dy) x
   [0, nz dz).  The gather is the linear shape function in three dimensions
   (Sec. 4, opening paragraph): trilinear interpolation on the 2 x 2 x 2 nodes
   of each component's own lattice, summed z plane by z plane, with gradients
   along x, y and z; (b.grad)b and (v_E.grad)b then include the z
   derivatives, and the guiding-center position R has three components.
   The cell size of the switch is dl = (dx dy dz)^(1/3) (Sec. 3, effective
   cell size).  Its adjoint is gcb_push_backward_3d. */
typedef struct {
    int32_t n[3];            /* nx, ny, nz: nodes per axis, each in [2, 2^24] */
    int32_t dtype;           /* GCB_F64 or GCB_F32: precision of the device copy */
    double  d[3];            /* dx, dy, dz > 0 */
    double  stagger[6][3];   /* offsets in cells, each in [0, 1); the 3D Yee
                                lattice is Ex (1/2,0,0), Ey (0,1/2,0), Ez (0,0,1/2),
                                Bx (0,1/2,1/2), By (1/2,0,1/2), Bz (1/2,1/2,0) */
} gcb_grid3_desc;

/* Copy the six components into context-owned device storage (node
   interleaved, converted to desc->dtype).  E[c] and B[c] point to nx*ny*nz
   doubles, element [(l*ny + j)*nx + i] at node (i, j, l), host (GCB_HOST) or
   device (GCB_DEVICE) memory, caller-owned.  Replaces earlier 3D fields; the
   2D and curved-spacetime fields are independent.  Host sources are copied
   before the call returns. */
int gcb_load_fields_3d(gcb_ctx* ctx, const gcb_grid3_desc* desc,
                       const double* const E[3], const double* const B[3],
                       int32_t src, void* stream);

/* 3D particle state: gcb_particles with z and its previous value. */
typedef struct {
    int64_t  n;
    double  *x, *y, *z;      /* x^n, wrapped into the box */
    double  *xp, *yp, *zp;   /* x^{n-1} (any periodic image) */
    void    *ux, *uy, *uz;   /* u^{n-1/2}: double (GCB_FORM_F64) or float (GCB_FORM_MIXED) */
    double  *qm;             /* optional per-particle q/m (NULL: params.qm) */
    int32_t *id;             /* optional particle ids; values in [0, n) when a switch
                                trace is requested with sorting */
    uint8_t *status;         /* required: sticky GCB_ST_* bits */
} gcb_particles3;

/* Advance by n_steps coupled steps in 3D.  Arguments, sorting (cubic tiles of
   params.tile cells, 0 = 6; the LDS window holds (tile + 2 halo)^3 nodes of
   six components and must fit in 160 KiB for the tiled kernel), switch trace,
   replay and stats behave as for gcb_push. */
int gcb_push_3d(gcb_ctx* ctx, gcb_particles3* p, const gcb_params* prm,
                int32_t n_steps, uint8_t* s_trace, gcb_stats* stats, void* stream);

/* Reverse-mode derivative of n_steps 3D pushes started from `start` (not
   modified), every switch decision held at its forward value: gcb_push_backward
   for the 3D state.  lam_end[9]: device arrays of length n with
   dL/d(x, y, z, xp, yp, zp, ux, uy, uz) at the end of the segment (double);
   lam_start[9]: output, the same at the segment start (double, overwritten).
   dE[3], dB[3]: device float arrays of nx*ny*nz elements, element
   [(l*ny + j)*nx + i] of component k, ACCUMULATED (+=) with dL/dF at every
   node.  Only GCB_FORM_F64 with 3D fields loaded as GCB_F64, the reduced
   frame, mu conserved and n_iter <= 8 (else GCB_EUNSUPPORTED).  As in 2D the
   call works in the tile order of the start positions, and the forward steps
   are recomputed internally: with params.sort_every > 0 and a tile window
   that fits in LDS by the tiled push in place (keep_order), else by the
   cache-served kernel; needs n_steps * n * 77 + n * 12 bytes of context
   scratch plus the gather-point records of up to 8 steps (84 bytes per
   gather point, at most 32 GiB and half the device memory free). */
int gcb_push_backward_3d(gcb_ctx* ctx, const gcb_particles3* start, const gcb_params* prm,
                         int32_t n_steps, const double* const lam_end[9],
                         double* const lam_start[9], float* const dE[3], float* const dB[3],
                         void* stream);

/* Kernel timing with HIP events recorded around every launch on the launch
   stream.  gcb_set_timing(ctx, 1) clears and enables; gcb_get_timing
   synchronises on the recorded events and returns, for each kernel class,
   the summed milliseconds and the launch count. */
#define GCB_TIMER_PUSH     0   /* push kernels (one launch per step) */
#define GCB_TIMER_SORT     1   /* every kernel of a cell-sort        */
#define GCB_TIMER_BACKWARD 2   /* adjoint kernels                    */
#define GCB_TIMER_OTHER    3
#define GCB_NTIMERS        4
int gcb_set_timing(gcb_ctx* ctx, int32_t enabled);
int gcb_get_timing(gcb_ctx* ctx, double ms[GCB_NTIMERS], int64_t launches[GCB_NTIMERS]);

#ifdef __cplusplus
}
#endif
#endif /* GCB_H */
