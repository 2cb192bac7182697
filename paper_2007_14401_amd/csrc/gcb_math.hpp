// Per-particle arithmetic of the coupled guiding-center / Boris pusher (device
// code), templated on the bulk arithmetic type R.
//
// R = double: the binary64 form.  Every expression is evaluated in a fixed
//   order with separate multiplies and adds (its translation unit is compiled
//   with -ffp-contract=off), so results are reproducible bit for bit.
// R = float: the mixed form.  Bulk arithmetic in binary32; positions, their
//   increments' accumulation, midpoints and the periodic wrap stay binary64;
//   binary64 is also used for the Lorentz factor of ultra-relativistic
//   particles (u^2/c^2 > 1e6), for 1 - v_E^2/c^2 when E/B > 0.9 (written as
//   ((B^2 - E^2) B^2 + (E.B)^2)/B^4, free of the cancellation of 1 - v_E^2),
//   and for the switch test when a ratio lies within 1e-4 of its threshold.
//
// The field source is a template parameter: the same arithmetic serves
// gathers from the LDS tile window and from global memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "gcb_access.hpp"
#include "gcb_common.hpp"
#include "gcb_trig.hpp"

// The arithmetic below is compiled once per form and contraction setting
// (each in a translation unit of its own); an inline namespace per setting
// keeps the instances of different units apart.
#ifndef GCB_ARITH_NS
#define GCB_ARITH_NS arith_exact
#endif

namespace gcb {
inline namespace GCB_ARITH_NS {

template <typename R>
constexpr bool kMixed = std::is_same<R, float>::value;

// The production form of the binary64 arithmetic (GCB_ARITH_FAST; its unit
// defines GCB_FAST_ARITH): besides contracted multiply-adds, a square root
// that only serves as a divisor becomes a reciprocal square root (B and 1/B
// from 1/sqrt(B^2), kappa and 1/kappa from 1/sqrt(1 - v_E^2/c^2), 1/Gamma
// from 1/sqrt(1 + u^2/c^2)) and divisions by per-launch constants become
// multiplications.  Each such value differs from the correctly rounded one
// by a few units in the last place.
#ifndef GCB_FAST_ARITH
#define GCB_FAST_ARITH 0
#endif
template <typename R>
constexpr bool kFastD = (GCB_FAST_ARITH != 0) && std::is_same<R, double>::value;

// A Lorentz factor and, in the production form, its reciprocal.
template <typename R>
struct Gam {
    R g, inv;
};

// num / Gamma: a division, or in the production form a multiplication by
// the reciprocal
template <typename R>
GCB_HD R over(R num, const Gam<R>& G) {
    if constexpr (kFastD<R>)
        return num * G.inv;
    else
        return num / G.g;
}

// Constants of a launch in the bulk type.
template <typename R>
struct Consts {
    R dt, h, c, c2, inv_c2, f_rho, f_E, inv_dl, inv_dx, inv_dy;
};

template <typename R>
GCB_HD Consts<R> make_consts(const PushConst& pc) {
    Consts<R> k;
    k.dt = (R)pc.dt;
    k.h = (R)(0.5 * pc.dt);
    k.c = (R)pc.c;
    k.c2 = (R)pc.c2;
    k.inv_c2 = (R)pc.inv_c2;
    k.f_rho = (R)pc.f_rho;
    k.f_E = (R)pc.f_E;
    k.inv_dl = (R)pc.inv_dl;
    k.inv_dx = (R)pc.inv_dx;
    k.inv_dy = (R)pc.inv_dy;
    return k;
}

// Register copy of one particle's state: positions binary64, u in R.
template <typename R>
struct Regs {
    double x, y, xp, yp;
    R ux, uy, uz;
    double qm;
};

// ---------------------------------------------------------------------------
// Gather (Sec. 4, opening paragraph): linear shape function on the 2x2 nodes
// of each component's own lattice; gradients by differentiating it.

template <typename R>
struct Sample {
    static constexpr bool kGradE = false;
    R E[3], B[3];
    R dBx[3], dBy[3];   // d B_i / dx, d B_i / dy
};

// A sample with the E gradients as well (the exact guiding-center frame with
// curvature: b* depends on E): W differentiated on each E lattice too.
template <typename R>
struct SampleEG : Sample<R> {
    static constexpr bool kGradE = true;
    R dEx[3], dEy[3];   // d E_i / dx, d E_i / dy
};

// One component at grid coordinates (gx, gy) = (X/dx, Y/dy) with lattice
// offset (sx, sy) in cells (runtime stagger table).
template <typename R, bool kGrad, class Acc>
GCB_HD void interp_comp(const Acc& acc, int k, double gx, double gy,
                                            double sx, double sy, const Consts<R>& K, R& val,
                                            R& ddx, R& ddy) {
    const double xi = gx - sx;
    const double eta = gy - sy;
    const double fi = floor(xi);
    const double fj = floor(eta);
    const R wx = (R)(xi - fi);
    const R wy = (R)(eta - fj);
    double f00d, f10d, f01d, f11d;
    acc.quad(k, (int)fi, (int)fj, f00d, f10d, f01d, f11d);
    const R f00 = (R)f00d, f10 = (R)f10d, f01 = (R)f01d, f11 = (R)f11d;
    const R ax = (R)1 - wx;
    const R ay = (R)1 - wy;
    val = (((ax * ay) * f00 + (wx * ay) * f10) + (ax * wy) * f01) + (wx * wy) * f11;
    if (kGrad) {
        ddx = (ay * (f10 - f00) + wy * (f11 - f01)) * K.inv_dx;
        ddy = (ax * (f01 - f00) + wx * (f11 - f10)) * K.inv_dy;
    }
}

// The six components from four located 2x2 stencils (2D Yee lattice): the
// same operations as interp_comp, with the floor/weight computations shared
// by the components of one weight set.
template <typename R, bool kGrad, class Loader, class S>
GCB_HD void interp_yee(const Loader& ld, const R wx[2], const R wy[2],
                                           const Consts<R>& K, S& s) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int set = kYeeSet[k];
        const R bx = wx[set & 1];
        const R by = wy[set >> 1];
        const R ax = (R)1 - bx;
        const R ay = (R)1 - by;
        R f00, f10, f01, f11;
        ld.template load4<R>(set, k, f00, f10, f01, f11);
        const R val = (((ax * ay) * f00 + (bx * ay) * f10) + (ax * by) * f01) + (bx * by) * f11;
        if (k < 3) {
            s.E[k] = val;
            if constexpr (S::kGradE) {
                s.dEx[k] = (ay * (f10 - f00) + by * (f11 - f01)) * K.inv_dx;
                s.dEy[k] = (ax * (f01 - f00) + bx * (f11 - f10)) * K.inv_dy;
            }
        } else {
            s.B[k - 3] = val;
            if (kGrad) {
                s.dBx[k - 3] = (ay * (f10 - f00) + by * (f11 - f01)) * K.inv_dx;
                s.dBy[k - 3] = (ax * (f01 - f00) + bx * (f11 - f10)) * K.inv_dy;
            }
        }
    }
}

template <typename R, bool kGrad, typename T, class S>
GCB_HD void yee_fetch(const GlobalAcc<T>& acc, int ia, int ib, int ja,
                                          int jb, const R wx[2], const R wy[2],
                                          const Consts<R>& K, S& s) {
    typename GlobalAcc<T>::Loc g;
    acc.locate(ia, ib, ja, jb, g);
    interp_yee<R, kGrad>(GlobalLoad<T>{g}, wx, wy, K, s);
}

template <typename R, bool kGrad, typename T, class S>
GCB_HD void yee_fetch(const TileAcc<T>& acc, int ia, int ib, int ja,
                                          int jb, const R wx[2], const R wy[2],
                                          const Consts<R>& K, S& s) {
    int off[4];
    typename GlobalAcc<T>::Loc g;
    if (acc.locate(ia, ib, ja, jb, off, g))
        interp_yee<R, kGrad>(LdsLoad<T>{acc.lds, off, acc.W, acc.W * acc.W}, wx, wy, K, s);
    else
        interp_yee<R, kGrad>(GlobalLoad<T>{g}, wx, wy, K, s);
}

// the gather at lattice coordinates (gx, gy) = (X/dx, Y/dy)
template <typename R, bool kGrad, bool kYee, class Acc, class S>
GCB_HD void gather_at(const Acc& acc, const PushConst& pc, const Consts<R>& K, double gx,
                      double gy, S& s) {
    if constexpr (kYee) {
        // lattice coordinate minus the offset: offset 0 leaves it unchanged
        const double xb = gx - 0.5;
        const double yb = gy - 0.5;
        const double fxa = floor(gx), fxb = floor(xb);
        const double fya = floor(gy), fyb = floor(yb);
        const R wx[2] = {(R)(gx - fxa), (R)(xb - fxb)};
        const R wy[2] = {(R)(gy - fya), (R)(yb - fyb)};
        yee_fetch<R, kGrad>(acc, (int)fxa, (int)fxb, (int)fya, (int)fyb, wx, wy, K, s);
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if constexpr (S::kGradE) {
                interp_comp<R, true>(acc, k, gx, gy, pc.stagger[k][0], pc.stagger[k][1], K,
                                     s.E[k], s.dEx[k], s.dEy[k]);
            } else {
                R d0, d1;
                interp_comp<R, false>(acc, k, gx, gy, pc.stagger[k][0], pc.stagger[k][1], K,
                                      s.E[k], d0, d1);
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
            interp_comp<R, kGrad>(acc, k + 3, gx, gy, pc.stagger[k + 3][0],
                                  pc.stagger[k + 3][1], K, s.B[k], s.dBx[k], s.dBy[k]);
    }
}

// All six components at (X, Y); B gradients when kGrad.  kYee: the 2D Yee
// offsets (the values of the runtime table when it holds them).  Lattice
// coordinates and weights are formed in binary64 from the binary64 position.
// A point whose lattice coordinates are NaN or of magnitude kFarLattice or
// more (a fixed-point iteration that ran away) has an all-NaN sample: it is
// gathered at the origin instead, so that every node index stays a small
// integer, and the values are replaced afterwards.
template <typename R, bool kGrad, bool kYee, class Acc, class S>
GCB_HD void gather(const Acc& acc, const PushConst& pc,
                                       const Consts<R>& K, double X, double Y, S& s) {
    double gx = X * pc.inv_dx;
    double gy = Y * pc.inv_dy;
    const bool far = !(fabs(gx) < kFarLattice && fabs(gy) < kFarLattice);
    if (__builtin_expect(far, 0)) {
        gx = 0.0;
        gy = 0.0;
    }
    gather_at<R, kGrad, kYee>(acc, pc, K, gx, gy, s);
    if (__builtin_expect(far, 0)) {
        const R q = (R)__builtin_nan("");
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            s.E[i] = q;
            s.B[i] = q;
            s.dBx[i] = q;
            s.dBy[i] = q;
            if constexpr (S::kGradE) {
                s.dEx[i] = q;
                s.dEy[i] = q;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Local guiding-center quantities (Sec. 2.2): b, v_E = c E x B / B^2,
// kappa = (1 - v_E^2/c^2)^(-1/2), E_par, d_j b_i by the chain rule,
// (b.grad)b, (v_E.grad)b, A = v_E.(b.grad)b, C = v_E.(v_E.grad)b.

template <typename R>
struct Local {
    R B, inv_B;
    R b[3], vE[3];
    R kappa, Epar;
    R inv_kappa;   // production form only: sqrt(1 - v_E^2/c^2)
    R bgb[3], vgb[3];
    R A, C;
    R gB[3];   // grad|B| (the 2D step fills x, y)
};

// b, v_E, kappa and E_par from E and B at the point.
template <typename R>
GCB_HD uint32_t local_fields(const R E[3], const R Bv[3], const Consts<R>& K, Local<R>& L) {
    uint32_t flags = 0;
    const R Ex = E[0], Ey = E[1], Ez = E[2];
    const R Bx = Bv[0], By = Bv[1], Bz = Bv[2];
    const R B2 = (Bx * Bx + By * By) + Bz * Bz;
    R B, inv_B;
    bool bzero;
    if constexpr (kFastD<R>) {
        // B^2 = 0 gives B = 1/B = 0, NaN stays NaN, as in the exact form
        bzero = B2 == (R)0;
        inv_B = B2 > (R)0 ? rsqrt_nr(B2) : (bzero ? (R)0 : B2);
        B = B2 * inv_B;
    } else {
        B = sqrt(B2);
        bzero = (B == (R)0);
        inv_B = bzero ? (R)0 : (R)1 / B;
    }
    if (bzero) flags |= ST_BZERO;
    L.B = B;
    L.inv_B = inv_B;
    const R bx = Bx * inv_B, by = By * inv_B, bz = Bz * inv_B;
    L.b[0] = bx; L.b[1] = by; L.b[2] = bz;
    const R sc = K.c * (inv_B * inv_B);
    const R vEx = sc * (Ey * Bz - Ez * By);
    const R vEy = sc * (Ez * Bx - Ex * Bz);
    const R vEz = sc * (Ex * By - Ey * Bx);
    L.vE[0] = vEx; L.vE[1] = vEy; L.vE[2] = vEz;
    const R vE2 = (vEx * vEx + vEy * vEy) + vEz * vEz;
    if constexpr (kMixed<R>) {
        double om;
        if (vE2 * K.inv_c2 > 0.81f && !bzero) {
            // E/B > 0.9: 1 - v_E^2/c^2 = ((B^2 - E^2) B^2 + (E.B)^2) / B^4 in binary64
            const double ex = Ex, ey = Ey, ez = Ez, qx = Bx, qy = By, qz = Bz;
            const double b2 = (qx * qx + qy * qy) + qz * qz;
            const double e2 = (ex * ex + ey * ey) + ez * ez;
            const double eb = (ex * qx + ey * qy) + ez * qz;
            om = ((b2 - e2) * b2 + eb * eb) / (b2 * b2);
        } else {
            om = (double)((R)1 - vE2 * K.inv_c2);
        }
        if (om < kKappaFloor) {
            om = kKappaFloor;
            flags |= ST_KAPPA;
        }
        L.kappa = (R)(1.0 / sqrt(om));
    } else {
        R om = (R)1 - vE2 * K.inv_c2;
        if (om < (R)kKappaFloor) {
            om = (R)kKappaFloor;
            flags |= ST_KAPPA;
        }
        if constexpr (kFastD<R>) {
            const R k = rsqrt_nr(om);
            L.kappa = k;
            L.inv_kappa = om * k;
        } else {
            L.kappa = (R)1 / sqrt(om);
        }
    }
    L.Epar = (Ex * bx + Ey * by) + Ez * bz;
    return flags;
}

// d_j b_i = (d_j B_i - b_i (b . d_j B)) / B for one direction j, from the
// gradient dB[i] = d_j B_i; returns d_j|B| = b . d_j B.
template <typename R>
GCB_HD R db_along(const Local<R>& L, const R dB[3], R db[3]) {
    const R dn = (L.b[0] * dB[0] + L.b[1] * dB[1]) + L.b[2] * dB[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) db[i] = (dB[i] - L.b[i] * dn) * L.inv_B;
    return dn;
}

// A = v_E.(b.grad)b and C = v_E.(v_E.grad)b from L.bgb and L.vgb.
template <typename R>
GCB_HD void curvature_scalars(Local<R>& L) {
    L.A = (L.vE[0] * L.bgb[0] + L.vE[1] * L.bgb[1]) + L.vE[2] * L.bgb[2];
    L.C = (L.vE[0] * L.vgb[0] + L.vE[1] * L.vgb[1]) + L.vE[2] * L.vgb[2];
}

// 2D: gradients along x and y only.
template <typename R>
GCB_HD uint32_t local_from_sample(const Sample<R>& s, const Consts<R>& K, Local<R>& L) {
    const uint32_t flags = local_fields(s.E, s.B, K, L);
    R dbx[3], dby[3];
    L.gB[0] = db_along(L, s.dBx, dbx);
    L.gB[1] = db_along(L, s.dBy, dby);
    L.gB[2] = (R)0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        L.bgb[i] = L.b[0] * dbx[i] + L.b[1] * dby[i];
        L.vgb[i] = L.vE[0] * dbx[i] + L.vE[1] * dby[i];
    }
    curvature_scalars(L);
    return flags;
}

// The exact frame of Sec. 2.2: the frame moving with v_E in which E and B
// are parallel.  With s = sqrt(1 - 4 w_E^2/c^2), w_E = c E x B/(E^2 + B^2):
// v_E = 2 w_E/(1 + s) (the paper's w_E (1 - s)/(2 w_E^2/c^2) without its
// 0/0), B' = sqrt((B^2 - E^2 + (E^2 + B^2) s)/2), E' = E.B/B',
// Psi = 2 E' B^2/(B' (E^2 + B^2)(1 + s)) (equal to E'(B^2 - B'^2)/(B' E_perp^2)),
// eta = 1/(B sqrt(Psi^2 E_perp^2/B^2 + 1)), b* = eta (Psi E_perp + B).
// Fills L with b = b*, the exact v_E and kappa, and E_par = E'/kappa (the
// parallel force in the moving frame, its clock slowed by kappa); the lab B
// stays in L.B.  The curvature terms are left at zero here: the
// zero-curvature scheme (Sec. 2.2.1) needs none, and local_exact_curv adds
// them for the curvature scheme.
template <typename R>
GCB_HD uint32_t local_fields_exact(const R E[3], const R Bv[3], const Consts<R>& K,
                                   Local<R>& L) {
    uint32_t flags = 0;
    const R Ex = E[0], Ey = E[1], Ez = E[2];
    const R Bx = Bv[0], By = Bv[1], Bz = Bv[2];
    const R E2 = (Ex * Ex + Ey * Ey) + Ez * Ez;
    const R B2 = (Bx * Bx + By * By) + Bz * Bz;
    const R EB = (Ex * Bx + Ey * By) + Ez * Bz;
    const R S = E2 + B2;
    const R B = sqrt(B2);
    const bool bzero = (B == (R)0);
    const R inv_B = bzero ? (R)0 : (R)1 / B;
    if (bzero) flags |= ST_BZERO;
    L.B = B;
    L.inv_B = inv_B;
    const R f = (S == (R)0) ? (R)0 : K.c / S;
    const R wx = f * (Ey * Bz - Ez * By);
    const R wy = f * (Ez * Bx - Ex * Bz);
    const R wz = f * (Ex * By - Ey * Bx);
    const R w2 = (wx * wx + wy * wy) + wz * wz;
    const R s_arg = (R)1 - ((R)4 * w2) * K.inv_c2;
    const R s = sqrt(s_arg > (R)0 ? s_arg : (R)0);
    const R g = (R)2 / ((R)1 + s);
    const R vEx = g * wx, vEy = g * wy, vEz = g * wz;
    L.vE[0] = vEx; L.vE[1] = vEy; L.vE[2] = vEz;
    const R vE2 = (vEx * vEx + vEy * vEy) + vEz * vEz;
    R om = (R)1 - vE2 * K.inv_c2;
    if (om < (R)kKappaFloor) {
        om = (R)kKappaFloor;
        flags |= ST_KAPPA;
    }
    const R kappa = (R)1 / sqrt(om);
    L.kappa = kappa;
    if constexpr (kFastD<R>) L.inv_kappa = (R)1 / kappa;
    const R Bp2 = (R)0.5 * ((B2 - E2) + S * s);
    const R Bp = sqrt(Bp2 > (R)0 ? Bp2 : (R)0);
    const bool bpzero = (Bp == (R)0);
    const R Ep = bpzero ? (R)0 : EB / Bp;
    const R a = bzero ? (R)0 : EB / B2;
    const R epx = Ex - a * Bx, epy = Ey - a * By, epz = Ez - a * Bz;
    const R Eperp2 = (epx * epx + epy * epy) + epz * epz;
    const R Psi = bpzero ? (R)0 : (((R)2 * Ep) * B2) / ((Bp * S) * ((R)1 + s));
    const R q = bzero ? (R)0 : ((Psi * Psi) * Eperp2) / B2;
    const R eta = bzero ? (R)0 : (R)1 / (B * sqrt(q + (R)1));
    const R xi = eta * Psi;
    L.b[0] = xi * epx + eta * Bx;
    L.b[1] = xi * epy + eta * By;
    L.b[2] = xi * epz + eta * Bz;
    L.Epar = Ep / kappa;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        L.bgb[i] = (R)0;
        L.vgb[i] = (R)0;
    }
    L.A = (R)0;
    L.C = (R)0;
    return flags;
}

// A value with its derivatives along nd directions (forward-mode
// differentiation): the gradient of b* is carried through the arithmetic of
// the frame by the chain rule, one operation at a time.
template <typename R, int nd>
struct Dual {
    R v;
    R d[nd];
};

template <typename R, int nd>
GCB_HD Dual<R, nd> dconst(R a) {
    Dual<R, nd> r;
    r.v = a;
#pragma unroll
    for (int j = 0; j < nd; ++j) r.d[j] = (R)0;
    return r;
}
template <typename R, int nd>
GCB_HD Dual<R, nd> operator+(const Dual<R, nd>& a, const Dual<R, nd>& b) {
    Dual<R, nd> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int j = 0; j < nd; ++j) r.d[j] = a.d[j] + b.d[j];
    return r;
}
template <typename R, int nd>
GCB_HD Dual<R, nd> operator-(const Dual<R, nd>& a, const Dual<R, nd>& b) {
    Dual<R, nd> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int j = 0; j < nd; ++j) r.d[j] = a.d[j] - b.d[j];
    return r;
}
template <typename R, int nd>
GCB_HD Dual<R, nd> operator*(const Dual<R, nd>& a, const Dual<R, nd>& b) {
    Dual<R, nd> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int j = 0; j < nd; ++j) r.d[j] = a.d[j] * b.v + a.v * b.d[j];
    return r;
}
template <typename R, int nd>
GCB_HD Dual<R, nd> operator*(R a, const Dual<R, nd>& b) {
    Dual<R, nd> r;
    r.v = a * b.v;
#pragma unroll
    for (int j = 0; j < nd; ++j) r.d[j] = a * b.d[j];
    return r;
}
// (a/b)' = (a' - (a/b) b')/b
template <typename R, int nd>
GCB_HD Dual<R, nd> operator/(const Dual<R, nd>& a, const Dual<R, nd>& b) {
    Dual<R, nd> r;
    r.v = a.v / b.v;
#pragma unroll
    for (int j = 0; j < nd; ++j) r.d[j] = (a.d[j] - r.v * b.d[j]) / b.v;
    return r;
}
// sqrt(a)' = a'/(2 sqrt(a)); a derivative of 0 where the root is 0 (the
// frame takes the root of a clamped argument there)
template <typename R, int nd>
GCB_HD Dual<R, nd> dsqrt(const Dual<R, nd>& a) {
    Dual<R, nd> r;
    r.v = sqrt(a.v);
    const R f = r.v > (R)0 ? (R)0.5 / r.v : (R)0;
#pragma unroll
    for (int j = 0; j < nd; ++j) r.d[j] = a.d[j] * f;
    return r;
}

// b* of the exact frame (the operations of local_fields_exact, the same
// selects) on values carrying their spatial derivatives: gives d_j b*_i.
template <typename R, int nd>
GCB_HD void bstar_dual(const Dual<R, nd> E[3], const Dual<R, nd> Bv[3], const Consts<R>& K,
                       Dual<R, nd> b[3]) {
    using D = Dual<R, nd>;
    const D zero = dconst<R, nd>((R)0);
    const D E2 = (E[0] * E[0] + E[1] * E[1]) + E[2] * E[2];
    const D B2 = (Bv[0] * Bv[0] + Bv[1] * Bv[1]) + Bv[2] * Bv[2];
    const D EB = (E[0] * Bv[0] + E[1] * Bv[1]) + E[2] * Bv[2];
    const D S = E2 + B2;
    const D B = dsqrt(B2);
    const bool bzero = B.v == (R)0;
    const D f = S.v == (R)0 ? zero : dconst<R, nd>(K.c) / S;
    const D w[3] = {f * (E[1] * Bv[2] - E[2] * Bv[1]), f * (E[2] * Bv[0] - E[0] * Bv[2]),
                    f * (E[0] * Bv[1] - E[1] * Bv[0])};
    const D w2 = (w[0] * w[0] + w[1] * w[1]) + w[2] * w[2];
    const D s_arg = dconst<R, nd>((R)1) - K.inv_c2 * ((R)4 * w2);
    const D s = s_arg.v > (R)0 ? dsqrt(s_arg) : zero;
    const D Bp2 = (R)0.5 * ((B2 - E2) + S * s);
    const D Bp = Bp2.v > (R)0 ? dsqrt(Bp2) : zero;
    const bool bpzero = Bp.v == (R)0;
    const D Ep = bpzero ? zero : EB / Bp;
    const D a = bzero ? zero : EB / B2;
    const D ep[3] = {E[0] - a * Bv[0], E[1] - a * Bv[1], E[2] - a * Bv[2]};
    const D Eperp2 = (ep[0] * ep[0] + ep[1] * ep[1]) + ep[2] * ep[2];
    const D one = dconst<R, nd>((R)1);
    const D Psi = bpzero ? zero : ((R)2 * Ep * B2) / ((Bp * S) * (one + s));
    const D q = bzero ? zero : ((Psi * Psi) * Eperp2) / B2;
    const D eta = bzero ? zero : one / (B * dsqrt(q + one));
    const D xi = eta * Psi;
#pragma unroll
    for (int i = 0; i < 3; ++i) b[i] = xi * ep[i] + eta * Bv[i];
}

// The exact frame with the curvature scheme (Sec. 2.2 with Sec. 2.2.2):
// the values of local_fields_exact, and (b*.grad)b*, (v_E.grad)b*, A, C
// from d_j b*, carried by forward-mode differentiation from the gather's E
// and B gradients (2D: j = x, y).
template <typename R>
GCB_HD uint32_t local_exact_curv(const SampleEG<R>& s, const Consts<R>& K, Local<R>& L) {
    const uint32_t flags = local_fields_exact(s.E, s.B, K, L);
    Dual<R, 2> E[3], Bv[3], b[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        E[i].v = s.E[i];
        E[i].d[0] = s.dEx[i];
        E[i].d[1] = s.dEy[i];
        Bv[i].v = s.B[i];
        Bv[i].d[0] = s.dBx[i];
        Bv[i].d[1] = s.dBy[i];
    }
    bstar_dual<R, 2>(E, Bv, K, b);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        L.bgb[i] = L.b[0] * b[i].d[0] + L.b[1] * b[i].d[1];
        L.vgb[i] = L.vE[0] * b[i].d[0] + L.vE[1] * b[i].d[1];
        L.gB[i] = (R)0;
    }
    curvature_scalars(L);
    return flags;
}

// the local quantities of the guiding-center step in the chosen frame (any
// sample type with E and B; the reduced frame's gradients come from it, the
// exact frame's curvature terms from a sample with the E gradients)
template <bool kExact, typename R, class S>
GCB_HD uint32_t local_in_frame(const S& s, const Consts<R>& K, Local<R>& L) {
    if constexpr (kExact && S::kGradE)
        return local_exact_curv(s, K, L);
    else if constexpr (kExact)
        return local_fields_exact(s.E, s.B, K, L);
    else
        return local_from_sample(s, K, L);
}

// Gyration state of a guiding-center step (Sec. 2.2): mu/m, conserved
// (eq. dmudt), or, with `fixed`, u_perp_g^2 held at its decomposed value
// over the step (the energy-conserving alternative of Sec. 2.2).  mu = 0 is
// the state of a step that discards the gyration.
template <typename R>
struct Gyr {
    R mu;
    R up2;
    bool fixed;
};

// u_perp_g^2 at a point: 2 mu B kappa/m, or the held value
template <typename R>
GCB_HD R uperp_sq(const Local<R>& L, const Gyr<R>& g) {
    return g.fixed ? g.up2 : (((R)2 * g.mu) * L.B) * L.kappa;
}

// Gamma(R, u_par) = kappa sqrt(1 + (u_par^2 + 2 mu B kappa/m)/c^2)  (eq. lfacgca2)
template <typename R>
GCB_HD R gamma_gca(const Local<R>& L, R upar, const Gyr<R>& gy, const Consts<R>& K) {
    const R uperp2 = uperp_sq(L, gy);
    const R arg = (R)1 + (upar * upar + uperp2) * K.inv_c2;
    if constexpr (kMixed<R>) {
        if (arg > 1.0e6f) {   // ultra-relativistic: binary64
            const double a = 1.0 + ((double)upar * (double)upar + (double)uperp2) *
                                       (1.0 / ((double)K.c * (double)K.c));
            return (R)((double)L.kappa * sqrt(a));
        }
    }
    return L.kappa * sqrt(arg);
}

// Gamma(R, u_par) (eq. lfacgca2) and, in the production form, 1/Gamma from
// one reciprocal square root
template <typename R>
GCB_HD Gam<R> gamma_gca2(const Local<R>& L, R upar, const Gyr<R>& gy, const Consts<R>& K) {
    if constexpr (kFastD<R>) {
        const R arg = (R)1 + (upar * upar + uperp_sq(L, gy)) * K.inv_c2;
        const R s = rsqrt_nr(arg);
        return {L.kappa * (arg * s), s * L.inv_kappa};
    } else {
        return {gamma_gca(L, upar, gy, K), (R)0};
    }
}

// Curvature drift (eq. curvdrift):
// (m c kappa^2 / (q B)) b x [ (u_par^2/Gamma)(b.grad)b + u_par (v_E.grad)b ]
template <typename R>
GCB_HD void v_curv(const Local<R>& L, R upar, R gam, R inv_qm,
                                       const Consts<R>& K, R vc[3]) {
    const R pre = ((K.c * L.kappa) * L.kappa) * (L.inv_B * inv_qm);
    const R a1 = (upar * upar) / gam;
    const R w0 = a1 * L.bgb[0] + upar * L.vgb[0];
    const R w1 = a1 * L.bgb[1] + upar * L.vgb[1];
    const R w2 = a1 * L.bgb[2] + upar * L.vgb[2];
    vc[0] = pre * (L.b[1] * w2 - L.b[2] * w1);
    vc[1] = pre * (L.b[2] * w0 - L.b[0] * w2);
    vc[2] = pre * (L.b[0] * w1 - L.b[1] * w0);
}

// The curvature drift with Gamma and its reciprocal: the same arithmetic, the
// division by Gamma a multiplication in the production form.
template <typename R>
GCB_HD void v_curv_g(const Local<R>& L, R upar, const Gam<R>& G, R inv_qm,
                     const Consts<R>& K, R vc[3]) {
    if constexpr (kFastD<R>) {
        const R pre = ((K.c * L.kappa) * L.kappa) * (L.inv_B * inv_qm);
        const R a1 = (upar * upar) * G.inv;
        const R w0 = a1 * L.bgb[0] + upar * L.vgb[0];
        const R w1 = a1 * L.bgb[1] + upar * L.vgb[1];
        const R w2 = a1 * L.bgb[2] + upar * L.vgb[2];
        vc[0] = pre * (L.b[1] * w2 - L.b[2] * w1);
        vc[1] = pre * (L.b[2] * w0 - L.b[0] * w2);
        vc[2] = pre * (L.b[0] * w1 - L.b[1] * w0);
    } else {
        v_curv(L, upar, G.g, inv_qm, K, vc);
    }
}

// Curvature drift with the grad-B drift in its bracket (the mirror option):
// (m c kappa^2/(q B)) b x [ (u_par^2/Gamma)(b.grad)b + u_par (v_E.grad)b
//                           + (mu/(m kappa Gamma)) grad|B| ]
// with grad(B/kappa) taken as grad|B|/kappa; kND gradient components (2 or 3).
template <int kND, typename R>
GCB_HD void v_curv_mirror(const Local<R>& L, R upar, R gam, R inv_qm, R mu,
                          const Consts<R>& K, R vc[3]) {
    const R pre = ((K.c * L.kappa) * L.kappa) * (L.inv_B * inv_qm);
    const R a1 = (upar * upar) / gam;
    R w[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) w[i] = a1 * L.bgb[i] + upar * L.vgb[i];
    const R a3 = (mu / L.kappa) / gam;
#pragma unroll
    for (int i = 0; i < kND; ++i) w[i] = w[i] + a3 * L.gB[i];
    vc[0] = pre * (L.b[1] * w[2] - L.b[2] * w[1]);
    vc[1] = pre * (L.b[2] * w[0] - L.b[0] * w[2]);
    vc[2] = pre * (L.b[0] * w[1] - L.b[1] * w[0]);
}

// Lorentz factor of the full four-velocity
template <typename R>
GCB_HD R gamma_full(R ux, R uy, R uz, const Consts<R>& K) {
    const R arg = (R)1 + ((ux * ux + uy * uy) + uz * uz) * K.inv_c2;
    if constexpr (kMixed<R>) {
        if (arg > 1.0e6f) {
            const double a = 1.0 + (((double)ux * ux + (double)uy * uy) + (double)uz * uz) *
                                       (1.0 / ((double)K.c * (double)K.c));
            return (R)sqrt(a);
        }
    }
    return sqrt(arg);
}

// the Lorentz factor of the full four-velocity and, in the production form,
// its reciprocal
template <typename R>
GCB_HD Gam<R> gamma_full2(R ux, R uy, R uz, const Consts<R>& K) {
    if constexpr (kFastD<R>) {
        const R arg = (R)1 + ((ux * ux + uy * uy) + uz * uz) * K.inv_c2;
        const R s = rsqrt_nr(arg);
        return {arg * s, s};
    } else {
        return {gamma_full(ux, uy, uz, K), (R)0};
    }
}

// ---------------------------------------------------------------------------
// Switch (Sec. 3 criteria, Sec. 4.1): guiding center iff B > 0,
// rho~/dl < f_rho and E/B < f_E, with rho~ = c^2 Gamma / (|q/m| B).

GCB_HD bool switch_gca_f64(const double E[3], const double Bv[3],
                                               double ux, double uy, double uz, double qm,
                                               const PushConst& pc) {
    const double B = sqrt((Bv[0] * Bv[0] + Bv[1] * Bv[1]) + Bv[2] * Bv[2]);
    const double E_ = sqrt((E[0] * E[0] + E[1] * E[1]) + E[2] * E[2]);
    const bool pos = B > 0.0;
    const double inv_B = pos ? 1.0 / B : 0.0;
    const double gf = sqrt(1.0 + ((ux * ux + uy * uy) + uz * uz) * pc.inv_c2);
    const double inv_absqm = fabs(1.0 / qm);
    const double rho = ((pc.c2 * gf) * inv_B) * inv_absqm;
    return pos && (rho * pc.inv_dl < pc.f_rho) && (E_ * inv_B < pc.f_E);
}

template <typename R>
GCB_HD bool switch_gca(const R E[3], const R Bv[3], R ux, R uy, R uz,
                                           double qm, const PushConst& pc,
                                           const Consts<R>& K) {
    if constexpr (!kMixed<R>) {
        return switch_gca_f64(E, Bv, ux, uy, uz, qm, pc);
    } else {
        const R B = sqrt((Bv[0] * Bv[0] + Bv[1] * Bv[1]) + Bv[2] * Bv[2]);
        const R E_ = sqrt((E[0] * E[0] + E[1] * E[1]) + E[2] * E[2]);
        const bool pos = B > (R)0;
        const R inv_B = pos ? (R)1 / B : (R)0;
        const R gf = gamma_full(ux, uy, uz, K);
        const R inv_absqm = fabs((R)1 / (R)qm);
        const R rr = (((K.c2 * gf) * inv_B) * inv_absqm) * K.inv_dl;
        const R er = E_ * inv_B;
        // near a threshold the test is repeated in binary64
        const bool near = fabs(rr - K.f_rho) <= 1.0e-4f * K.f_rho ||
                          fabs(er - K.f_E) <= 1.0e-4f * K.f_E;
        if (near) {
            const double Ed[3] = {E[0], E[1], E[2]};
            const double Bd[3] = {Bv[0], Bv[1], Bv[2]};
            return switch_gca_f64(Ed, Bd, ux, uy, uz, qm, pc);
        }
        return pos && (rr < K.f_rho) && (er < K.f_E);
    }
}

// ---------------------------------------------------------------------------
// Periodic box (binary64)

GCB_HD double wrap(double x, double L) {
    double w = x - L * floor(x / L);
    if (w < 0.0) w = w + L;
    if (w >= L) w = w - L;
    return w;
}

GCB_HD double min_image(double d, double L) {
    return d - L * floor(d / L + 0.5);
}

// the same with 1/L given: the division becomes a multiplication in the
// production form
template <typename R>
GCB_HD double wrap_i(double x, double L, double inv_L) {
    if constexpr (kFastD<R>) {
        double w = x - L * floor(x * inv_L);
        if (w < 0.0) w = w + L;
        if (w >= L) w = w - L;
        return w;
    } else {
        return wrap(x, L);
    }
}

template <typename R>
GCB_HD double min_image_i(double d, double L, double inv_L) {
    if constexpr (kFastD<R>)
        return d - L * floor(d * inv_L + 0.5);
    else
        return min_image(d, L);
}

// ---------------------------------------------------------------------------
// Relativistic Boris push (Sec. 2.1), fields at x^n

template <typename R>
GCB_HD void boris(const R E[3], const R Bv[3], R& ux, R& uy, R& uz,
                                      R qm, const Consts<R>& K) {
    const R hq = (qm * K.dt) * (R)0.5;
    const R umx = ux + hq * E[0], umy = uy + hq * E[1], umz = uz + hq * E[2];
    const R gm = gamma_full(umx, umy, umz, K);
    const R f = hq / (K.c * gm);
    const R tx = f * Bv[0], ty = f * Bv[1], tz = f * Bv[2];
    const R t2 = (tx * tx + ty * ty) + tz * tz;
    const R g = (R)2 / ((R)1 + t2);
    const R sx = g * tx, sy = g * ty, sz = g * tz;
    const R upx = umx + (umy * tz - umz * ty);
    const R upy = umy + (umz * tx - umx * tz);
    const R upz = umz + (umx * ty - umy * tx);
    const R uqx = umx + (upy * sz - upz * sy);
    const R uqy = umy + (upz * sx - upx * sz);
    const R uqz = umz + (upx * sy - upy * sx);
    ux = uqx + hq * E[0];
    uy = uqy + hq * E[1];
    uz = uqz + hq * E[2];
}

// Full-orbit step: u^{n-1/2} -> u^{n+1/2}, x^{n+1} = x^n + dt u/Gamma.
template <typename R>
GCB_HD void boris_step(const Sample<R>& s, Regs<R>& r, const PushConst& pc,
                                           const Consts<R>& K) {
    boris(s.E, s.B, r.ux, r.uy, r.uz, (R)r.qm, K);
    R inv_g;
    if constexpr (kFastD<R>) {
        inv_g = gamma_full2(r.ux, r.uy, r.uz, K).inv;
    } else {
        const R gn = gamma_full(r.ux, r.uy, r.uz, K);
        inv_g = (R)1 / gn;
    }
    const double xn = r.x + pc.dt * (double)(r.ux * inv_g);
    const double yn = r.y + pc.dt * (double)(r.uy * inv_g);
    r.xp = r.x;
    r.yp = r.y;
    r.x = wrap_i<R>(xn, pc.Lx, pc.inv_Lx);
    r.y = wrap_i<R>(yn, pc.Ly, pc.inv_Ly);
}

// ---------------------------------------------------------------------------
// Guiding-center leapfrog (Sec. 2.2.1 / 2.2.2) inside the coupled step (Sec. 3.1)

// u_par^{n-1/2} -> u_par^{n+1/2} at R^n.  With curvature: the positive root
// of k1 G^2 + k2 G + k3 = 0 for G = Gamma(R^n, u_par^{n+1/2}), evaluated
// without cancellation, then eq. dupardtcase2discsol.  With `shifted`, the
// explicit change `shift` (the mirror force over the step) is subtracted
// from the known part of the update.
template <typename R>
GCB_HD R parallel_update(const Local<R>& Ln, R upar, const Gyr<R>& gy, R qm,
                                             bool curvature, const Consts<R>& K,
                                             uint32_t& flags, bool shifted = false,
                                             R shift = (R)0) {
    const R dtqm = qm * K.dt;
    if (!curvature) return upar + dtqm * Ln.Epar;
    const R h = K.h;
    const R A = Ln.A, C = Ln.C;
    const R G0 = gamma_gca2(Ln, upar, gy, K).g;
    R upr = (upar * ((R)1 + h * A) + dtqm * Ln.Epar) + (h * G0) * C;
    if (shifted) upr = upr - shift;
    const R D = (R)1 - h * A;
    const R DD = D * D;
    R k1;
    if constexpr (kFastD<R>)
        k1 = (h * h) * (C * C) - (K.c2 * DD) * (Ln.inv_kappa * Ln.inv_kappa);
    else
        k1 = (h * h) * (C * C) - (K.c2 * DD) / (Ln.kappa * Ln.kappa);
    const R k2 = (upr * K.dt) * C;
    const R k3 = upr * upr + (K.c2 + uperp_sq(Ln, gy)) * DD;
    const R disc = k2 * k2 - ((R)4 * k1) * k3;
    const bool dok = fabs(D) >= (R)kDFloor;
    bool ok = (k1 < (R)0) && (disc >= (R)0) && dok;
    const R sq = sqrt(disc >= (R)0 ? disc : (R)0);
    const bool pos_k2 = k2 >= (R)0;
    const R num = pos_k2 ? k2 + sq : (R)2 * k3;
    R den = pos_k2 ? (R)(-2) * k1 : sq - k2;
    den = (ok && den > (R)0) ? den : (R)1;
    const R gp = num / den;
    ok = ok && (gp > (R)0) && __builtin_isfinite(gp);
    const R Ds = dok ? D : (R)1;
    if (ok) return (upr + (h * gp) * C) / Ds;
    flags |= ST_QUAD;
    if (dok) {
        const R gfb = gamma_gca(Ln, upr / Ds, gy, K);
        return (upr + (h * gfb) * C) / Ds;
    }
    const R uexp = upar + dtqm * Ln.Epar;
    return shifted ? uexp - shift : uexp;
}

// The parallel update with the mirror force -(mu/(m kappa Gamma)) b.grad|B|
// (the mirror option), Gamma centred by one predictor-corrector pass: the
// predictor takes 1/Gamma(R^n, u_par^{n-1/2}), the corrector the mean of that
// and 1/Gamma(R^n, u_par*) at the predictor's result u_par*.  Flags of both
// passes are kept.  kND gradient components (2 or 3).
template <int kND, typename R>
GCB_HD R mirror_parallel(const Local<R>& Ln, R upar, const Gyr<R>& gy, R qm,
                         const Consts<R>& K, uint32_t& flags) {
    R M = Ln.b[0] * Ln.gB[0] + Ln.b[1] * Ln.gB[1];
    if constexpr (kND == 3) M = M + Ln.b[2] * Ln.gB[2];
    const R ds = (K.dt * (gy.mu / Ln.kappa)) * M;
    const R G0 = gamma_gca(Ln, upar, gy, K);
    const R u1 = parallel_update(Ln, upar, gy, qm, true, K, flags, true, ds / G0);
    const R G1 = gamma_gca(Ln, u1, gy, K);
    return parallel_update(Ln, upar, gy, qm, true, K, flags, true,
                           ds * ((R)0.5 * ((R)1 / G0 + (R)1 / G1)));
}

// x, y components of u_par b / Gamma + v_E + v_c at a point (v_c with the
// grad-B drift under the mirror option).
template <typename R>
GCB_HD void drift_terms(const Local<R>& L, R upn, const Gyr<R>& gy, R inv_qm,
                                            bool curvature, const Consts<R>& K, R& Fx,
                                            R& Fy, bool mirror = false) {
    const Gam<R> G = gamma_gca2(L, upn, gy, K);
    const R a = over(upn, G);
    if (curvature) {
        R vc[3];
        if (mirror)
            v_curv_mirror<2>(L, upn, G.g, inv_qm, gy.mu, K, vc);
        else
            v_curv_g(L, upn, G, inv_qm, K, vc);
        Fx = (a * L.b[0] + L.vE[0]) + vc[0];
        Fy = (a * L.b[1] + L.vE[1]) + vc[1];
    } else {
        Fx = a * L.b[0] + L.vE[0];
        Fy = a * L.b[1] + L.vE[1];
    }
}

// The check of the neglect of the mirror terms (Sec. 2.2): ST_MIRROR where
// (v_perp_g/c)^2 = u_perp_g^2/(Gamma^2 c^2) exceeds pc.mirror_tol (> 0) at
// the decomposition, Gamma of the full four-velocity.  up2 and gf come from
// the decomposition of u (ux, uy, uz) with the local quantities Lh and the
// curvature drift vc there.  In the mixed form a comparison within 1e-4 of
// the threshold is taken again in binary64 (the decomposition redone in
// binary64 from the same binary32 inputs), as the switch test is.
template <typename R>
GCB_HD uint32_t mirror_check(R ux, R uy, R uz, const Local<R>& Lh, const R vc[3], R up2, R gf,
                             const PushConst& pc, const Consts<R>& K) {
    if (!(pc.mirror_tol > 0.0)) return 0u;
    const R lhs = up2 * K.inv_c2;
    const R rhs = (R)pc.mirror_tol * (gf * gf);
    if constexpr (kMixed<R>) {
        if (fabs(lhs - rhs) <= 1.0e-4f * rhs) {
            const double u[3] = {ux, uy, uz};
            const double b[3] = {Lh.b[0], Lh.b[1], Lh.b[2]};
            const double g = sqrt(1.0 + ((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]) * pc.inv_c2);
            const double upar = (u[0] * b[0] + u[1] * b[1]) + u[2] * b[2];
            double q = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double w = (u[i] - upar * b[i]) - ((double)Lh.vE[i] + (double)vc[i]) * g;
                q = q + w * w;
            }
            return q * pc.inv_c2 > pc.mirror_tol * (g * g) ? (uint32_t)ST_MIRROR : 0u;
        }
    }
    return lhs > rhs ? (uint32_t)ST_MIRROR : 0u;
}

// The gyro-phase option (GYR_PHASE, kernel instances of their own): the
// gyration direction d turned about b at R^n by -(q/m) B dt/(c kappa Gamma),
// Gamma of eq. lfacgca2 at R^n with the mean of u_par before and after the
// parallel update -- the gyration frequency of a particle whose guiding
// center drifts with v_E -- by Rodrigues' formula
// d cos + (b x d) sin + b (b.d)(1 - cos).
template <typename R>
GCB_HD void phase_advance(const Local<R>& Ln, R upar, R upn, const Gyr<R>& gy, R qm,
                          const Consts<R>& K, R d[3]) {
    const R gn = gamma_gca(Ln, (R)0.5 * (upar + upn), gy, K);
    const R ang = -((qm * Ln.B) * K.dt) / ((K.c * Ln.kappa) * gn);
    R sn, cs;
    sincos_poly<R>((double)ang, sn, cs);
    const R bd = (Ln.b[0] * d[0] + Ln.b[1] * d[1]) + Ln.b[2] * d[2];
    const R cx = Ln.b[1] * d[2] - Ln.b[2] * d[1];
    const R cy = Ln.b[2] * d[0] - Ln.b[0] * d[2];
    const R cz = Ln.b[0] * d[1] - Ln.b[1] * d[0];
    const R w = bd * ((R)1 - cs);
    const R d0 = (d[0] * cs + cx * sn) + Ln.b[0] * w;
    const R d1 = (d[1] * cs + cy * sn) + Ln.b[1] * w;
    const R d2 = (d[2] * cs + cz * sn) + Ln.b[2] * w;
    d[0] = d0;
    d[1] = d1;
    d[2] = d2;
}

GCB_HD double nan_max(double a, double b) {
    if (a != a) return a;
    if (b != b) return b;
    return a > b ? a : b;
}

// One guiding-center step.  sn is the gather (with gradients) at x^n.
// Returns status flags; res receives |R^K - R^{K-1}|_inf.
// kExact: the exact frame of Sec. 2.2 (with kExCurv its curvature scheme);
// kMirror: the mirror force and grad-B drift (curvature scheme only);
// kPhase: the gyration phase advanced over the step (GYR_PHASE).
template <typename R, bool kYee, bool kExact = false, bool kMirror = false, bool kPhase = false,
          bool kExCurv = false, class Acc>
GCB_HD uint32_t gca_step(const Acc& acc, const Sample<R>& sn, Regs<R>& r,
                                             const PushConst& pc, const Consts<R>& K,
                                             double& res) {
    // kExCurv: the exact frame with the curvature scheme, whose gathers carry
    // the E gradients
    static_assert(!kExCurv || kExact, "kExCurv is a form of the exact frame");
    using Smp = std::conditional_t<kExCurv, SampleEG<R>, Sample<R>>;
    uint32_t flags = 0;
    const bool curv = kExCurv || (!kExact && pc.curvature != 0);
    // the mirror terms ride on the curvature scheme (the host refuses others)
    const bool mirror = kMirror && curv;
    const double x = r.x, y = r.y;
    const R ux = r.ux, uy = r.uy, uz = r.uz;
    const R qm = (R)r.qm;
    const R inv_qm = (R)1 / qm;

    // 1. guiding-center variables at R^{n-1/2} = (x^n + x^{n-1})/2
    R upar, bpx, bpy, bpz;
    Gyr<R> gy;
    {
        const double Rhx = x - 0.5 * min_image_i<R>(x - r.xp, pc.Lx, pc.inv_Lx);
        const double Rhy = y - 0.5 * min_image_i<R>(y - r.yp, pc.Ly, pc.inv_Ly);
        Smp sh;
        gather<R, true, kYee>(acc, pc, K, Rhx, Rhy, sh);
        Local<R> Lh;
        flags |= local_in_frame<kExact>(sh, K, Lh);
        upar = (ux * Lh.b[0] + uy * Lh.b[1]) + uz * Lh.b[2];
        const Gam<R> G = gamma_full2(ux, uy, uz, K);
        const R gf = G.g;
        R vc[3] = {(R)0, (R)0, (R)0};
        if (curv) v_curv_g(Lh, upar, G, inv_qm, K, vc);
        const R upx = (ux - upar * Lh.b[0]) - (Lh.vE[0] + vc[0]) * gf;
        const R upy = (uy - upar * Lh.b[1]) - (Lh.vE[1] + vc[1]) * gf;
        const R upz = (uz - upar * Lh.b[2]) - (Lh.vE[2] + vc[2]) * gf;
        const R up2 = (upx * upx + upy * upy) + upz * upz;
        flags |= mirror_check(ux, uy, uz, Lh, vc, up2, gf, pc, K);
        R mu;
        if constexpr (kFastD<R>)
            mu = (((R)0.5 * up2) * Lh.inv_B) * Lh.inv_kappa;
        else
            mu = (((R)0.5 * up2) * Lh.inv_B) / Lh.kappa;
        gy.mu = pc.gyration == GYR_ZERO ? (R)0 : mu;
        gy.up2 = up2;
        gy.fixed = pc.gyration == GYR_UPERP;
        R inv_nu;
        if constexpr (kFastD<R>) {
            inv_nu = up2 > (R)0 ? rsqrt_nr(up2) : (R)0;
        } else {
            const R nu = sqrt(up2);
            inv_nu = nu > (R)0 ? (R)1 / nu : (R)0;
        }
        bpx = upx * inv_nu;
        bpy = upy * inv_nu;
        bpz = upz * inv_nu;
    }

    // 2.-3. local quantities at R^n = x^n and the parallel update
    R upn, Fnx, Fny;
    {
        Local<R> Ln;
        if constexpr (kExCurv) {
            SampleEG<R> se;
            gather<R, true, kYee>(acc, pc, K, x, y, se);
            flags |= local_in_frame<kExact>(se, K, Ln);
        } else {
            flags |= local_in_frame<kExact>(sn, K, Ln);
        }
        if (mirror)
            upn = mirror_parallel<2>(Ln, upar, gy, qm, K, flags);
        else
            upn = parallel_update(Ln, upar, gy, qm, curv, K, flags);
        drift_terms(Ln, upn, gy, inv_qm, curv, K, Fnx, Fny, mirror);
        if constexpr (kPhase) {
            R d[3] = {bpx, bpy, bpz};
            phase_advance(Ln, upar, upn, gy, qm, K, d);
            bpx = d[0];
            bpy = d[1];
            bpz = d[2];
        }
    }

    // 4. R^{n+1}: K fixed-point iterations R^{k+1} = R^k - H(R^k), R^0 = R^n
    //    (positions binary64, drift velocities in R)
    double Rx = x, Ry = y;
    res = 0.0;
    for (int k = 0; k < pc.n_iter; ++k) {
        R Fkx, Fky;
        if (k == 0) {
            Fkx = Fnx;
            Fky = Fny;
        } else {
            Smp sk;
            gather<R, true, kYee>(acc, pc, K, Rx, Ry, sk);
            Local<R> Lk;
            flags |= local_in_frame<kExact>(sk, K, Lk);
            drift_terms(Lk, upn, gy, inv_qm, curv, K, Fkx, Fky, mirror);
        }
        const double Rx_new = x + (double)(K.h * (Fnx + Fkx));
        const double Ry_new = y + (double)(K.h * (Fny + Fky));
        res = nan_max(fabs(Rx_new - Rx), fabs(Ry_new - Ry));
        Rx = Rx_new;
        Ry = Ry_new;
    }
    if (res > pc.fp_tol) flags |= ST_FPRES;

    // 5. particle variables at R^{n+1/2} = (R^n + R^{n+1})/2, gyration
    //    direction held fixed (or advanced, kPhase)
    {
        const double Rmx = x + 0.5 * (Rx - x);
        const double Rmy = y + 0.5 * (Ry - y);
        Smp sm;
        gather<R, true, kYee>(acc, pc, K, Rmx, Rmy, sm);
        Local<R> Lm;
        flags |= local_in_frame<kExact>(sm, K, Lm);
        const Gam<R> G = gamma_gca2(Lm, upn, gy, K);
        const R gr = G.g;
        R vc[3] = {(R)0, (R)0, (R)0};
        if (curv) v_curv_g(Lm, upn, G, inv_qm, K, vc);
        const R um = sqrt(uperp_sq(Lm, gy));
        r.ux = (upn * Lm.b[0] + (Lm.vE[0] + vc[0]) * gr) + um * bpx;
        r.uy = (upn * Lm.b[1] + (Lm.vE[1] + vc[1]) * gr) + um * bpy;
        r.uz = (upn * Lm.b[2] + (Lm.vE[2] + vc[2]) * gr) + um * bpz;
    }

    // 6. store
    r.xp = x;
    r.yp = y;
    r.x = wrap_i<R>(Rx, pc.Lx, pc.inv_Lx);
    r.y = wrap_i<R>(Ry, pc.Ly, pc.inv_Ly);
    return flags;
}

template <typename R>
GCB_HD uint32_t finite_flag(const Regs<R>& r) {
    const bool ok = __builtin_isfinite(r.x) && __builtin_isfinite(r.y) && __builtin_isfinite(r.ux) && __builtin_isfinite(r.uy) &&
                    __builtin_isfinite(r.uz);
    return ok ? 0u : (uint32_t)ST_NONFINITE;
}

}  // inline namespace GCB_ARITH_NS
}  // namespace gcb
