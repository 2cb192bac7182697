// The curved-spacetime coupled step (Sec. 2.3, 2.4, 3.2) in spherical
// Kerr-Schild coordinates, binary64.
//
// Geometrized units (c = G = M = 1).  A particle carries x^i = (r, theta, phi)
// and the covariant spatial four-velocity u_i, both at the integer time level
// (not staggered, Sec. 3.2).  The spacetime is Kerr in Kerr-Schild form,
// evaluated analytically at every point (lapse alpha, shift beta^r, gamma^ij,
// gamma_ij, sqrt(gamma) and the r, theta derivatives of alpha, beta^r and
// gamma^ij); the fields D^i, B^i come from a uniform (r, theta) grid of nodes
// with the linear shape function; d/dphi = 0 (axisymmetry).
//
// One step:
//   switch (Sec. 3, 4.2): guiding center iff B > 0, Gamma/(|q/m| B dl) <
//     f_rho and D/B < f_E, with Gamma of the full u, magnitudes in the metric
//     and dl the square root of the proper area of the particle's cell;
//   full orbit (Sec. 2.3): half Lorentz push in the local frame of the normal
//     observer (orthonormal triad from the Cholesky factor L of gamma_ij:
//     u^ = L^-1 u, V^ = L^T V; there the push is the special-relativistic
//     Boris push with time step alpha dt/2), implicit-midpoint geodesic
//     update of (x, u) solved by K fixed-point iterations, second half push;
//   guiding center (Sec. 2.4): u = u_par b + v_E Gamma + u_perp_g at R^n = x^n
//     (Gamma of the full u), half parallel push alpha (q/m)(dt/2) D.b,
//     K fixed-point iterations of the implicit midpoint rule on (R, u_par)
//     with Gamma of eq. grgcalfac and the full u for the geodesic term rebuilt
//     with the gyration direction of the step start, second half push at
//     R^{n+1}, u rebuilt there (Sec. 3.2, step 5).
// Every expression is evaluated in a fixed order without fused multiply-add
// (the binary64 unit is compiled with -ffp-contract=off), sin and cos come
// from the fixed polynomial below, and square roots and quotients are IEEE,
// so the binary64 step is reproducible operation by operation.
//
// The arithmetic type R of the bulk work is a template parameter: double for
// the plain path, float for the precision form (binary32 fields, metric,
// four-velocity and bulk arithmetic; positions and their updates binary64;
// binary64 also for Gamma when |u|^2 > 1e6, for 1 - v_E^2 when v_E^2 > 0.81
// (recomputed from the binary64 metric), and for the switch when a ratio is
// within a relative 1e-4 of its threshold).
#pragma once

#include <type_traits>

#include "gcb_common.hpp"
#include "gcb_trig.hpp"

namespace gcb {
namespace gr {

constexpr uint8_t kStOut = 64;   // left the (r, theta) domain; no longer advanced

constexpr double kPi = 3.141592653589793;
constexpr double kTwoPi = 2.0 * kPi;

template <typename R>
constexpr bool kF32 = std::is_same<R, float>::value;

// The production form of the binary64 arithmetic (GCB_ARITH_FAST; its unit
// defines GCB_FAST_ARITH): besides contracted multiply-adds, the metric's
// quotients share the reciprocals of rho^2 and 1 + z, and a square root that
// only serves as a divisor (the lapse, the triad's diagonal, Gamma in the
// geodesic terms, B and kappa in the decomposition) becomes a reciprocal
// square root.  Each such value differs from the correctly rounded one by a
// few units in the last place.
#ifndef GCB_FAST_ARITH
#define GCB_FAST_ARITH 0
#endif
template <typename R>
constexpr bool kGrFast = (GCB_FAST_ARITH != 0) && std::is_same<R, double>::value;

// ---------------------------------------------------------------------------
// metric

template <typename R>
struct Metric {
    R alpha, beta_r;
    R gu_rr, gu_rph, gu_thth, gu_phph;   // gamma^ij
    R gd_rr, gd_rph, gd_thth, gd_phph;   // gamma_ij
    R sqrtg;
    // d/dr, d/dtheta
    R dalpha[2], dbeta_r[2], dgu_rr[2], dgu_rph[2], dgu_thth[2], dgu_phph[2];
};

// Kerr (M = 1, spin a) in Kerr-Schild form: rho^2 = r^2 + a^2 cos^2,
// z = 2r/rho^2, alpha = (1+z)^-1/2, beta^r = z/(1+z),
// gamma_rr = 1+z, gamma_rphi = -a(1+z) sin^2, gamma_thth = rho^2,
// gamma_phph = sin^2 (rho^2 + a^2 (1+z) sin^2), and the inverse
// gamma^rr = 1/(1+z) + a^2 sin^2/rho^2, gamma^rphi = a/rho^2,
// gamma^thth = 1/rho^2, gamma^phph = 1/(rho^2 sin^2).
template <bool kDerivs, typename R>
GCB_HD void kerr_schild(double a_, double r_, double th, Metric<R>& m) {
    const R a = (R)a_, r = (R)r_;
    const R a2 = a * a;
    R sn, cs;
    sincos_poly(th, sn, cs);
    const R s2 = sn * sn;
    const R c2 = cs * cs;
    const R rho2 = r * r + a2 * c2;
    if constexpr (kGrFast<R>) {
        const R ir2 = rcp_nr(rho2);
        const R z = ((R)2 * r) * ir2;
        const R opz = (R)1 + z;
        const R al = rsqrt_nr(opz);
        const R iopz = al * al;
        m.alpha = al;
        m.beta_r = z * iopz;
        m.gu_rr = iopz + (a2 * s2) * ir2;
        m.gu_rph = a * ir2;
        m.gu_thth = ir2;
        // 1/(rho^2 sin^2), infinite on the axis
        const R rs2 = rho2 * s2;
        m.gu_phph = rs2 == (R)0 ? (R)__builtin_inf() : rcp_nr(rs2);
        m.gd_rr = opz;
        m.gd_rph = -(a * opz) * s2;
        m.gd_thth = rho2;
        m.gd_phph = s2 * (rho2 + (a2 * opz) * s2);
        m.sqrtg = ((opz * al) * rho2) * sn;
        if (kDerivs) {
            const R sc = sn * cs;
            const R drho2[2] = {(R)2 * r, (R)-2 * (a2 * sc)};
            const R ir4 = ir2 * ir2;
            const R dz[2] = {((R)2 * (a2 * c2 - r * r)) * ir4, ((R)4 * (r * (a2 * sc))) * ir4};
            const R iopz2 = iopz * iopz;
            const R gp2 = m.gu_phph * m.gu_phph;
            for (int i = 0; i < 2; ++i) {
                m.dalpha[i] = (R)-0.5 * (al * iopz) * dz[i];
                m.dbeta_r[i] = dz[i] * iopz2;
                m.dgu_rph[i] = -(a * drho2[i]) * ir4;
                m.dgu_thth[i] = -drho2[i] * ir4;
            }
            m.dgu_rr[0] = -(dz[0] * iopz2) - (a2 * s2) * drho2[0] * ir4;
            m.dgu_rr[1] = (-(dz[1] * iopz2) + (a2 * ((R)2 * sc)) * ir2) -
                          (a2 * s2) * drho2[1] * ir4;
            m.dgu_phph[0] = -(drho2[0] * s2) * gp2;
            m.dgu_phph[1] = -(drho2[1] * s2 + rho2 * ((R)2 * sc)) * gp2;
        }
        return;
    }
    const R z = ((R)2 * r) / rho2;
    const R opz = (R)1 + z;
    const R sq = sqrt(opz);
    m.alpha = (R)1 / sq;
    m.beta_r = z / opz;
    m.gu_rr = (R)1 / opz + (a2 * s2) / rho2;
    m.gu_rph = a / rho2;
    m.gu_thth = (R)1 / rho2;
    m.gu_phph = (R)1 / (rho2 * s2);
    m.gd_rr = opz;
    m.gd_rph = -(a * opz) * s2;
    m.gd_thth = rho2;
    m.gd_phph = s2 * (rho2 + (a2 * opz) * s2);
    m.sqrtg = (sq * rho2) * sn;
    if (kDerivs) {
        const R sc = sn * cs;
        const R drho2[2] = {(R)2 * r, (R)-2 * (a2 * sc)};
        const R rho4 = rho2 * rho2;
        const R dz[2] = {((R)2 * (a2 * c2 - r * r)) / rho4, ((R)4 * (r * (a2 * sc))) / rho4};
        const R opz2 = opz * opz;
        for (int i = 0; i < 2; ++i) {
            m.dalpha[i] = (R)-0.5 * (m.alpha / opz) * dz[i];
            m.dbeta_r[i] = dz[i] / opz2;
            m.dgu_rph[i] = -(a * drho2[i]) / rho4;
            m.dgu_thth[i] = -drho2[i] / rho4;
        }
        m.dgu_rr[0] = -(dz[0] / opz2) - (a2 * s2) * drho2[0] / rho4;
        m.dgu_rr[1] = (-(dz[1] / opz2) + (a2 * ((R)2 * sc)) / rho2) - (a2 * s2) * drho2[1] / rho4;
        const R rs2 = rho2 * s2;
        m.dgu_phph[0] = -(drho2[0] * s2) / (rs2 * rs2);
        m.dgu_phph[1] = -(drho2[1] * s2 + rho2 * ((R)2 * sc)) / (rs2 * rs2);
    }
}

// ---------------------------------------------------------------------------
// fields on the (r, theta) grid: node-interleaved F[(j*(nr+1) + i)*6 + k],
// k = D^r, D^th, D^ph, B^r, B^th, B^ph at r_min + i dr, theta = j dth

struct GrConst {
    double a, dt, qm, f_rho, f_E, fp_tol;
    double mirror_tol;   // > 0: ST_MIRROR where (v_perp_g/c)^2 exceeds it
    double r_min, r_max, inv_dr, inv_dth;
    int nr, nth, n_iter;
};

template <typename R>
struct GrSample {
    R D[3], B[3];
};

// clamped cell of a point (a NaN coordinate is taken at the lower edge)
GCB_HD void grid_cell(const GrConst& g, double r, double th, int& i, int& j, double& wx,
                      double& wy) {
    double rc = r < g.r_min ? g.r_min : (r > g.r_max ? g.r_max : r);
    double tc = th < 0.0 ? 0.0 : (th > kPi ? kPi : th);
    if (rc != rc) rc = g.r_min;
    if (tc != tc) tc = 0.0;
    const double xi = (rc - g.r_min) * g.inv_dr;
    const double eta = tc * g.inv_dth;
    double fi = floor(xi), fj = floor(eta);
    fi = fi > (double)(g.nr - 1) ? (double)(g.nr - 1) : fi;
    fj = fj > (double)(g.nth - 1) ? (double)(g.nth - 1) : fj;
    i = (int)fi;
    j = (int)fj;
    wx = xi - fi;
    wy = eta - fj;
}

template <typename R, typename T>
GCB_HD void grid_sample(const T* __restrict__ F, const GrConst& g, double r, double th,
                        GrSample<R>& s) {
    int i, j;
    double wxd, wyd;
    grid_cell(g, r, th, i, j, wxd, wyd);
    const R wx = (R)wxd, wy = (R)wyd;
    const R ax = (R)1 - wx, ay = (R)1 - wy;
    const int W = g.nr + 1;
    const T* p0 = F + ((size_t)j * W + i) * 6;
    const T* p1 = p0 + (size_t)W * 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const R f00 = (R)p0[k], f10 = (R)p0[6 + k];
        const R f01 = (R)p1[k], f11 = (R)p1[6 + k];
        const R v = ay * (ax * f00 + wx * f10) + wy * (ax * f01 + wx * f11);
        if (k < 3)
            s.D[k] = v;
        else
            s.B[k - 3] = v;
    }
}

template <typename R>
GCB_HD GrSample<double> to_f64(const GrSample<R>& f) {
    GrSample<double> d;
    for (int i = 0; i < 3; ++i) {
        d.D[i] = (double)f.D[i];
        d.B[i] = (double)f.B[i];
    }
    return d;
}

GCB_HD bool inside(const GrConst& g, double r, double th) {
    return r >= g.r_min && r < g.r_max && th >= 0.0 && th <= kPi;
}

// ---------------------------------------------------------------------------
// index gymnastics

template <typename R>
GCB_HD void lower(const Metric<R>& m, const R V[3], R out[3]) {
    out[0] = m.gd_rr * V[0] + m.gd_rph * V[2];
    out[1] = m.gd_thth * V[1];
    out[2] = m.gd_rph * V[0] + m.gd_phph * V[2];
}

template <typename R>
GCB_HD void raise(const Metric<R>& m, const R w[3], R out[3]) {
    out[0] = m.gu_rr * w[0] + m.gu_rph * w[2];
    out[1] = m.gu_thth * w[1];
    out[2] = m.gu_rph * w[0] + m.gu_phph * w[2];
}

template <typename R>
GCB_HD R norm2_cov(const Metric<R>& m, const R w[3]) {
    R up[3];
    raise(m, w, up);
    return (w[0] * up[0] + w[1] * up[1]) + w[2] * up[2];
}

template <typename R>
GCB_HD R norm2_con(const Metric<R>& m, const R V[3]) {
    R lo[3];
    lower(m, V, lo);
    return (V[0] * lo[0] + V[1] * lo[1]) + V[2] * lo[2];
}

template <typename R>
GCB_HD R gamma_of(const Metric<R>& m, const R u[3]) {
    const R n2 = norm2_cov(m, u);
    if constexpr (kF32<R>) {
        if (n2 > 1.0e6f) return (R)sqrt(1.0 + (double)n2);   // ultra-relativistic: binary64
    }
    return sqrt((R)1 + n2);
}

GCB_HD double max_nan(double a, double b) { return (a > b || a != a) ? a : b; }

// A Lorentz factor and, in the production form, its reciprocal (the
// geodesic terms divide by it).
template <typename R>
struct Lorentz {
    R g, inv;
};

template <typename R>
GCB_HD Lorentz<R> lorentz_of(const Metric<R>& m, const R u[3]) {
    if constexpr (kGrFast<R>) {
        const R s = (R)1 + norm2_cov(m, u);
        const R inv = rsqrt_nr(s);
        return {s * inv, inv};
    } else {
        return {gamma_of(m, u), (R)0};
    }
}

// ---------------------------------------------------------------------------
// local-frame half push: Lorentz force over dt/2 (Boris with step alpha dt/2)

template <typename R>
GCB_HD void half_push(const Metric<R>& m, const GrSample<R>& f, R u[3], double qm_,
                      double dt_) {
    const R qm = (R)qm_, dt = (R)dt_;
    R L11, L22, L31, L33, u1, u2, u3;
    if constexpr (kGrFast<R>) {
        const R i11 = rsqrt_nr(m.gd_rr);
        const R i22 = rsqrt_nr(m.gd_thth);
        L11 = m.gd_rr * i11;
        L22 = m.gd_thth * i22;
        L31 = m.gd_rph * i11;
        const R q33 = m.gd_phph - L31 * L31;
        const R i33 = rsqrt_nr(q33);
        L33 = q33 * i33;
        u1 = u[0] * i11;
        u2 = u[1] * i22;
        u3 = (u[2] - L31 * u1) * i33;
    } else {
        L11 = sqrt(m.gd_rr);
        L22 = sqrt(m.gd_thth);
        L31 = m.gd_rph / L11;
        L33 = sqrt(m.gd_phph - L31 * L31);
        u1 = u[0] / L11;
        u2 = u[1] / L22;
        u3 = (u[2] - L31 * u1) / L33;
    }
    const R D1 = L11 * f.D[0] + L31 * f.D[2], D2 = L22 * f.D[1], D3 = L33 * f.D[2];
    const R B1 = L11 * f.B[0] + L31 * f.B[2], B2 = L22 * f.B[1], B3 = L33 * f.B[2];
    const R hq = (qm * (m.alpha * ((R)0.5 * dt))) * (R)0.5;
    const R umx = u1 + hq * D1, umy = u2 + hq * D2, umz = u3 + hq * D3;
    const R gm2 = (R)1 + ((umx * umx + umy * umy) + umz * umz);
    R fq;
    if constexpr (kGrFast<R>)
        fq = hq * rsqrt_nr(gm2);
    else
        fq = hq / sqrt(gm2);
    const R tx = fq * B1, ty = fq * B2, tz = fq * B3;
    const R t2 = (tx * tx + ty * ty) + tz * tz;
    R g;
    if constexpr (kGrFast<R>)
        g = (R)2 * rcp_nr((R)1 + t2);
    else
        g = (R)2 / ((R)1 + t2);
    const R sx = g * tx, sy = g * ty, sz = g * tz;
    const R upx = umx + (umy * tz - umz * ty);
    const R upy = umy + (umz * tx - umx * tz);
    const R upz = umz + (umx * ty - umy * tx);
    const R uqx = umx + (upy * sz - upz * sy);
    const R uqy = umy + (upz * sx - upx * sz);
    const R uqz = umz + (upx * sy - upy * sx);
    const R v1 = uqx + hq * D1, v2 = uqy + hq * D2, v3 = uqz + hq * D3;
    u[0] = L11 * v1;
    u[1] = L22 * v2;
    u[2] = L31 * v1 + L33 * v3;
}

// geodesic terms (Sec. 2.3): V^i = alpha gamma^ij u_j/Gamma - beta^i and
// G_i = -Gamma d_i alpha + u_j d_i beta^j - alpha u_j u_k d_i gamma^jk/(2 Gamma)
// for i = r, theta (G_phi = 0)
template <typename R>
GCB_HD void geo_V(const Metric<R>& m, const R u[3], const Lorentz<R>& Gam, R V[3]) {
    R up[3];
    raise(m, u, up);
    R ag;
    if constexpr (kGrFast<R>)
        ag = m.alpha * Gam.inv;
    else
        ag = m.alpha / Gam.g;
    V[0] = ag * up[0] - m.beta_r;
    V[1] = ag * up[1];
    V[2] = ag * up[2];
}

template <typename R>
GCB_HD void geo_G(const Metric<R>& m, const R u[3], const Lorentz<R>& Gam, R G[2]) {
    const R ur = u[0], ut = u[1], up = u[2];
    R h;
    if constexpr (kGrFast<R>)
        h = ((R)0.5 * m.alpha) * Gam.inv;
    else
        h = m.alpha / ((R)2 * Gam.g);
    for (int i = 0; i < 2; ++i) {
        const R q = ((ur * ur) * m.dgu_rr[i] + ((R)2 * (ur * up)) * m.dgu_rph[i]) +
                    ((ut * ut) * m.dgu_thth[i] + (up * up) * m.dgu_phph[i]);
        G[i] = (-(Gam.g * m.dalpha[i]) + ur * m.dbeta_r[i]) - h * q;
    }
}

// guiding-center quantities at a point
template <typename R>
struct GcLocal {
    R B, kappa, Dpar;
    R b_up[3], b_dn[3], vE[3];
    R inv_B, inv_kappa;   // the production form's reciprocals
};

// (a, r, th) locate the point for the binary64 recomputation of 1 - v_E^2
// in the precision form
template <typename R>
GCB_HD uint32_t gc_local(const Metric<R>& m, const GrSample<R>& f, GcLocal<R>& L, double a,
                         double r, double th) {
    uint32_t flags = 0;
    R Bl[3];
    lower(m, f.B, Bl);
    const R B2 = (f.B[0] * Bl[0] + f.B[1] * Bl[1]) + f.B[2] * Bl[2];
    R Bm, inv_B;
    bool bzero;
    if constexpr (kGrFast<R>) {
        // 1/B from 1/sqrt(B^2); a negative or NaN B^2 gives NaN as sqrt does
        bzero = B2 == (R)0;
        inv_B = B2 > (R)0 ? rsqrt_nr(B2) : (bzero ? (R)0 : sqrt(B2));
        Bm = bzero ? (R)0 : B2 * inv_B;
    } else {
        Bm = sqrt(B2);
        bzero = Bm == (R)0;
        inv_B = bzero ? (R)0 : (R)1 / Bm;
    }
    if (bzero) flags |= ST_BZERO;
    L.B = Bm;
    L.inv_B = inv_B;
    for (int i = 0; i < 3; ++i) {
        L.b_up[i] = f.B[i] * inv_B;
        L.b_dn[i] = Bl[i] * inv_B;
    }
    const R DxB[3] = {m.sqrtg * (f.D[1] * f.B[2] - f.D[2] * f.B[1]),
                      m.sqrtg * (f.D[2] * f.B[0] - f.D[0] * f.B[2]),
                      m.sqrtg * (f.D[0] * f.B[1] - f.D[1] * f.B[0])};
    const R ib2 = inv_B * inv_B;
    for (int i = 0; i < 3; ++i) L.vE[i] = DxB[i] * ib2;
    const R vE2 = norm2_cov(m, L.vE);
    if constexpr (kF32<R>) {
        double om = 1.0 - (double)vE2;
        if (vE2 > 0.81f && !bzero) {
            // D/B > 0.9: 1 - v_E^2 cancels; redo it in binary64
            Metric<double> md;
            kerr_schild<false>(a, r, th, md);
            const GrSample<double> fd = to_f64(f);
            GcLocal<double> Ld;
            (void)gc_local(md, fd, Ld, a, r, th);
            om = 1.0 - norm2_cov(md, Ld.vE);
        }
        if (om < kKappaFloor) {
            om = kKappaFloor;
            flags |= ST_KAPPA;
        }
        L.kappa = (R)(1.0 / sqrt(om));
    } else {
        R om = (R)1 - vE2;
        if (om < (R)kKappaFloor) {
            om = (R)kKappaFloor;
            flags |= ST_KAPPA;
        }
        if constexpr (kGrFast<R>) {
            L.kappa = rsqrt_nr(om);
            L.inv_kappa = om * L.kappa;
        } else {
            L.kappa = (R)1 / sqrt(om);
        }
    }
    L.Dpar = (f.D[0] * L.b_dn[0] + f.D[1] * L.b_dn[1]) + f.D[2] * L.b_dn[2];
    return flags;
}

// eq. grgcalfac with m = 1
template <typename R>
GCB_HD R gamma_gc(const GcLocal<R>& L, R upar, R mu) {
    return L.kappa * sqrt(((R)1 + upar * upar) + (((R)2 * mu) * L.B) * L.kappa);
}

// the same with, in the production form, its reciprocal
template <typename R>
GCB_HD Lorentz<R> lorentz_gc(const GcLocal<R>& L, R upar, R mu) {
    if constexpr (kGrFast<R>) {
        const R s = ((R)1 + upar * upar) + (((R)2 * mu) * L.B) * L.kappa;
        const R rs = rsqrt_nr(s);
        return {L.kappa * (s * rs), L.inv_kappa * rs};
    } else {
        return {gamma_gc(L, upar, mu), (R)0};
    }
}

template <typename R>
GCB_HD bool switch_gca(const Metric<R>& m, const GrSample<R>& f, const R u[3], double qm,
                       double dl, const GrConst& g, double r, double th) {
    const R Bm = sqrt(norm2_con(m, f.B));
    const R Dm = sqrt(norm2_con(m, f.D));
    const R Gam = gamma_of(m, u);
    const R safe = Bm > (R)0 ? Bm : (R)1;
    const R rho = Gam / ((R)fabs(qm) * safe);
    const R rr = rho / (R)dl, er = Dm / safe;
    if constexpr (kF32<R>) {
        // near a threshold the test is repeated in binary64
        const bool near = fabs(rr - (R)g.f_rho) <= 1.0e-4f * (R)g.f_rho ||
                          fabs(er - (R)g.f_E) <= 1.0e-4f * (R)g.f_E;
        if (near) {
            Metric<double> md;
            kerr_schild<false>(g.a, r, th, md);
            const double ud[3] = {(double)u[0], (double)u[1], (double)u[2]};
            return switch_gca<double>(md, to_f64(f), ud, qm, dl, g, r, th);
        }
    }
    return Bm > (R)0 && rr < (R)g.f_rho && er < (R)g.f_E;
}

GCB_HD double wrap_phi(double ph) {
    double w = ph - kTwoPi * floor(ph / kTwoPi);
    if (w < 0.0) w = w + kTwoPi;
    if (w >= kTwoPi) w = w - kTwoPi;
    return w;
}

// The switch (Sec. 4.1) at x^n from the metric and the fields there.
template <typename R>
GCB_HD bool switch_with(const Metric<R>& m0, const GrSample<R>& f0,
                        const double* __restrict__ dl_table, const GrConst& g,
                        const double x[3], const R u[3], double qm) {
    int ci, cj;
    double wx, wy;
    grid_cell(g, x[0], x[1], ci, cj, wx, wy);
    const double dl = dl_table[(size_t)cj * g.nr + ci];
    return switch_gca(m0, f0, u, qm, dl, g, x[0], x[1]);
}

// The same with the metric and the fields at x^n evaluated here (the start
// of a step, kept for the step's decomposition or half push).
template <typename R, typename T>
GCB_HD bool switch_at(const T* __restrict__ F, const double* __restrict__ dl_table,
                      const GrConst& g, const double x[3], const R u[3], double qm,
                      Metric<R>& m0, GrSample<R>& f0) {
    kerr_schild<false>(g.a, x[0], x[1], m0);
    grid_sample(F, g, x[0], x[1], f0);
    return switch_with(m0, f0, dl_table, g, x, u, qm);
}

// The metric and the fields at a particle's position as the end of one step
// evaluated them, for the start of the next: the same point, so the same
// values, evaluated once.
template <typename R>
struct StepStart {
    Metric<R> m;   // without the derivatives
    GrSample<R> f;
    bool valid;
};

// The branch the next step of a particle takes: true for the guiding
// center; a particle outside the domain is not advanced and counts as not.
template <typename R, typename T>
GCB_HD bool starts_gca(const T* __restrict__ F, const double* __restrict__ dl_table,
                       const GrConst& g, const double x[3], const R u[3], double qm,
                       uint8_t status) {
    if ((status & kStOut) || !inside(g, x[0], x[1])) return false;
    Metric<R> m0;
    GrSample<R> f0;
    return switch_at(F, dl_table, g, x, u, qm, m0, f0);
}

// One coupled step (Sec. 3.2) of one particle.  Returns S: 0 guiding
// center, 1 full orbit, 2 not advanced (outside the domain).
//
// Full orbit (Sec. 2.3): half push at x^n; K fixed-point iterations of the
// implicit midpoint rule x^{n+1} = x^n + dt V(xb, ub), u'' = u' + dt G(xb, ub)
// with xb, ub the midpoints; half push at x^{n+1}.
// Guiding center (Sec. 2.4): decomposition at R^n = x^n with Gamma of the
// full u, u_par' = u_par + alpha (q/m)(dt/2) D.b; K iterations of
// R^{n+1} = R^n + dt V~(Rb, pb), u_par'' = u_par' + dt G(Rb, ub).b with
// Gamma(Rb, pb) of eq. grgcalfac and ub = pb b + v_E Gamma + u_perp_g bperp;
// second half push and reconstruction at R^{n+1}.
//
// The two branches share their skeleton -- metric and fields at x^n, K
// midpoint iterations that each need the metric and its derivatives and the
// geodesic force G, metric and fields at x^{n+1} -- so they are evaluated in
// one pass: a wavefront whose lanes took different branches runs the shared
// metric evaluations once, and only the branch-specific parts diverge.
//
// `start` carries the metric and the fields at x^{n+1} into the next step of
// the same particle (start.valid false: evaluated here).
template <typename R, typename T>
GCB_HD int coupled_step(const T* __restrict__ F, const double* __restrict__ dl_table,
                        const GrConst& g, double x[3], R u[3], double qm, uint8_t& status,
                        double& res, StepStart<R>& start) {
    res = 0.0;
    if ((status & kStOut) || !inside(g, x[0], x[1])) {
        if (!inside(g, x[0], x[1])) status |= kStOut;
        return 2;
    }
    const R dt = (R)g.dt;
    Metric<R> m0;
    GrSample<R> f0;
    bool gca;
    if (start.valid) {
        m0 = start.m;
        f0 = start.f;
        gca = switch_with(m0, f0, dl_table, g, x, u, qm);
    } else {
        gca = switch_at(F, dl_table, g, x, u, qm, m0, f0);
    }

    uint32_t fl = 0;
    // guiding-center state: mu, gyration direction, u_par after the half push
    R mu = (R)0, bperp[3] = {(R)0, (R)0, (R)0}, p1 = (R)0, pk = (R)0;
    // full-orbit state: u after the half push, the iterate u''
    R u1[3] = {u[0], u[1], u[2]}, uk[3];
    if (gca) {
        GcLocal<R> L0;
        fl |= gc_local(m0, f0, L0, g.a, x[0], x[1]);
        const R Gf = gamma_of(m0, u);
        const R upar = (L0.b_up[0] * u[0] + L0.b_up[1] * u[1]) + L0.b_up[2] * u[2];
        R uperp[3];
        for (int i = 0; i < 3; ++i) uperp[i] = (u[i] - upar * L0.b_dn[i]) - L0.vE[i] * Gf;
        const R up2 = norm2_cov(m0, uperp);
        // the check of the neglect of the mirror terms (c = 1)
        if (g.mirror_tol > 0.0 && up2 > (R)g.mirror_tol * (Gf * Gf)) fl |= ST_MIRROR;
        R inv_nu;
        if constexpr (kGrFast<R>) {
            mu = (((R)0.5 * up2) * L0.inv_B) * L0.inv_kappa;
            inv_nu = up2 > (R)0 ? rsqrt_nr(up2) : (R)0;
        } else {
            mu = (((R)0.5 * up2) / L0.B) / L0.kappa;
            const R nu = sqrt(up2);
            inv_nu = nu > (R)0 ? (R)1 / nu : (R)0;
        }
        if (!(L0.B > (R)0)) mu = (R)0;
        for (int i = 0; i < 3; ++i) bperp[i] = uperp[i] * inv_nu;
        p1 = upar + ((R)qm * (m0.alpha * ((R)0.5 * dt))) * L0.Dpar;
        pk = p1;
    } else {
        half_push(m0, f0, u1, qm, g.dt);
    }
    for (int i = 0; i < 3; ++i) uk[i] = u1[i];

    double Xk[3] = {x[0], x[1], x[2]};
    for (int k = 0; k < g.n_iter; ++k) {
        double Xb[3];
        for (int i = 0; i < 3; ++i) Xb[i] = 0.5 * (Xk[i] + x[i]);
        Metric<R> mb;
        kerr_schild<true>(g.a, Xb[0], Xb[1], mb);
        R V[3], ub[3];
        Lorentz<R> Gam;
        R bup0 = (R)0, bup1 = (R)0;
        if (gca) {
            const R pb = (R)0.5 * (pk + p1);
            GrSample<R> fb;
            grid_sample(F, g, Xb[0], Xb[1], fb);
            GcLocal<R> Lb;
            fl |= gc_local(mb, fb, Lb, g.a, Xb[0], Xb[1]);
            Gam = lorentz_gc(Lb, pb, mu);
            R vu[3];
            raise(mb, Lb.vE, vu);
            R bG[3];
            for (int i = 0; i < 3; ++i) {
                if constexpr (kGrFast<R>)
                    bG[i] = Lb.b_up[i] * Gam.inv;
                else
                    bG[i] = Lb.b_up[i] / Gam.g;
            }
            V[0] = mb.alpha * (pb * bG[0] + vu[0]) - mb.beta_r;
            V[1] = mb.alpha * (pb * bG[1] + vu[1]);
            V[2] = mb.alpha * (pb * bG[2] + vu[2]);
            const R upg = sqrt((((R)2 * mu) * Lb.kappa) * Lb.B);
            for (int i = 0; i < 3; ++i)
                ub[i] = (pb * Lb.b_dn[i] + Lb.vE[i] * Gam.g) + upg * bperp[i];
            bup0 = Lb.b_up[0];
            bup1 = Lb.b_up[1];
        } else {
            for (int i = 0; i < 3; ++i) ub[i] = (R)0.5 * (uk[i] + u1[i]);
            Gam = lorentz_of(mb, ub);
            geo_V(mb, ub, Gam, V);
        }
        R G[2];
        geo_G(mb, ub, Gam, G);
        double Xn[3];
        for (int i = 0; i < 3; ++i) Xn[i] = x[i] + (double)(dt * V[i]);
        res = max_nan(max_nan(fabs(Xn[0] - Xk[0]), fabs(Xn[1] - Xk[1])), fabs(Xn[2] - Xk[2]));
        for (int i = 0; i < 3; ++i) Xk[i] = Xn[i];
        if (gca) {
            const R Gb = G[0] * bup0 + G[1] * bup1;
            pk = p1 + dt * Gb;
        } else {
            uk[0] = u1[0] + dt * G[0];
            uk[1] = u1[1] + dt * G[1];
            uk[2] = u1[2];
        }
    }

    Metric<R> m1;
    kerr_schild<false>(g.a, Xk[0], Xk[1], m1);
    GrSample<R> f1;
    grid_sample(F, g, Xk[0], Xk[1], f1);
    R un[3];
    if (gca) {
        GcLocal<R> L1;
        fl |= gc_local(m1, f1, L1, g.a, Xk[0], Xk[1]);
        const R upar1 = pk + ((R)qm * (m1.alpha * ((R)0.5 * dt))) * L1.Dpar;
        const R Gam1 = gamma_gc(L1, upar1, mu);
        const R upg1 = sqrt((((R)2 * mu) * L1.kappa) * L1.B);
        for (int i = 0; i < 3; ++i)
            un[i] = (upar1 * L1.b_dn[i] + L1.vE[i] * Gam1) + upg1 * bperp[i];
    } else {
        half_push(m1, f1, uk, qm, g.dt);
        for (int i = 0; i < 3; ++i) un[i] = uk[i];
    }

    if (res > g.fp_tol) fl |= ST_FPRES;
    bool fin = true;
    for (int i = 0; i < 3; ++i) fin = fin && __builtin_isfinite(Xk[i]) && __builtin_isfinite(un[i]);
    if (!fin) fl |= ST_NONFINITE;
    if (!inside(g, Xk[0], Xk[1])) fl |= kStOut;
    x[0] = Xk[0];
    x[1] = Xk[1];
    x[2] = wrap_phi(Xk[2]);
    for (int i = 0; i < 3; ++i) u[i] = un[i];
    status = (uint8_t)(status | fl);
    start.m = m1;
    start.f = f1;
    start.valid = true;
    return gca ? 0 : 1;
}

// sqrt(proper area) of cell (i, j) by 2 x 2 Gauss-Legendre points
GCB_HD double cell_length(const GrConst& g, double dr, double dth, int i, int j) {
    const double hr = 0.5 * dr;
    const double ht = 0.5 * dth;
    const double q = 1.0 / sqrt(3.0);
    const double rc = g.r_min + ((double)i + 0.5) * dr;
    const double tc = ((double)j + 0.5) * dth;
    const double rm = rc - hr * q, rp = rc + hr * q;
    const double tm = tc - ht * q, tp = tc + ht * q;
    auto f = [&](double r, double t) {
        Metric<double> m;
        kerr_schild<false>(g.a, r, t, m);
        return sqrt(m.gd_rr * m.gd_thth);
    };
    const double tot = ((f(rm, tm) + f(rp, tm)) + f(rm, tp)) + f(rp, tp);
    return sqrt(tot * (hr * ht));
}

}  // namespace gr
}  // namespace gcb
