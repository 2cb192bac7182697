// Reverse-mode derivative (vector-Jacobian products) of one binary64 step of
// the coupled pusher, with the switch decision held at its forward value.
//
// Every building block of the forward step in gcb_math.hpp has a hand-written
// adjoint here; a block's adjoint recomputes the forward values it needs from
// its inputs.  Cotangents are accumulated (+=) into the *Bar structures.
//   gather_vjp       linear shape function: the position cotangent,
//                    including the mixed second derivative of W carried by
//                    the B-gradient cotangents; the gather point and its
//                    cotangents go to a sink
//   scatter_sample   node cotangents of one recorded gather point
//   local_vjp        b, v_E, kappa, E_par, d_j b_i, (b.grad)b, (v_E.grad)b
//   gamma_vjp        Gamma(R, u_par) (eq. lfacgca2)
//   vcurv_vjp        curvature drift (eq. curvdrift)
//   drift_vjp        u_par b/Gamma + v_E + v_c
//   parallel_vjp     the parallel update (Sec. 2.2.2) through the root of the
//                    quadratic by the implicit-function derivative
//                    dG = -(G^2 dk1 + G dk2 + dk3)/(2 k1 G + k2)
//   boris_step_vjp   relativistic Boris push and position update
//   gca_step_vjp     the guiding-center step (Sec. 3.1): decomposition,
//                    parallel update, K fixed-point iterations (reversed in
//                    order), reconstruction
#pragma once

#include "gcb_math.hpp"

namespace gcb {
namespace adj {

using SampleD = Sample<double>;
using LocalD = Local<double>;
using KD = Consts<double>;

struct SampleBar {
    double E[3], B[3], dBx[3], dBy[3];
};

struct LocalBar {
    double B, inv_B, b[3], vE[3], kappa, Epar, bgb[3], vgb[3], A, C;
};

GCB_HD void zero(SampleBar& s) {
    for (int i = 0; i < 3; ++i) s.E[i] = s.B[i] = s.dBx[i] = s.dBy[i] = 0.0;
}

GCB_HD void zero(LocalBar& l) {
    l.B = l.inv_B = l.kappa = l.Epar = l.A = l.C = 0.0;
    for (int i = 0; i < 3; ++i) l.b[i] = l.vE[i] = l.bgb[i] = l.vgb[i] = 0.0;
}

// cotangent of a x b: a_bar += b x z_bar, b_bar += z_bar x a
GCB_HD void cross_vjp(const double a[3], const double b[3], const double zb[3], double ab[3],
                      double bb[3]) {
    ab[0] += b[1] * zb[2] - b[2] * zb[1];
    ab[1] += b[2] * zb[0] - b[0] * zb[2];
    ab[2] += b[0] * zb[1] - b[1] * zb[0];
    bb[0] += zb[1] * a[2] - zb[2] * a[1];
    bb[1] += zb[2] * a[0] - zb[0] * a[2];
    bb[2] += zb[0] * a[1] - zb[1] * a[0];
}

// ---------------------------------------------------------------------------
// gather

// Node cotangents of one gather point: the cotangents of the six interpolated
// components and of the B gradients at (X, Y) spread over the four nodes of
// each component's cell, `add(k, i, j, g)` with global node indices (any
// periodic image).
template <class Add>
GCB_HD void scatter_sample(Add& add, const PushConst& pc, bool yee, double X, double Y,
                           const SampleBar& sb) {
    const double gx = X * pc.inv_dx;
    const double gy = Y * pc.inv_dy;
    const double idx = pc.inv_dx, idy = pc.inv_dy;
    // a runaway point's sample is a constant NaN: no node cotangent
    if (!(fabs(gx) < kFarLattice && fabs(gy) < kFarLattice)) return;
    for (int k = 0; k < 6; ++k) {
        const double sx = yee ? kYeeStagger[k][0] : pc.stagger[k][0];
        const double sy = yee ? kYeeStagger[k][1] : pc.stagger[k][1];
        const double vb = k < 3 ? sb.E[k] : sb.B[k - 3];
        const double dxb = k < 3 ? 0.0 : sb.dBx[k - 3];
        const double dyb = k < 3 ? 0.0 : sb.dBy[k - 3];
        if (vb == 0.0 && dxb == 0.0 && dyb == 0.0) continue;
        const double xi = gx - sx, eta = gy - sy;
        const double fi = floor(xi), fj = floor(eta);
        const double wx = xi - fi, wy = eta - fj;
        const int i = (int)fi, j = (int)fj;
        const double ax = 1.0 - wx, ay = 1.0 - wy;
        add(k, i, j, vb * (ax * ay) - dxb * (ay * idx) - dyb * (ax * idy));
        add(k, i + 1, j, vb * (wx * ay) + dxb * (ay * idx) - dyb * (wx * idy));
        add(k, i, j + 1, vb * (ax * wy) - dxb * (wy * idx) + dyb * (ax * idy));
        add(k, i + 1, j + 1, vb * (wx * wy) + dxb * (wy * idx) + dyb * (wx * idy));
    }
}

// Cotangent of the gather at (X, Y): the position cotangent, including the
// mixed second derivative of W carried by the B-gradient cotangents, is added
// to (Xb, Yb); the gather point and its cotangents go to `sink.sample`, which
// owns the node cotangents (scatter_sample spreads them).
template <class Acc, class Sink>
GCB_HD void gather_vjp(const Acc& acc, Sink& sink, const PushConst& pc, bool yee, double X,
                       double Y, const SampleBar& sb, double& Xb, double& Yb) {
    sink.sample(X, Y, sb);
    const double gx = X * pc.inv_dx;
    const double gy = Y * pc.inv_dy;
    const double idx = pc.inv_dx, idy = pc.inv_dy;
    // a runaway point's sample is a constant NaN: it does not depend on (X, Y)
    if (!(fabs(gx) < kFarLattice && fabs(gy) < kFarLattice)) return;
    for (int k = 0; k < 6; ++k) {
        const double sx = yee ? kYeeStagger[k][0] : pc.stagger[k][0];
        const double sy = yee ? kYeeStagger[k][1] : pc.stagger[k][1];
        const double vb = k < 3 ? sb.E[k] : sb.B[k - 3];
        const double dxb = k < 3 ? 0.0 : sb.dBx[k - 3];
        const double dyb = k < 3 ? 0.0 : sb.dBy[k - 3];
        if (vb == 0.0 && dxb == 0.0 && dyb == 0.0) continue;
        const double xi = gx - sx, eta = gy - sy;
        const double fi = floor(xi), fj = floor(eta);
        const double wx = xi - fi, wy = eta - fj;
        const int i = (int)fi, j = (int)fj;
        double f00, f10, f01, f11;
        acc.quad(k, i, j, f00, f10, f01, f11);
        const double ax = 1.0 - wx, ay = 1.0 - wy;
        const double cross = (((f11 - f01) - f10) + f00) * (idx * idy);
        Xb += vb * ((ay * (f10 - f00) + wy * (f11 - f01)) * idx) + dyb * cross;
        Yb += vb * ((ax * (f01 - f00) + wx * (f11 - f10)) * idy) + dxb * cross;
    }
}

// ---------------------------------------------------------------------------
// local quantities

// Cotangents of E, B and of the ND B-gradient directions G[j][i] = d_j B_i
// (ND = 2 in the plane, 3 in space) from those of the local quantities.
template <int ND>
GCB_HD void local_vjp_nd(const double E[3], const double Bv[3], const double G[ND][3],
                         const KD& K, const LocalBar& Lb, double Eb[3], double Bb[3],
                         double Gb[ND][3]) {
    for (int i = 0; i < 3; ++i) Eb[i] = Bb[i] = 0.0;
    for (int j = 0; j < ND; ++j)
        for (int i = 0; i < 3; ++i) Gb[j][i] = 0.0;
    const double B = sqrt((Bv[0] * Bv[0] + Bv[1] * Bv[1]) + Bv[2] * Bv[2]);
    if (B == 0.0) return;   // b, v_E and the curvature terms are held at 0 there
    const double inv_B = 1.0 / B;
    const double b[3] = {Bv[0] * inv_B, Bv[1] * inv_B, Bv[2] * inv_B};
    const double sc = K.c * (inv_B * inv_B);
    const double ExB[3] = {E[1] * Bv[2] - E[2] * Bv[1], E[2] * Bv[0] - E[0] * Bv[2],
                           E[0] * Bv[1] - E[1] * Bv[0]};
    const double vE[3] = {sc * ExB[0], sc * ExB[1], sc * ExB[2]};
    const double vE2 = (vE[0] * vE[0] + vE[1] * vE[1]) + vE[2] * vE[2];
    const double om = 1.0 - vE2 * K.inv_c2;
    const bool clamped = om < kKappaFloor;
    const double kappa = 1.0 / sqrt(clamped ? kKappaFloor : om);
    double dn[ND], db[ND][3], bgb[3], vgb[3];
    for (int j = 0; j < ND; ++j) {
        dn[j] = (b[0] * G[j][0] + b[1] * G[j][1]) + b[2] * G[j][2];
        for (int i = 0; i < 3; ++i) db[j][i] = (G[j][i] - b[i] * dn[j]) * inv_B;
    }
    for (int i = 0; i < 3; ++i) {
        bgb[i] = 0.0;
        vgb[i] = 0.0;
        for (int j = 0; j < ND; ++j) {
            bgb[i] += b[j] * db[j][i];
            vgb[i] += vE[j] * db[j][i];
        }
    }

    double vEb[3], bb[3], bgbb[3], vgbb[3];
    for (int i = 0; i < 3; ++i) {
        vEb[i] = Lb.vE[i] + Lb.A * bgb[i] + Lb.C * vgb[i];
        bb[i] = Lb.b[i];
        bgbb[i] = Lb.bgb[i] + Lb.A * vE[i];
        vgbb[i] = Lb.vgb[i] + Lb.C * vE[i];
    }
    double invBb = Lb.inv_B;
    double Bmb = Lb.B;
    double dbb[ND][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < ND; ++j) {
            vEb[j] += vgbb[i] * db[j][i];
            bb[j] += bgbb[i] * db[j][i];
            dbb[j][i] = vgbb[i] * vE[j] + bgbb[i] * b[j];
        }
    double dnb[ND];
    for (int j = 0; j < ND; ++j) {
        dnb[j] = 0.0;
        for (int i = 0; i < 3; ++i) {
            Gb[j][i] = dbb[j][i] * inv_B;
            bb[i] -= dbb[j][i] * dn[j] * inv_B;
            dnb[j] -= dbb[j][i] * b[i] * inv_B;
            invBb += dbb[j][i] * (G[j][i] - b[i] * dn[j]);
        }
    }
    for (int j = 0; j < ND; ++j)
        for (int i = 0; i < 3; ++i) {
            bb[i] += dnb[j] * G[j][i];
            Gb[j][i] += dnb[j] * b[i];
        }
    for (int i = 0; i < 3; ++i) {
        Eb[i] = Lb.Epar * b[i];
        bb[i] += Lb.Epar * E[i];
    }
    if (!clamped) {
        const double omb = Lb.kappa * (-0.5) * kappa * kappa * kappa;
        const double vE2b = -omb * K.inv_c2;
        for (int i = 0; i < 3; ++i) vEb[i] += 2.0 * vE[i] * vE2b;
    }
    const double scb = (vEb[0] * ExB[0] + vEb[1] * ExB[1]) + vEb[2] * ExB[2];
    const double ExBb[3] = {vEb[0] * sc, vEb[1] * sc, vEb[2] * sc};
    cross_vjp(E, Bv, ExBb, Eb, Bb);
    invBb += scb * 2.0 * K.c * inv_B;
    for (int i = 0; i < 3; ++i) {
        Bb[i] += bb[i] * inv_B;
        invBb += bb[i] * Bv[i];
    }
    Bmb += -invBb * inv_B * inv_B;
    for (int i = 0; i < 3; ++i) Bb[i] += Bmb * b[i];
}

GCB_HD void local_vjp(const SampleD& s, const KD& K, const LocalBar& Lb, SampleBar& sb) {
    const double G[2][3] = {{s.dBx[0], s.dBx[1], s.dBx[2]}, {s.dBy[0], s.dBy[1], s.dBy[2]}};
    double Eb[3], Bb[3], Gb[2][3];
    local_vjp_nd<2>(s.E, s.B, G, K, Lb, Eb, Bb, Gb);
    for (int i = 0; i < 3; ++i) {
        sb.E[i] += Eb[i];
        sb.B[i] += Bb[i];
        sb.dBx[i] += Gb[0][i];
        sb.dBy[i] += Gb[1][i];
    }
}

// ---------------------------------------------------------------------------
// Gamma, curvature drift, drift terms

// the gyration state of the differentiated step: mu conserved (the adjoint
// serves the paper's eq. dmudt only)
GCB_HD Gyr<double> conserved_mu(double mu) { return Gyr<double>{mu, 0.0, false}; }

GCB_HD void gamma_vjp(const LocalD& L, double upar, double mu, const KD& K, double Gb,
                      LocalBar& Lb, double& uparb, double& mub) {
    const double uperp2 = ((2.0 * mu) * L.B) * L.kappa;
    const double s = sqrt(1.0 + (upar * upar + uperp2) * K.inv_c2);
    Lb.kappa += Gb * s;
    const double argb = Gb * L.kappa / (2.0 * s);
    uparb += argb * 2.0 * upar * K.inv_c2;
    const double u2b = argb * K.inv_c2;
    mub += u2b * 2.0 * L.B * L.kappa;
    Lb.B += u2b * 2.0 * mu * L.kappa;
    Lb.kappa += u2b * 2.0 * mu * L.B;
}

GCB_HD void vcurv_vjp(const LocalD& L, double upar, double gam, double inv_qm, const KD& K,
                      const double vcb[3], LocalBar& Lb, double& uparb, double& gamb) {
    const double pre = ((K.c * L.kappa) * L.kappa) * (L.inv_B * inv_qm);
    const double a1 = (upar * upar) / gam;
    const double w[3] = {a1 * L.bgb[0] + upar * L.vgb[0], a1 * L.bgb[1] + upar * L.vgb[1],
                         a1 * L.bgb[2] + upar * L.vgb[2]};
    const double z[3] = {L.b[1] * w[2] - L.b[2] * w[1], L.b[2] * w[0] - L.b[0] * w[2],
                         L.b[0] * w[1] - L.b[1] * w[0]};
    const double preb = (vcb[0] * z[0] + vcb[1] * z[1]) + vcb[2] * z[2];
    const double zb[3] = {pre * vcb[0], pre * vcb[1], pre * vcb[2]};
    double wb[3] = {0.0, 0.0, 0.0};
    cross_vjp(L.b, w, zb, Lb.b, wb);
    const double a1b = (wb[0] * L.bgb[0] + wb[1] * L.bgb[1]) + wb[2] * L.bgb[2];
    for (int i = 0; i < 3; ++i) {
        Lb.bgb[i] += a1 * wb[i];
        Lb.vgb[i] += upar * wb[i];
    }
    uparb += (wb[0] * L.vgb[0] + wb[1] * L.vgb[1]) + wb[2] * L.vgb[2];
    uparb += a1b * 2.0 * upar / gam;
    gamb += -a1b * a1 / gam;
    Lb.kappa += preb * 2.0 * K.c * L.kappa * L.inv_B * inv_qm;
    Lb.inv_B += preb * K.c * L.kappa * L.kappa * inv_qm;
}

GCB_HD void drift_vjp(const LocalD& L, double upn, double mu, double inv_qm, bool curv,
                      const KD& K, const double Fb[2], LocalBar& Lb, double& upnb,
                      double& mub) {
    const double g = gamma_gca(L, upn, conserved_mu(mu), K);
    const double a = upn / g;
    const double ab = Fb[0] * L.b[0] + Fb[1] * L.b[1];
    Lb.b[0] += a * Fb[0];
    Lb.b[1] += a * Fb[1];
    Lb.vE[0] += Fb[0];
    Lb.vE[1] += Fb[1];
    double gb = -ab * a / g;
    upnb += ab / g;
    if (curv) {
        const double vcb[3] = {Fb[0], Fb[1], 0.0};
        vcurv_vjp(L, upn, g, inv_qm, K, vcb, Lb, upnb, gb);
    }
    gamma_vjp(L, upn, mu, K, gb, Lb, upnb, mub);
}

// ---------------------------------------------------------------------------
// parallel update

GCB_HD void parallel_vjp(const LocalD& Ln, double upar, double mu, double qm, bool curv,
                         const KD& K, double upnb, LocalBar& Lb, double& uparb, double& mub) {
    const double dtqm = qm * K.dt;
    if (!curv) {
        uparb += upnb;
        Lb.Epar += dtqm * upnb;
        return;
    }
    const double h = K.h;
    const double A = Ln.A, C = Ln.C;
    const double G0 = gamma_gca(Ln, upar, conserved_mu(mu), K);
    const double upr = (upar * (1.0 + h * A) + dtqm * Ln.Epar) + (h * G0) * C;
    const double D = 1.0 - h * A;
    const double DD = D * D;
    const double kap = Ln.kappa;
    const double k1 = (h * h) * (C * C) - (K.c2 * DD) / (kap * kap);
    const double k2 = (upr * K.dt) * C;
    const double u2 = ((2.0 * mu) * Ln.B) * kap;
    const double k3 = upr * upr + (K.c2 + u2) * DD;
    const double disc = k2 * k2 - (4.0 * k1) * k3;
    const bool dok = fabs(D) >= kDFloor;
    bool ok = (k1 < 0.0) && (disc >= 0.0) && dok;
    const double sq = sqrt(disc >= 0.0 ? disc : 0.0);
    const bool pos_k2 = k2 >= 0.0;
    const double num = pos_k2 ? k2 + sq : 2.0 * k3;
    double den = pos_k2 ? -2.0 * k1 : sq - k2;
    den = (ok && den > 0.0) ? den : 1.0;
    const double gp = num / den;
    ok = ok && (gp > 0.0) && __builtin_isfinite(gp);
    if (!ok && !dok) {
        uparb += upnb;
        Lb.Epar += dtqm * upnb;
        return;
    }
    double uprb, Db, Cb = 0.0;
    if (ok) {
        const double upn = (upr + (h * gp) * C) / D;
        uprb = upnb / D;
        const double gpb = upnb * h * C / D;
        Cb += upnb * h * gp / D;
        Db = -upnb * upn / D;
        const double dP = 2.0 * k1 * gp + k2;
        const double k1b = -gpb * gp * gp / dP;
        const double k2b = -gpb * gp / dP;
        const double k3b = -gpb / dP;
        uprb += k3b * 2.0 * upr;
        double DDb = k3b * (K.c2 + u2);
        const double u2b = k3b * DD;
        mub += u2b * 2.0 * Ln.B * kap;
        Lb.B += u2b * 2.0 * mu * kap;
        Lb.kappa += u2b * 2.0 * mu * Ln.B;
        uprb += k2b * K.dt * C;
        Cb += k2b * upr * K.dt;
        Cb += k1b * 2.0 * (h * h) * C;
        DDb += -k1b * K.c2 / (kap * kap);
        Lb.kappa += k1b * 2.0 * K.c2 * DD / (kap * kap * kap);
        Db += DDb * 2.0 * D;
    } else {
        // fallback: Gamma taken at u'/D (no implicit term)
        const double v = upr / D;
        const double gfb = gamma_gca(Ln, v, conserved_mu(mu), K);
        const double upn = (upr + (h * gfb) * C) / D;
        uprb = upnb / D;
        const double gfbb = upnb * h * C / D;
        Cb += upnb * h * gfb / D;
        Db = -upnb * upn / D;
        double vb = 0.0;
        gamma_vjp(Ln, v, mu, K, gfbb, Lb, vb, mub);
        uprb += vb / D;
        Db += -vb * v / D;
    }
    Lb.A += -h * Db;
    uparb += uprb * (1.0 + h * A);
    Lb.A += uprb * upar * h;
    Lb.Epar += uprb * dtqm;
    const double G0b = uprb * h * C;
    Cb += uprb * h * G0;
    Lb.C += Cb;
    gamma_vjp(Ln, upar, mu, K, G0b, Lb, uparb, mub);
}

// ---------------------------------------------------------------------------
// steps.  st[7] = (x, y, xp, yp, ux, uy, uz) at the step start; lam[7] holds
// the cotangents of the step outputs on entry and of its inputs on return.

template <bool kYee, class Acc, class Sink>
GCB_HD void boris_step_vjp(const Acc& acc, Sink& sink, const PushConst& pc, const KD& K,
                           const double st[7], double qm, double lam[7]) {
    const double x = st[0], y = st[1];
    SampleD s;
    gather<double, false, kYee>(acc, pc, K, x, y, s);
    const double* E = s.E;
    const double* Bv = s.B;
    const double u[3] = {st[4], st[5], st[6]};
    // forward
    const double hq = (qm * K.dt) * 0.5;
    const double um[3] = {u[0] + hq * E[0], u[1] + hq * E[1], u[2] + hq * E[2]};
    const double gm = gamma_full(um[0], um[1], um[2], K);
    const double f = hq / (K.c * gm);
    const double t[3] = {f * Bv[0], f * Bv[1], f * Bv[2]};
    const double t2 = (t[0] * t[0] + t[1] * t[1]) + t[2] * t[2];
    const double g = 2.0 / (1.0 + t2);
    const double sv[3] = {g * t[0], g * t[1], g * t[2]};
    const double up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]),
                          um[1] + (um[2] * t[0] - um[0] * t[2]),
                          um[2] + (um[0] * t[1] - um[1] * t[0])};
    const double un[3] = {um[0] + (up[1] * sv[2] - up[2] * sv[1]) + hq * E[0],
                          um[1] + (up[2] * sv[0] - up[0] * sv[2]) + hq * E[1],
                          um[2] + (up[0] * sv[1] - up[1] * sv[0]) + hq * E[2]};
    const double gn = gamma_full(un[0], un[1], un[2], K);
    const double ig = 1.0 / gn;
    // reverse
    const double xnb = lam[0], ynb = lam[1];
    double unb[3] = {lam[4] + pc.dt * ig * xnb, lam[5] + pc.dt * ig * ynb, lam[6]};
    const double igb = pc.dt * (un[0] * xnb + un[1] * ynb);
    const double gnb = -igb * ig * ig;
    for (int i = 0; i < 3; ++i) unb[i] += gnb * un[i] * K.inv_c2 / gn;
    SampleBar sb;
    zero(sb);
    // un = uq + hq E, uq = um + up x s
    for (int i = 0; i < 3; ++i) sb.E[i] += hq * unb[i];
    double umb[3] = {unb[0], unb[1], unb[2]};
    double upb[3] = {0.0, 0.0, 0.0}, svb[3] = {0.0, 0.0, 0.0};
    cross_vjp(up, sv, unb, upb, svb);
    // up = um + um x t
    double tb[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 3; ++i) umb[i] += upb[i];
    cross_vjp(um, t, upb, umb, tb);
    // s = g t
    const double gb = (svb[0] * t[0] + svb[1] * t[1]) + svb[2] * t[2];
    for (int i = 0; i < 3; ++i) tb[i] += g * svb[i];
    const double t2b = -gb * g * g * 0.5;
    for (int i = 0; i < 3; ++i) tb[i] += 2.0 * t[i] * t2b;
    // t = f B
    const double fb = (tb[0] * Bv[0] + tb[1] * Bv[1]) + tb[2] * Bv[2];
    for (int i = 0; i < 3; ++i) sb.B[i] += f * tb[i];
    const double gmb = -fb * f / gm;
    for (int i = 0; i < 3; ++i) umb[i] += gmb * um[i] * K.inv_c2 / gm;
    // um = u + hq E
    for (int i = 0; i < 3; ++i) sb.E[i] += hq * umb[i];
    double Xb = xnb + lam[2], Yb = ynb + lam[3];
    gather_vjp(acc, sink, pc, kYee, x, y, sb, Xb, Yb);
    lam[0] = Xb;
    lam[1] = Yb;
    lam[2] = 0.0;
    lam[3] = 0.0;
    lam[4] = umb[0];
    lam[5] = umb[1];
    lam[6] = umb[2];
}

// local quantities at a point, with the sample kept for local_vjp
template <bool kYee, class Acc>
GCB_HD void local_at(const Acc& acc, const PushConst& pc, const KD& K, double X, double Y,
                     SampleD& s, LocalD& L) {
    gather<double, true, kYee>(acc, pc, K, X, Y, s);
    local_from_sample(s, K, L);
}

template <bool kYee, class Acc, class Sink>
GCB_HD void local_bar_to_position(const Acc& acc, Sink& sink, const PushConst& pc,
                                  const KD& K, const SampleD& s, double X, double Y,
                                  const LocalBar& Lb, double& Xb, double& Yb) {
    SampleBar sb;
    zero(sb);
    local_vjp(s, K, Lb, sb);
    gather_vjp(acc, sink, pc, kYee, X, Y, sb, Xb, Yb);
}

constexpr int kMaxAdjIter = 8;   // fixed-point iterations the adjoint supports

// Field samples of the forward recomputation that the reverse sweep takes
// again instead of gathering them a second time: slot 0 is R^{n-1/2}, slot 1
// R^n, slot 1 + k the iterate R^k; `put` may drop a slot, and `get` then
// says so.  NoSamples keeps none.
struct NoSamples {
    GCB_HD void put(int, const SampleD&) {}
    GCB_HD bool get(int, SampleD&) const { return false; }
};

// local quantities at a point, from a kept sample when there is one
template <bool kYee, class Acc, class Keep>
GCB_HD void local_again(const Acc& acc, const Keep& keep, int slot, const PushConst& pc,
                        const KD& K, double X, double Y, SampleD& s, LocalD& L) {
    if (keep.get(slot, s))
        local_from_sample(s, K, L);
    else
        local_at<kYee>(acc, pc, K, X, Y, s, L);
}

// Number of gather points whose cotangents gca_step_vjp hands to its sink:
// R^{n+1/2}, the iterates R^1..R^{K-1}, R^n and R^{n-1/2}.
GCB_HD int gca_vjp_samples(int n_iter) {
    const int Kit = n_iter < kMaxAdjIter ? n_iter : kMaxAdjIter;
    return (Kit > 1 ? Kit - 1 : 0) + 3;
}

template <bool kYee, class Acc, class Sink, class Keep = NoSamples>
GCB_HD void gca_step_vjp(const Acc& acc, Sink& sink, const PushConst& pc, const KD& K,
                         const double st[7], double qm, double lam[7], Keep keep = Keep()) {
    const bool curv = pc.curvature != 0;
    const double x = st[0], y = st[1];
    const double ux = st[4], uy = st[5], uz = st[6];
    const double inv_qm = 1.0 / qm;
    const double h = K.h;
    const int Kit = pc.n_iter < kMaxAdjIter ? pc.n_iter : kMaxAdjIter;

    // ---- forward recomputation (values the reverse sweep needs)
    const double Rhx = x - 0.5 * min_image(x - st[2], pc.Lx);
    const double Rhy = y - 0.5 * min_image(y - st[3], pc.Ly);
    double upar, mu, gf, nu, up[3], bp[3], vch[3] = {0.0, 0.0, 0.0};
    {
        SampleD s;
        LocalD L;
        local_at<kYee>(acc, pc, K, Rhx, Rhy, s, L);
        keep.put(0, s);
        upar = (ux * L.b[0] + uy * L.b[1]) + uz * L.b[2];
        gf = gamma_full(ux, uy, uz, K);
        if (curv) v_curv(L, upar, gf, inv_qm, K, vch);
        up[0] = (ux - upar * L.b[0]) - (L.vE[0] + vch[0]) * gf;
        up[1] = (uy - upar * L.b[1]) - (L.vE[1] + vch[1]) * gf;
        up[2] = (uz - upar * L.b[2]) - (L.vE[2] + vch[2]) * gf;
        const double up2 = (up[0] * up[0] + up[1] * up[1]) + up[2] * up[2];
        mu = ((0.5 * up2) * L.inv_B) / L.kappa;
        nu = sqrt(up2);
        const double inv_nu = nu > 0.0 ? 1.0 / nu : 0.0;
        for (int i = 0; i < 3; ++i) bp[i] = up[i] * inv_nu;
    }
    double upn, Fn[2];
    {
        SampleD s;
        LocalD L;
        local_at<kYee>(acc, pc, K, x, y, s, L);
        keep.put(1, s);
        uint32_t fl = 0;
        upn = parallel_update(L, upar, conserved_mu(mu), qm, curv, K, fl);
        drift_terms(L, upn, conserved_mu(mu), inv_qm, curv, K, Fn[0], Fn[1]);
    }
    double Rk[kMaxAdjIter + 1][2];
    Rk[0][0] = x;
    Rk[0][1] = y;
    for (int k = 0; k < Kit; ++k) {
        double F[2];
        if (k == 0) {
            F[0] = Fn[0];
            F[1] = Fn[1];
        } else {
            SampleD s;
            LocalD L;
            local_at<kYee>(acc, pc, K, Rk[k][0], Rk[k][1], s, L);
            keep.put(1 + k, s);
            drift_terms(L, upn, conserved_mu(mu), inv_qm, curv, K, F[0], F[1]);
        }
        Rk[k + 1][0] = x + h * (Fn[0] + F[0]);
        Rk[k + 1][1] = y + h * (Fn[1] + F[1]);
    }
    const double Rmx = x + 0.5 * (Rk[Kit][0] - x);
    const double Rmy = y + 0.5 * (Rk[Kit][1] - y);

    // ---- reverse sweep
    double xb = lam[2], yb = lam[3];   // xp_out = x
    double RKb[2] = {lam[0], lam[1]};  // x_out = wrap(R^K)
    const double ub[3] = {lam[4], lam[5], lam[6]};
    double upnb = 0.0, mub = 0.0, bpb[3] = {0.0, 0.0, 0.0};

    // 5. reconstruction at R^{n+1/2}
    {
        SampleD s;
        LocalD L;
        local_at<kYee>(acc, pc, K, Rmx, Rmy, s, L);
        LocalBar Lb;
        zero(Lb);
        const double gr = gamma_gca(L, upn, conserved_mu(mu), K);
        double vc[3] = {0.0, 0.0, 0.0};
        if (curv) v_curv(L, upn, gr, inv_qm, K, vc);
        const double um = sqrt(((2.0 * mu) * L.B) * L.kappa);
        upnb += (ub[0] * L.b[0] + ub[1] * L.b[1]) + ub[2] * L.b[2];
        double vcb[3], grb = 0.0, umb = 0.0;
        for (int i = 0; i < 3; ++i) {
            Lb.b[i] += upn * ub[i];
            Lb.vE[i] += gr * ub[i];
            vcb[i] = gr * ub[i];
            grb += (L.vE[i] + vc[i]) * ub[i];
            umb += bp[i] * ub[i];
            bpb[i] += um * ub[i];
        }
        if (um > 0.0) {
            const double Xb_ = umb / (2.0 * um);
            mub += Xb_ * 2.0 * L.B * L.kappa;
            Lb.B += Xb_ * 2.0 * mu * L.kappa;
            Lb.kappa += Xb_ * 2.0 * mu * L.B;
        }
        if (curv) vcurv_vjp(L, upn, gr, inv_qm, K, vcb, Lb, upnb, grb);
        gamma_vjp(L, upn, mu, K, grb, Lb, upnb, mub);
        double Rmb[2] = {0.0, 0.0};
        local_bar_to_position<kYee>(acc, sink, pc, K, s, Rmx, Rmy, Lb, Rmb[0], Rmb[1]);
        xb += 0.5 * Rmb[0];
        yb += 0.5 * Rmb[1];
        RKb[0] += 0.5 * Rmb[0];
        RKb[1] += 0.5 * Rmb[1];
    }

    // 4. fixed-point iterations in reverse order
    double Fnb[2] = {0.0, 0.0};
    double Rb[2] = {RKb[0], RKb[1]};
    for (int k = Kit - 1; k >= 0; --k) {
        xb += Rb[0];
        yb += Rb[1];
        Fnb[0] += h * Rb[0];
        Fnb[1] += h * Rb[1];
        const double Fkb[2] = {h * Rb[0], h * Rb[1]};
        if (k == 0) {
            Fnb[0] += Fkb[0];
            Fnb[1] += Fkb[1];
            Rb[0] = Rb[1] = 0.0;
        } else {
            SampleD s;
            LocalD L;
            local_again<kYee>(acc, keep, 1 + k, pc, K, Rk[k][0], Rk[k][1], s, L);
            LocalBar Lb;
            zero(Lb);
            drift_vjp(L, upn, mu, inv_qm, curv, K, Fkb, Lb, upnb, mub);
            double nb[2] = {0.0, 0.0};
            local_bar_to_position<kYee>(acc, sink, pc, K, s, Rk[k][0], Rk[k][1], Lb, nb[0],
                                        nb[1]);
            Rb[0] = nb[0];
            Rb[1] = nb[1];
        }
    }

    // 3.-2. drift at R^n and the parallel update
    double uparb = 0.0;
    {
        SampleD s;
        LocalD L;
        local_again<kYee>(acc, keep, 1, pc, K, x, y, s, L);
        LocalBar Lb;
        zero(Lb);
        drift_vjp(L, upn, mu, inv_qm, curv, K, Fnb, Lb, upnb, mub);
        parallel_vjp(L, upar, mu, qm, curv, K, upnb, Lb, uparb, mub);
        local_bar_to_position<kYee>(acc, sink, pc, K, s, x, y, Lb, xb, yb);
    }

    // 1. decomposition at R^{n-1/2}
    double uxb = 0.0, uyb = 0.0, uzb = 0.0, xpb = 0.0, ypb = 0.0;
    {
        SampleD s;
        LocalD L;
        local_again<kYee>(acc, keep, 0, pc, K, Rhx, Rhy, s, L);
        LocalBar Lb;
        zero(Lb);
        double upb[3] = {0.0, 0.0, 0.0};
        if (nu > 0.0) {
            const double d = (bp[0] * bpb[0] + bp[1] * bpb[1]) + bp[2] * bpb[2];
            for (int i = 0; i < 3; ++i) upb[i] += (bpb[i] - bp[i] * d) / nu;
        }
        const double up2 = nu * nu;
        const double up2b = mub * 0.5 * L.inv_B / L.kappa;
        Lb.inv_B += mub * 0.5 * up2 / L.kappa;
        Lb.kappa += -mub * mu / L.kappa;
        for (int i = 0; i < 3; ++i) upb[i] += 2.0 * up[i] * up2b;
        double gfb = 0.0, vcb[3];
        const double u[3] = {ux, uy, uz};
        double uvb[3] = {upb[0], upb[1], upb[2]};
        for (int i = 0; i < 3; ++i) {
            uparb += -L.b[i] * upb[i];
            Lb.b[i] += -upar * upb[i];
            Lb.vE[i] += -gf * upb[i];
            vcb[i] = -gf * upb[i];
            gfb += -(L.vE[i] + vch[i]) * upb[i];
        }
        if (curv) vcurv_vjp(L, upar, gf, inv_qm, K, vcb, Lb, uparb, gfb);
        for (int i = 0; i < 3; ++i) {
            uvb[i] += gfb * u[i] * K.inv_c2 / gf;
            uvb[i] += uparb * L.b[i];
            Lb.b[i] += uparb * u[i];
        }
        double Rhb[2] = {0.0, 0.0};
        local_bar_to_position<kYee>(acc, sink, pc, K, s, Rhx, Rhy, Lb, Rhb[0], Rhb[1]);
        xb += 0.5 * Rhb[0];
        yb += 0.5 * Rhb[1];
        xpb += 0.5 * Rhb[0];
        ypb += 0.5 * Rhb[1];
        uxb = uvb[0];
        uyb = uvb[1];
        uzb = uvb[2];
    }
    lam[0] = xb;
    lam[1] = yb;
    lam[2] = xpb;
    lam[3] = ypb;
    lam[4] = uxb;
    lam[5] = uyb;
    lam[6] = uzb;
}

}  // namespace adj
}  // namespace gcb
