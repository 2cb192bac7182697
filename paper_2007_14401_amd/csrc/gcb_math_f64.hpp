// Per-particle arithmetic of the coupled guiding-center / Boris pusher in
// binary64 (device code).  Every expression is evaluated in a fixed order
// with separate multiplies and adds (translation units including this header
// are compiled with -ffp-contract=off), so results are reproducible bit for
// bit.  The field source is a template parameter: the same arithmetic serves
// gathers from the LDS tile window and from global memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gcb_access.hpp"
#include "gcb_common.hpp"

namespace gcb {

// ---------------------------------------------------------------------------
// Gather (Sec. 4, opening paragraph): linear shape function on the 2x2 nodes
// of each component's own lattice; gradients by differentiating it.

struct Sample {
    double E[3], B[3];
    double dBx[3], dBy[3];   // d B_i / dx, d B_i / dy
};

// One component at grid coordinates (gx, gy) = (X/dx, Y/dy) with lattice
// offset (sx, sy) in cells.
template <bool kGrad, class Acc>
__device__ __forceinline__ void interp_comp(const Acc& acc, int k, double gx, double gy,
                                            double sx, double sy, double inv_dx,
                                            double inv_dy, double& val, double& ddx,
                                            double& ddy) {
    const double xi = gx - sx;
    const double eta = gy - sy;
    const double fi = floor(xi);
    const double fj = floor(eta);
    const double wx = xi - fi;
    const double wy = eta - fj;
    double f00, f10, f01, f11;
    acc.quad(k, (int)fi, (int)fj, f00, f10, f01, f11);
    const double ax = 1.0 - wx;
    const double ay = 1.0 - wy;
    val = (((ax * ay) * f00 + (wx * ay) * f10) + (ax * wy) * f01) + (wx * wy) * f11;
    if (kGrad) {
        ddx = (ay * (f10 - f00) + wy * (f11 - f01)) * inv_dx;
        ddy = (ax * (f01 - f00) + wx * (f11 - f10)) * inv_dy;
    }
}

// The six components from four located 2x2 stencils (2D Yee lattice): the
// same operations as interp_comp, with the floor/weight computations shared
// by the components of one weight set.
template <bool kGrad, class Loader>
__device__ __forceinline__ void interp_yee(const Loader& ld, const double wx[2],
                                           const double wy[2], double inv_dx, double inv_dy,
                                           Sample& s) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int set = kYeeSet[k];
        const double ax = 1.0 - wx[set & 1];
        const double ay = 1.0 - wy[set >> 1];
        const double bx = wx[set & 1];
        const double by = wy[set >> 1];
        double f00, f10, f01, f11;
        ld.load4(set, k, f00, f10, f01, f11);
        const double val =
            (((ax * ay) * f00 + (bx * ay) * f10) + (ax * by) * f01) + (bx * by) * f11;
        if (k < 3) {
            s.E[k] = val;
        } else {
            s.B[k - 3] = val;
            if (kGrad) {
                s.dBx[k - 3] = (ay * (f10 - f00) + by * (f11 - f01)) * inv_dx;
                s.dBy[k - 3] = (ax * (f01 - f00) + bx * (f11 - f10)) * inv_dy;
            }
        }
    }
}

template <bool kGrad, typename T>
__device__ __forceinline__ void yee_fetch(const GlobalAcc<T>& acc, int ia, int ib, int ja,
                                          int jb, const double wx[2], const double wy[2],
                                          const PushConst& pc, Sample& s) {
    typename GlobalAcc<T>::Loc g;
    acc.locate(ia, ib, ja, jb, g);
    interp_yee<kGrad>(GlobalLoad<T>{g}, wx, wy, pc.inv_dx, pc.inv_dy, s);
}

template <bool kGrad, typename T>
__device__ __forceinline__ void yee_fetch(const TileAcc<T>& acc, int ia, int ib, int ja,
                                          int jb, const double wx[2], const double wy[2],
                                          const PushConst& pc, Sample& s) {
    int off[4];
    typename GlobalAcc<T>::Loc g;
    if (acc.locate(ia, ib, ja, jb, off, g))
        interp_yee<kGrad>(LdsLoad<T>{acc.lds, off, acc.W * 6}, wx, wy, pc.inv_dx, pc.inv_dy,
                          s);
    else
        interp_yee<kGrad>(GlobalLoad<T>{g}, wx, wy, pc.inv_dx, pc.inv_dy, s);
}

// All six components at (X, Y); B gradients when kGrad.  kYee: the 2D Yee
// offsets (the values of the runtime table when it holds them).
template <bool kGrad, bool kYee, class Acc>
__device__ __forceinline__ void gather(const Acc& acc, const PushConst& pc, double X,
                                       double Y, Sample& s) {
    const double gx = X * pc.inv_dx;
    const double gy = Y * pc.inv_dy;
    if constexpr (kYee) {
        // lattice coordinate minus the offset: offset 0 leaves it unchanged
        const double xb = gx - 0.5;
        const double yb = gy - 0.5;
        const double fxa = floor(gx), fxb = floor(xb);
        const double fya = floor(gy), fyb = floor(yb);
        const double wx[2] = {gx - fxa, xb - fxb};
        const double wy[2] = {gy - fya, yb - fyb};
        yee_fetch<kGrad>(acc, (int)fxa, (int)fxb, (int)fya, (int)fyb, wx, wy, pc, s);
    } else {
        double d0, d1;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            interp_comp<false>(acc, k, gx, gy, pc.stagger[k][0], pc.stagger[k][1],
                               pc.inv_dx, pc.inv_dy, s.E[k], d0, d1);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            interp_comp<kGrad>(acc, k + 3, gx, gy, pc.stagger[k + 3][0], pc.stagger[k + 3][1],
                               pc.inv_dx, pc.inv_dy, s.B[k], s.dBx[k], s.dBy[k]);
    }
}

// ---------------------------------------------------------------------------
// Local guiding-center quantities (Sec. 2.2): b, v_E = c E x B / B^2,
// kappa = (1 - v_E^2/c^2)^(-1/2), E_par, d_j b_i by the chain rule,
// (b.grad)b, (v_E.grad)b, A = v_E.(b.grad)b, C = v_E.(v_E.grad)b.

struct Local {
    double B, inv_B;
    double b[3], vE[3];
    double kappa, Epar;
    double bgb[3], vgb[3];
    double A, C;
};

__device__ __forceinline__ uint32_t local_from_sample(const Sample& s, const PushConst& pc,
                                                      Local& L) {
    uint32_t flags = 0;
    const double Ex = s.E[0], Ey = s.E[1], Ez = s.E[2];
    const double Bx = s.B[0], By = s.B[1], Bz = s.B[2];
    const double B2 = (Bx * Bx + By * By) + Bz * Bz;
    const double B = sqrt(B2);
    const bool bzero = (B == 0.0);
    const double inv_B = bzero ? 0.0 : 1.0 / B;
    if (bzero) flags |= ST_BZERO;
    L.B = B;
    L.inv_B = inv_B;
    const double bx = Bx * inv_B, by = By * inv_B, bz = Bz * inv_B;
    L.b[0] = bx; L.b[1] = by; L.b[2] = bz;
    const double sc = pc.c * (inv_B * inv_B);
    const double vEx = sc * (Ey * Bz - Ez * By);
    const double vEy = sc * (Ez * Bx - Ex * Bz);
    const double vEz = sc * (Ex * By - Ey * Bx);
    L.vE[0] = vEx; L.vE[1] = vEy; L.vE[2] = vEz;
    const double vE2 = (vEx * vEx + vEy * vEy) + vEz * vEz;
    double om = 1.0 - vE2 * pc.inv_c2;
    if (om < kKappaFloor) {
        om = kKappaFloor;
        flags |= ST_KAPPA;
    }
    L.kappa = 1.0 / sqrt(om);
    L.Epar = (Ex * bx + Ey * by) + Ez * bz;
    // d_j b_i = (d_j B_i - b_i (b . d_j B)) / B
    const double dnx = (bx * s.dBx[0] + by * s.dBx[1]) + bz * s.dBx[2];
    const double dny = (bx * s.dBy[0] + by * s.dBy[1]) + bz * s.dBy[2];
    double dbx[3], dby[3];
    dbx[0] = (s.dBx[0] - bx * dnx) * inv_B;
    dbx[1] = (s.dBx[1] - by * dnx) * inv_B;
    dbx[2] = (s.dBx[2] - bz * dnx) * inv_B;
    dby[0] = (s.dBy[0] - bx * dny) * inv_B;
    dby[1] = (s.dBy[1] - by * dny) * inv_B;
    dby[2] = (s.dBy[2] - bz * dny) * inv_B;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        L.bgb[i] = bx * dbx[i] + by * dby[i];
        L.vgb[i] = vEx * dbx[i] + vEy * dby[i];
    }
    L.A = (vEx * L.bgb[0] + vEy * L.bgb[1]) + vEz * L.bgb[2];
    L.C = (vEx * L.vgb[0] + vEy * L.vgb[1]) + vEz * L.vgb[2];
    return flags;
}

// Gamma(R, u_par) = kappa sqrt(1 + (u_par^2 + 2 mu B kappa/m)/c^2)  (eq. lfacgca2)
__device__ __forceinline__ double gamma_gca(const Local& L, double upar, double mu,
                                            const PushConst& pc) {
    const double uperp2 = ((2.0 * mu) * L.B) * L.kappa;
    return L.kappa * sqrt(1.0 + (upar * upar + uperp2) * pc.inv_c2);
}

// Curvature drift (eq. curvdrift):
// (m c kappa^2 / (q B)) b x [ (u_par^2/Gamma)(b.grad)b + u_par (v_E.grad)b ]
__device__ __forceinline__ void v_curv(const Local& L, double upar, double gam,
                                       double inv_qm, const PushConst& pc, double vc[3]) {
    const double pre = ((pc.c * L.kappa) * L.kappa) * (L.inv_B * inv_qm);
    const double a1 = (upar * upar) / gam;
    const double w0 = a1 * L.bgb[0] + upar * L.vgb[0];
    const double w1 = a1 * L.bgb[1] + upar * L.vgb[1];
    const double w2 = a1 * L.bgb[2] + upar * L.vgb[2];
    vc[0] = pre * (L.b[1] * w2 - L.b[2] * w1);
    vc[1] = pre * (L.b[2] * w0 - L.b[0] * w2);
    vc[2] = pre * (L.b[0] * w1 - L.b[1] * w0);
}

// ---------------------------------------------------------------------------
// Switch (Sec. 3 criteria, Sec. 4.1): guiding center iff B > 0,
// rho~/dl < f_rho and E/B < f_E, with rho~ = c^2 Gamma / (|q/m| B).

__device__ __forceinline__ bool switch_gca(const double E[3], const double Bv[3], double ux,
                                           double uy, double uz, double qm,
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

// ---------------------------------------------------------------------------
// Periodic box

__device__ __forceinline__ double wrap(double x, double L) {
    double w = x - L * floor(x / L);
    if (w < 0.0) w = w + L;
    if (w >= L) w = w - L;
    return w;
}

__device__ __forceinline__ double min_image(double d, double L) {
    return d - L * floor(d / L + 0.5);
}

// ---------------------------------------------------------------------------
// Relativistic Boris push (Sec. 2.1), fields at x^n

__device__ __forceinline__ void boris(const double E[3], const double Bv[3], double& ux,
                                      double& uy, double& uz, double qm,
                                      const PushConst& pc) {
    const double hq = (qm * pc.dt) * 0.5;
    const double umx = ux + hq * E[0], umy = uy + hq * E[1], umz = uz + hq * E[2];
    const double gm = sqrt(1.0 + ((umx * umx + umy * umy) + umz * umz) * pc.inv_c2);
    const double f = hq / (pc.c * gm);
    const double tx = f * Bv[0], ty = f * Bv[1], tz = f * Bv[2];
    const double t2 = (tx * tx + ty * ty) + tz * tz;
    const double g = 2.0 / (1.0 + t2);
    const double sx = g * tx, sy = g * ty, sz = g * tz;
    const double upx = umx + (umy * tz - umz * ty);
    const double upy = umy + (umz * tx - umx * tz);
    const double upz = umz + (umx * ty - umy * tx);
    const double uqx = umx + (upy * sz - upz * sy);
    const double uqy = umy + (upz * sx - upx * sz);
    const double uqz = umz + (upx * sy - upy * sx);
    ux = uqx + hq * E[0];
    uy = uqy + hq * E[1];
    uz = uqz + hq * E[2];
}

// Full-orbit step: u^{n-1/2} -> u^{n+1/2}, x^{n+1} = x^n + dt u/Gamma.
__device__ __forceinline__ void boris_step(const Sample& s, ParticleRegs& r,
                                           const PushConst& pc) {
    boris(s.E, s.B, r.ux, r.uy, r.uz, r.qm, pc);
    const double gn = sqrt(1.0 + ((r.ux * r.ux + r.uy * r.uy) + r.uz * r.uz) * pc.inv_c2);
    const double inv_g = 1.0 / gn;
    const double xn = r.x + pc.dt * (r.ux * inv_g);
    const double yn = r.y + pc.dt * (r.uy * inv_g);
    r.xp = r.x;
    r.yp = r.y;
    r.x = wrap(xn, pc.Lx);
    r.y = wrap(yn, pc.Ly);
}

// ---------------------------------------------------------------------------
// Guiding-center leapfrog (Sec. 2.2.1 / 2.2.2) inside the coupled step (Sec. 3.1)

// u_par^{n-1/2} -> u_par^{n+1/2} at R^n.  With curvature: the positive root
// of k1 G^2 + k2 G + k3 = 0 for G = Gamma(R^n, u_par^{n+1/2}), evaluated
// without cancellation, then eq. dupardtcase2discsol.
__device__ __forceinline__ double parallel_update(const Local& Ln, double upar, double mu,
                                                  double qm, const PushConst& pc,
                                                  uint32_t& flags) {
    const double dtqm = qm * pc.dt;
    if (!pc.curvature) return upar + dtqm * Ln.Epar;
    const double h = 0.5 * pc.dt;
    const double A = Ln.A, C = Ln.C;
    const double G0 = gamma_gca(Ln, upar, mu, pc);
    const double upr = (upar * (1.0 + h * A) + dtqm * Ln.Epar) + (h * G0) * C;
    const double D = 1.0 - h * A;
    const double DD = D * D;
    const double k1 = (h * h) * (C * C) - (pc.c2 * DD) / (Ln.kappa * Ln.kappa);
    const double k2 = (upr * pc.dt) * C;
    const double k3 = upr * upr + (pc.c2 + ((2.0 * mu) * Ln.B) * Ln.kappa) * DD;
    const double disc = k2 * k2 - (4.0 * k1) * k3;
    const bool dok = fabs(D) >= kDFloor;
    bool ok = (k1 < 0.0) && (disc >= 0.0) && dok;
    const double sq = sqrt(disc >= 0.0 ? disc : 0.0);
    const bool pos_k2 = k2 >= 0.0;
    const double num = pos_k2 ? k2 + sq : 2.0 * k3;
    double den = pos_k2 ? -2.0 * k1 : sq - k2;
    den = (ok && den > 0.0) ? den : 1.0;
    const double gp = num / den;
    ok = ok && (gp > 0.0) && isfinite(gp);
    const double Ds = dok ? D : 1.0;
    if (ok) return (upr + (h * gp) * C) / Ds;
    flags |= ST_QUAD;
    if (dok) {
        const double gfb = gamma_gca(Ln, upr / Ds, mu, pc);
        return (upr + (h * gfb) * C) / Ds;
    }
    return upar + dtqm * Ln.Epar;
}

// x, y components of u_par b / Gamma + v_E + v_c at a point.
__device__ __forceinline__ void drift_terms(const Local& L, double upn, double mu,
                                            double inv_qm, const PushConst& pc,
                                            double& Fx, double& Fy) {
    const double g = gamma_gca(L, upn, mu, pc);
    const double a = upn / g;
    if (pc.curvature) {
        double vc[3];
        v_curv(L, upn, g, inv_qm, pc, vc);
        Fx = (a * L.b[0] + L.vE[0]) + vc[0];
        Fy = (a * L.b[1] + L.vE[1]) + vc[1];
    } else {
        Fx = a * L.b[0] + L.vE[0];
        Fy = a * L.b[1] + L.vE[1];
    }
}

__device__ __forceinline__ double nan_max(double a, double b) {
    if (a != a) return a;
    if (b != b) return b;
    return a > b ? a : b;
}

// One guiding-center step.  sn is the gather (with gradients) at x^n.
// Returns status flags; res receives |R^K - R^{K-1}|_inf.
template <bool kYee, class Acc>
__device__ __forceinline__ uint32_t gca_step(const Acc& acc, const Sample& sn,
                                             ParticleRegs& r, const PushConst& pc,
                                             double& res) {
    uint32_t flags = 0;
    const double x = r.x, y = r.y;
    const double ux = r.ux, uy = r.uy, uz = r.uz;
    const double inv_qm = 1.0 / r.qm;

    // 1. guiding-center variables at R^{n-1/2} = (x^n + x^{n-1})/2
    double upar, mu, bpx, bpy, bpz;
    {
        const double Rhx = x - 0.5 * min_image(x - r.xp, pc.Lx);
        const double Rhy = y - 0.5 * min_image(y - r.yp, pc.Ly);
        Sample sh;
        gather<true, kYee>(acc, pc, Rhx, Rhy, sh);
        Local Lh;
        flags |= local_from_sample(sh, pc, Lh);
        upar = (ux * Lh.b[0] + uy * Lh.b[1]) + uz * Lh.b[2];
        const double gf = sqrt(1.0 + ((ux * ux + uy * uy) + uz * uz) * pc.inv_c2);
        double vc[3] = {0.0, 0.0, 0.0};
        if (pc.curvature) v_curv(Lh, upar, gf, inv_qm, pc, vc);
        const double upx = (ux - upar * Lh.b[0]) - (Lh.vE[0] + vc[0]) * gf;
        const double upy = (uy - upar * Lh.b[1]) - (Lh.vE[1] + vc[1]) * gf;
        const double upz = (uz - upar * Lh.b[2]) - (Lh.vE[2] + vc[2]) * gf;
        const double up2 = (upx * upx + upy * upy) + upz * upz;
        mu = ((0.5 * up2) * Lh.inv_B) / Lh.kappa;
        const double nu = sqrt(up2);
        const double inv_nu = nu > 0.0 ? 1.0 / nu : 0.0;
        bpx = upx * inv_nu;
        bpy = upy * inv_nu;
        bpz = upz * inv_nu;
    }

    // 2.-3. local quantities at R^n = x^n and the parallel update
    double upn, Fnx, Fny;
    {
        Local Ln;
        flags |= local_from_sample(sn, pc, Ln);
        upn = parallel_update(Ln, upar, mu, r.qm, pc, flags);
        drift_terms(Ln, upn, mu, inv_qm, pc, Fnx, Fny);
    }

    // 4. R^{n+1}: K fixed-point iterations R^{k+1} = R^k - H(R^k), R^0 = R^n
    const double h = 0.5 * pc.dt;
    double Rx = x, Ry = y;
    res = 0.0;
    for (int k = 0; k < pc.n_iter; ++k) {
        double Fkx, Fky;
        if (k == 0) {
            Fkx = Fnx;
            Fky = Fny;
        } else {
            Sample sk;
            gather<true, kYee>(acc, pc, Rx, Ry, sk);
            Local Lk;
            flags |= local_from_sample(sk, pc, Lk);
            drift_terms(Lk, upn, mu, inv_qm, pc, Fkx, Fky);
        }
        const double Rx_new = x + h * (Fnx + Fkx);
        const double Ry_new = y + h * (Fny + Fky);
        res = nan_max(fabs(Rx_new - Rx), fabs(Ry_new - Ry));
        Rx = Rx_new;
        Ry = Ry_new;
    }
    if (res > pc.fp_tol) flags |= ST_FPRES;

    // 5. particle variables at R^{n+1/2} = (R^n + R^{n+1})/2, gyration
    //    direction held fixed
    {
        const double Rmx = x + 0.5 * (Rx - x);
        const double Rmy = y + 0.5 * (Ry - y);
        Sample sm;
        gather<true, kYee>(acc, pc, Rmx, Rmy, sm);
        Local Lm;
        flags |= local_from_sample(sm, pc, Lm);
        const double gr = gamma_gca(Lm, upn, mu, pc);
        double vc[3] = {0.0, 0.0, 0.0};
        if (pc.curvature) v_curv(Lm, upn, gr, inv_qm, pc, vc);
        const double um = sqrt(((2.0 * mu) * Lm.B) * Lm.kappa);
        r.ux = (upn * Lm.b[0] + (Lm.vE[0] + vc[0]) * gr) + um * bpx;
        r.uy = (upn * Lm.b[1] + (Lm.vE[1] + vc[1]) * gr) + um * bpy;
        r.uz = (upn * Lm.b[2] + (Lm.vE[2] + vc[2]) * gr) + um * bpz;
    }

    // 6. store
    r.xp = x;
    r.yp = y;
    r.x = wrap(Rx, pc.Lx);
    r.y = wrap(Ry, pc.Ly);
    return flags;
}

__device__ __forceinline__ uint32_t finite_flag(const ParticleRegs& r) {
    const bool ok = isfinite(r.x) && isfinite(r.y) && isfinite(r.ux) && isfinite(r.uy) &&
                    isfinite(r.uz);
    return ok ? 0u : (uint32_t)ST_NONFINITE;
}

}  // namespace gcb
