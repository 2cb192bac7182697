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
// (the unit is compiled with -ffp-contract=off), sin and cos come from the
// fixed polynomial below, and square roots and quotients are IEEE, so the
// step is reproducible operation by operation.
#pragma once

#include "gcb_common.hpp"

namespace gcb {
namespace gr {

constexpr uint8_t kStOut = 64;   // left the (r, theta) domain; no longer advanced

constexpr double kPi = 3.141592653589793;
constexpr double kTwoPi = 2.0 * kPi;

// ---------------------------------------------------------------------------
// sin and cos: Cody-Waite additive reduction by pi/2 with a two-part constant
// (first part 33 significant bits, so k * kPio2Hi is exact for small k) and
// Taylor polynomials of degree 19 (sin) and 20 (cos) on [-pi/4, pi/4], Horner
// form.  Within one unit in the last place of the correctly rounded values.

constexpr double kPio2Hi = 1.57079632673412561417e+00;
constexpr double kPio2Lo = 6.07710050650619224932e-11;

GCB_HD void sincos_poly(double th, double& sn, double& cs) {
    const double k = floor(th * (2.0 / kPi) + 0.5);
    const double y = (th - k * kPio2Hi) - k * kPio2Lo;
    const double z = y * y;
    double ps = -1.0 / 121645100408832000.0;           // -1/19!
    ps = ps * z + 1.0 / 355687428096000.0;             // 1/17!
    ps = ps * z + -1.0 / 1307674368000.0;              // -1/15!
    ps = ps * z + 1.0 / 6227020800.0;                  // 1/13!
    ps = ps * z + -1.0 / 39916800.0;                   // -1/11!
    ps = ps * z + 1.0 / 362880.0;                      // 1/9!
    ps = ps * z + -1.0 / 5040.0;                       // -1/7!
    ps = ps * z + 1.0 / 120.0;                         // 1/5!
    ps = ps * z + -1.0 / 6.0;                          // -1/3!
    const double s = y + (y * z) * ps;
    double pc = 1.0 / 2432902008176640000.0;           // 1/20!
    pc = pc * z + -1.0 / 6402373705728000.0;           // -1/18!
    pc = pc * z + 1.0 / 20922789888000.0;              // 1/16!
    pc = pc * z + -1.0 / 87178291200.0;                // -1/14!
    pc = pc * z + 1.0 / 479001600.0;                   // 1/12!
    pc = pc * z + -1.0 / 3628800.0;                    // -1/10!
    pc = pc * z + 1.0 / 40320.0;                       // 1/8!
    pc = pc * z + -1.0 / 720.0;                        // -1/6!
    pc = pc * z + 1.0 / 24.0;                          // 1/4!
    pc = pc * z + -1.0 / 2.0;                          // -1/2!
    const double c = 1.0 + z * pc;
    const int q = (int)((long long)k & 3);
    sn = q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c;
    cs = q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
}

// ---------------------------------------------------------------------------
// metric

struct Metric {
    double alpha, beta_r;
    double gu_rr, gu_rph, gu_thth, gu_phph;   // gamma^ij
    double gd_rr, gd_rph, gd_thth, gd_phph;   // gamma_ij
    double sqrtg;
    // d/dr, d/dtheta
    double dalpha[2], dbeta_r[2], dgu_rr[2], dgu_rph[2], dgu_thth[2], dgu_phph[2];
};

// Kerr (M = 1, spin a) in Kerr-Schild form: rho^2 = r^2 + a^2 cos^2,
// z = 2r/rho^2, alpha = (1+z)^-1/2, beta^r = z/(1+z),
// gamma_rr = 1+z, gamma_rphi = -a(1+z) sin^2, gamma_thth = rho^2,
// gamma_phph = sin^2 (rho^2 + a^2 (1+z) sin^2), and the inverse
// gamma^rr = 1/(1+z) + a^2 sin^2/rho^2, gamma^rphi = a/rho^2,
// gamma^thth = 1/rho^2, gamma^phph = 1/(rho^2 sin^2).
template <bool kDerivs>
GCB_HD void kerr_schild(double a, double r, double th, Metric& m) {
    const double a2 = a * a;
    double sn, cs;
    sincos_poly(th, sn, cs);
    const double s2 = sn * sn;
    const double c2 = cs * cs;
    const double rho2 = r * r + a2 * c2;
    const double z = (2.0 * r) / rho2;
    const double opz = 1.0 + z;
    const double sq = sqrt(opz);
    m.alpha = 1.0 / sq;
    m.beta_r = z / opz;
    m.gu_rr = 1.0 / opz + (a2 * s2) / rho2;
    m.gu_rph = a / rho2;
    m.gu_thth = 1.0 / rho2;
    m.gu_phph = 1.0 / (rho2 * s2);
    m.gd_rr = opz;
    m.gd_rph = -(a * opz) * s2;
    m.gd_thth = rho2;
    m.gd_phph = s2 * (rho2 + (a2 * opz) * s2);
    m.sqrtg = (sq * rho2) * sn;
    if (kDerivs) {
        const double sc = sn * cs;
        const double drho2[2] = {2.0 * r, -2.0 * (a2 * sc)};
        const double rho4 = rho2 * rho2;
        const double dz[2] = {(2.0 * (a2 * c2 - r * r)) / rho4, (4.0 * (r * (a2 * sc))) / rho4};
        const double opz2 = opz * opz;
        for (int i = 0; i < 2; ++i) {
            m.dalpha[i] = -0.5 * (m.alpha / opz) * dz[i];
            m.dbeta_r[i] = dz[i] / opz2;
            m.dgu_rph[i] = -(a * drho2[i]) / rho4;
            m.dgu_thth[i] = -drho2[i] / rho4;
        }
        m.dgu_rr[0] = -(dz[0] / opz2) - (a2 * s2) * drho2[0] / rho4;
        m.dgu_rr[1] = (-(dz[1] / opz2) + (a2 * (2.0 * sc)) / rho2) - (a2 * s2) * drho2[1] / rho4;
        const double rs2 = rho2 * s2;
        m.dgu_phph[0] = -(drho2[0] * s2) / (rs2 * rs2);
        m.dgu_phph[1] = -(drho2[1] * s2 + rho2 * (2.0 * sc)) / (rs2 * rs2);
    }
}

// ---------------------------------------------------------------------------
// fields on the (r, theta) grid: node-interleaved F[(j*(nr+1) + i)*6 + k],
// k = D^r, D^th, D^ph, B^r, B^th, B^ph at r_min + i dr, theta = j dth

struct GrConst {
    double a, dt, qm, f_rho, f_E, fp_tol;
    double r_min, r_max, inv_dr, inv_dth;
    int nr, nth, n_iter;
};

struct GrSample {
    double D[3], B[3];
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

template <typename T>
GCB_HD void grid_sample(const T* __restrict__ F, const GrConst& g, double r, double th,
                        GrSample& s) {
    int i, j;
    double wx, wy;
    grid_cell(g, r, th, i, j, wx, wy);
    const double ax = 1.0 - wx, ay = 1.0 - wy;
    const int W = g.nr + 1;
    const T* p0 = F + ((size_t)j * W + i) * 6;
    const T* p1 = p0 + (size_t)W * 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double f00 = (double)p0[k], f10 = (double)p0[6 + k];
        const double f01 = (double)p1[k], f11 = (double)p1[6 + k];
        const double v = ay * (ax * f00 + wx * f10) + wy * (ax * f01 + wx * f11);
        if (k < 3)
            s.D[k] = v;
        else
            s.B[k - 3] = v;
    }
}

GCB_HD bool inside(const GrConst& g, double r, double th) {
    return r >= g.r_min && r < g.r_max && th >= 0.0 && th <= kPi;
}

// ---------------------------------------------------------------------------
// index gymnastics

GCB_HD void lower(const Metric& m, const double V[3], double out[3]) {
    out[0] = m.gd_rr * V[0] + m.gd_rph * V[2];
    out[1] = m.gd_thth * V[1];
    out[2] = m.gd_rph * V[0] + m.gd_phph * V[2];
}

GCB_HD void raise(const Metric& m, const double w[3], double out[3]) {
    out[0] = m.gu_rr * w[0] + m.gu_rph * w[2];
    out[1] = m.gu_thth * w[1];
    out[2] = m.gu_rph * w[0] + m.gu_phph * w[2];
}

GCB_HD double norm2_cov(const Metric& m, const double w[3]) {
    double up[3];
    raise(m, w, up);
    return (w[0] * up[0] + w[1] * up[1]) + w[2] * up[2];
}

GCB_HD double norm2_con(const Metric& m, const double V[3]) {
    double lo[3];
    lower(m, V, lo);
    return (V[0] * lo[0] + V[1] * lo[1]) + V[2] * lo[2];
}

GCB_HD double gamma_of(const Metric& m, const double u[3]) {
    return sqrt(1.0 + norm2_cov(m, u));
}

GCB_HD double max_nan(double a, double b) { return (a > b || a != a) ? a : b; }

// ---------------------------------------------------------------------------
// local-frame half push: Lorentz force over dt/2 (Boris with step alpha dt/2)

GCB_HD void half_push(const Metric& m, const GrSample& f, double u[3], double qm, double dt) {
    const double L11 = sqrt(m.gd_rr);
    const double L22 = sqrt(m.gd_thth);
    const double L31 = m.gd_rph / L11;
    const double L33 = sqrt(m.gd_phph - L31 * L31);
    const double u1 = u[0] / L11;
    const double u2 = u[1] / L22;
    const double u3 = (u[2] - L31 * u1) / L33;
    const double D1 = L11 * f.D[0] + L31 * f.D[2], D2 = L22 * f.D[1], D3 = L33 * f.D[2];
    const double B1 = L11 * f.B[0] + L31 * f.B[2], B2 = L22 * f.B[1], B3 = L33 * f.B[2];
    const double hq = (qm * (m.alpha * (0.5 * dt))) * 0.5;
    const double umx = u1 + hq * D1, umy = u2 + hq * D2, umz = u3 + hq * D3;
    const double gm = sqrt(1.0 + ((umx * umx + umy * umy) + umz * umz));
    const double fq = hq / gm;
    const double tx = fq * B1, ty = fq * B2, tz = fq * B3;
    const double t2 = (tx * tx + ty * ty) + tz * tz;
    const double g = 2.0 / (1.0 + t2);
    const double sx = g * tx, sy = g * ty, sz = g * tz;
    const double upx = umx + (umy * tz - umz * ty);
    const double upy = umy + (umz * tx - umx * tz);
    const double upz = umz + (umx * ty - umy * tx);
    const double uqx = umx + (upy * sz - upz * sy);
    const double uqy = umy + (upz * sx - upx * sz);
    const double uqz = umz + (upx * sy - upy * sx);
    const double v1 = uqx + hq * D1, v2 = uqy + hq * D2, v3 = uqz + hq * D3;
    u[0] = L11 * v1;
    u[1] = L22 * v2;
    u[2] = L31 * v1 + L33 * v3;
}

// geodesic terms (Sec. 2.3): V^i = alpha gamma^ij u_j/Gamma - beta^i and
// G_i = -Gamma d_i alpha + u_j d_i beta^j - alpha u_j u_k d_i gamma^jk/(2 Gamma)
// for i = r, theta (G_phi = 0)
GCB_HD void geo_V(const Metric& m, const double u[3], double Gam, double V[3]) {
    double up[3];
    raise(m, u, up);
    const double ag = m.alpha / Gam;
    V[0] = ag * up[0] - m.beta_r;
    V[1] = ag * up[1];
    V[2] = ag * up[2];
}

GCB_HD void geo_G(const Metric& m, const double u[3], double Gam, double G[2]) {
    const double ur = u[0], ut = u[1], up = u[2];
    const double h = m.alpha / (2.0 * Gam);
    for (int i = 0; i < 2; ++i) {
        const double q = ((ur * ur) * m.dgu_rr[i] + (2.0 * (ur * up)) * m.dgu_rph[i]) +
                         ((ut * ut) * m.dgu_thth[i] + (up * up) * m.dgu_phph[i]);
        G[i] = (-(Gam * m.dalpha[i]) + ur * m.dbeta_r[i]) - h * q;
    }
}

// guiding-center quantities at a point
struct GcLocal {
    double B, kappa, Dpar;
    double b_up[3], b_dn[3], vE[3];
};

GCB_HD uint32_t gc_local(const Metric& m, const GrSample& f, GcLocal& L) {
    uint32_t flags = 0;
    double Bl[3];
    lower(m, f.B, Bl);
    const double B2 = (f.B[0] * Bl[0] + f.B[1] * Bl[1]) + f.B[2] * Bl[2];
    const double Bm = sqrt(B2);
    const bool bzero = Bm == 0.0;
    const double inv_B = bzero ? 0.0 : 1.0 / Bm;
    if (bzero) flags |= ST_BZERO;
    L.B = Bm;
    for (int i = 0; i < 3; ++i) {
        L.b_up[i] = f.B[i] * inv_B;
        L.b_dn[i] = Bl[i] * inv_B;
    }
    const double DxB[3] = {m.sqrtg * (f.D[1] * f.B[2] - f.D[2] * f.B[1]),
                           m.sqrtg * (f.D[2] * f.B[0] - f.D[0] * f.B[2]),
                           m.sqrtg * (f.D[0] * f.B[1] - f.D[1] * f.B[0])};
    const double ib2 = inv_B * inv_B;
    for (int i = 0; i < 3; ++i) L.vE[i] = DxB[i] * ib2;
    double om = 1.0 - norm2_cov(m, L.vE);
    if (om < kKappaFloor) {
        om = kKappaFloor;
        flags |= ST_KAPPA;
    }
    L.kappa = 1.0 / sqrt(om);
    L.Dpar = (f.D[0] * L.b_dn[0] + f.D[1] * L.b_dn[1]) + f.D[2] * L.b_dn[2];
    return flags;
}

// eq. grgcalfac with m = 1
GCB_HD double gamma_gc(const GcLocal& L, double upar, double mu) {
    return L.kappa * sqrt((1.0 + upar * upar) + ((2.0 * mu) * L.B) * L.kappa);
}

GCB_HD bool switch_gca(const Metric& m, const GrSample& f, const double u[3], double qm,
                       double dl, const GrConst& g) {
    const double Bm = sqrt(norm2_con(m, f.B));
    const double Dm = sqrt(norm2_con(m, f.D));
    const double Gam = gamma_of(m, u);
    const double safe = Bm > 0.0 ? Bm : 1.0;
    const double rho = Gam / (fabs(qm) * safe);
    return Bm > 0.0 && rho / dl < g.f_rho && Dm / safe < g.f_E;
}

GCB_HD double wrap_phi(double ph) {
    double w = ph - kTwoPi * floor(ph / kTwoPi);
    if (w < 0.0) w = w + kTwoPi;
    if (w >= kTwoPi) w = w - kTwoPi;
    return w;
}

// ---------------------------------------------------------------------------
// the two branches: x, u in/out; return flags, res = last position increment

template <typename T>
GCB_HD uint32_t greom_step(const T* __restrict__ F, const GrConst& g, double x[3], double u[3],
                           double qm, double& res) {
    Metric m0;
    kerr_schild<false>(g.a, x[0], x[1], m0);
    GrSample f0;
    grid_sample(F, g, x[0], x[1], f0);
    double u1[3] = {u[0], u[1], u[2]};
    half_push(m0, f0, u1, qm, g.dt);
    double xk[3] = {x[0], x[1], x[2]};
    double uk[3] = {u1[0], u1[1], u1[2]};
    res = 0.0;
    for (int k = 0; k < g.n_iter; ++k) {
        double xb[3], ub[3];
        for (int i = 0; i < 3; ++i) {
            xb[i] = 0.5 * (xk[i] + x[i]);
            ub[i] = 0.5 * (uk[i] + u1[i]);
        }
        Metric mb;
        kerr_schild<true>(g.a, xb[0], xb[1], mb);
        const double Gam = gamma_of(mb, ub);
        double V[3], G[2];
        geo_V(mb, ub, Gam, V);
        geo_G(mb, ub, Gam, G);
        double xn[3];
        for (int i = 0; i < 3; ++i) xn[i] = x[i] + g.dt * V[i];
        res = max_nan(max_nan(fabs(xn[0] - xk[0]), fabs(xn[1] - xk[1])), fabs(xn[2] - xk[2]));
        for (int i = 0; i < 3; ++i) xk[i] = xn[i];
        uk[0] = u1[0] + g.dt * G[0];
        uk[1] = u1[1] + g.dt * G[1];
        uk[2] = u1[2];
    }
    Metric m1;
    kerr_schild<false>(g.a, xk[0], xk[1], m1);
    GrSample f1;
    grid_sample(F, g, xk[0], xk[1], f1);
    half_push(m1, f1, uk, qm, g.dt);
    for (int i = 0; i < 3; ++i) {
        x[i] = xk[i];
        u[i] = uk[i];
    }
    return 0;
}

template <typename T>
GCB_HD uint32_t grgca_step(const T* __restrict__ F, const GrConst& g, double x[3], double u[3],
                           double qm, double& res) {
    Metric m0;
    kerr_schild<false>(g.a, x[0], x[1], m0);
    GrSample f0;
    grid_sample(F, g, x[0], x[1], f0);
    GcLocal L0;
    uint32_t flags = gc_local(m0, f0, L0);
    const double Gf = gamma_of(m0, u);
    const double upar = (L0.b_up[0] * u[0] + L0.b_up[1] * u[1]) + L0.b_up[2] * u[2];
    double uperp[3];
    for (int i = 0; i < 3; ++i) uperp[i] = (u[i] - upar * L0.b_dn[i]) - L0.vE[i] * Gf;
    const double up2 = norm2_cov(m0, uperp);
    double mu = ((0.5 * up2) / L0.B) / L0.kappa;
    if (!(L0.B > 0.0)) mu = 0.0;
    const double nu = sqrt(up2);
    const double inv_nu = nu > 0.0 ? 1.0 / nu : 0.0;
    double bperp[3];
    for (int i = 0; i < 3; ++i) bperp[i] = uperp[i] * inv_nu;
    const double p1 = upar + (qm * (m0.alpha * (0.5 * g.dt))) * L0.Dpar;
    double Rk[3] = {x[0], x[1], x[2]};
    double pk = p1;
    res = 0.0;
    for (int k = 0; k < g.n_iter; ++k) {
        double Rb[3];
        for (int i = 0; i < 3; ++i) Rb[i] = 0.5 * (Rk[i] + x[i]);
        const double pb = 0.5 * (pk + p1);
        Metric mb;
        kerr_schild<true>(g.a, Rb[0], Rb[1], mb);
        GrSample fb;
        grid_sample(F, g, Rb[0], Rb[1], fb);
        GcLocal Lb;
        flags |= gc_local(mb, fb, Lb);
        const double Gam = gamma_gc(Lb, pb, mu);
        double vu[3];
        raise(mb, Lb.vE, vu);
        double V[3];
        V[0] = mb.alpha * (pb * (Lb.b_up[0] / Gam) + vu[0]) - mb.beta_r;
        V[1] = mb.alpha * (pb * (Lb.b_up[1] / Gam) + vu[1]);
        V[2] = mb.alpha * (pb * (Lb.b_up[2] / Gam) + vu[2]);
        const double upg = sqrt(((2.0 * mu) * Lb.kappa) * Lb.B);
        double ub[3];
        for (int i = 0; i < 3; ++i) ub[i] = (pb * Lb.b_dn[i] + Lb.vE[i] * Gam) + upg * bperp[i];
        double G[2];
        geo_G(mb, ub, Gam, G);
        const double Gb = G[0] * Lb.b_up[0] + G[1] * Lb.b_up[1];
        double Rn[3];
        for (int i = 0; i < 3; ++i) Rn[i] = x[i] + g.dt * V[i];
        res = max_nan(max_nan(fabs(Rn[0] - Rk[0]), fabs(Rn[1] - Rk[1])), fabs(Rn[2] - Rk[2]));
        for (int i = 0; i < 3; ++i) Rk[i] = Rn[i];
        pk = p1 + g.dt * Gb;
    }
    Metric m1;
    kerr_schild<false>(g.a, Rk[0], Rk[1], m1);
    GrSample f1;
    grid_sample(F, g, Rk[0], Rk[1], f1);
    GcLocal L1;
    flags |= gc_local(m1, f1, L1);
    const double upar1 = pk + (qm * (m1.alpha * (0.5 * g.dt))) * L1.Dpar;
    const double Gam1 = gamma_gc(L1, upar1, mu);
    const double upg1 = sqrt(((2.0 * mu) * L1.kappa) * L1.B);
    for (int i = 0; i < 3; ++i) {
        x[i] = Rk[i];
        u[i] = (upar1 * L1.b_dn[i] + L1.vE[i] * Gam1) + upg1 * bperp[i];
    }
    return flags;
}

// One coupled step (Sec. 3.2) of one particle.  Returns S: 0 guiding
// center, 1 full orbit, 2 not advanced (outside the domain).
//
// The two branches share their skeleton -- metric and fields at x^n, K
// midpoint iterations that each need the metric and its derivatives and the
// geodesic force G, metric and fields at x^{n+1} -- so they are evaluated in
// one pass: a wavefront whose lanes took different branches then runs the
// shared metric evaluations once, and only the branch-specific parts
// diverge.  Per lane the operations are exactly those of greom_step /
// grgca_step above (same values, same order).
template <typename T>
GCB_HD int coupled_step(const T* __restrict__ F, const double* __restrict__ dl_table,
                        const GrConst& g, double x[3], double u[3], double qm, uint8_t& status,
                        double& res) {
    res = 0.0;
    if ((status & kStOut) || !inside(g, x[0], x[1])) {
        if (!inside(g, x[0], x[1])) status |= kStOut;
        return 2;
    }
    Metric m0;
    kerr_schild<false>(g.a, x[0], x[1], m0);
    GrSample f0;
    grid_sample(F, g, x[0], x[1], f0);
    int ci, cj;
    double wx, wy;
    grid_cell(g, x[0], x[1], ci, cj, wx, wy);
    const double dl = dl_table[(size_t)cj * g.nr + ci];
    const bool gca = switch_gca(m0, f0, u, qm, dl, g);

    uint32_t fl = 0;
    // guiding-center state: mu, gyration direction, u_par after the half push
    double mu = 0.0, bperp[3] = {0.0, 0.0, 0.0}, p1 = 0.0, pk = 0.0;
    // full-orbit state: u after the half push, the iterate u''
    double u1[3] = {u[0], u[1], u[2]}, uk[3];
    if (gca) {
        GcLocal L0;
        fl |= gc_local(m0, f0, L0);
        const double Gf = gamma_of(m0, u);
        const double upar = (L0.b_up[0] * u[0] + L0.b_up[1] * u[1]) + L0.b_up[2] * u[2];
        double uperp[3];
        for (int i = 0; i < 3; ++i) uperp[i] = (u[i] - upar * L0.b_dn[i]) - L0.vE[i] * Gf;
        const double up2 = norm2_cov(m0, uperp);
        mu = ((0.5 * up2) / L0.B) / L0.kappa;
        if (!(L0.B > 0.0)) mu = 0.0;
        const double nu = sqrt(up2);
        const double inv_nu = nu > 0.0 ? 1.0 / nu : 0.0;
        for (int i = 0; i < 3; ++i) bperp[i] = uperp[i] * inv_nu;
        p1 = upar + (qm * (m0.alpha * (0.5 * g.dt))) * L0.Dpar;
        pk = p1;
    } else {
        half_push(m0, f0, u1, qm, g.dt);
    }
    for (int i = 0; i < 3; ++i) uk[i] = u1[i];

    double Xk[3] = {x[0], x[1], x[2]};
    for (int k = 0; k < g.n_iter; ++k) {
        double Xb[3];
        for (int i = 0; i < 3; ++i) Xb[i] = 0.5 * (Xk[i] + x[i]);
        Metric mb;
        kerr_schild<true>(g.a, Xb[0], Xb[1], mb);
        double V[3], ub[3], Gam;
        double bup0 = 0.0, bup1 = 0.0;
        if (gca) {
            const double pb = 0.5 * (pk + p1);
            GrSample fb;
            grid_sample(F, g, Xb[0], Xb[1], fb);
            GcLocal Lb;
            fl |= gc_local(mb, fb, Lb);
            Gam = gamma_gc(Lb, pb, mu);
            double vu[3];
            raise(mb, Lb.vE, vu);
            V[0] = mb.alpha * (pb * (Lb.b_up[0] / Gam) + vu[0]) - mb.beta_r;
            V[1] = mb.alpha * (pb * (Lb.b_up[1] / Gam) + vu[1]);
            V[2] = mb.alpha * (pb * (Lb.b_up[2] / Gam) + vu[2]);
            const double upg = sqrt(((2.0 * mu) * Lb.kappa) * Lb.B);
            for (int i = 0; i < 3; ++i)
                ub[i] = (pb * Lb.b_dn[i] + Lb.vE[i] * Gam) + upg * bperp[i];
            bup0 = Lb.b_up[0];
            bup1 = Lb.b_up[1];
        } else {
            for (int i = 0; i < 3; ++i) ub[i] = 0.5 * (uk[i] + u1[i]);
            Gam = gamma_of(mb, ub);
            geo_V(mb, ub, Gam, V);
        }
        double G[2];
        geo_G(mb, ub, Gam, G);
        double Xn[3];
        for (int i = 0; i < 3; ++i) Xn[i] = x[i] + g.dt * V[i];
        res = max_nan(max_nan(fabs(Xn[0] - Xk[0]), fabs(Xn[1] - Xk[1])), fabs(Xn[2] - Xk[2]));
        for (int i = 0; i < 3; ++i) Xk[i] = Xn[i];
        if (gca) {
            const double Gb = G[0] * bup0 + G[1] * bup1;
            pk = p1 + g.dt * Gb;
        } else {
            uk[0] = u1[0] + g.dt * G[0];
            uk[1] = u1[1] + g.dt * G[1];
            uk[2] = u1[2];
        }
    }

    Metric m1;
    kerr_schild<false>(g.a, Xk[0], Xk[1], m1);
    GrSample f1;
    grid_sample(F, g, Xk[0], Xk[1], f1);
    double un[3];
    if (gca) {
        GcLocal L1;
        fl |= gc_local(m1, f1, L1);
        const double upar1 = pk + (qm * (m1.alpha * (0.5 * g.dt))) * L1.Dpar;
        const double Gam1 = gamma_gc(L1, upar1, mu);
        const double upg1 = sqrt(((2.0 * mu) * L1.kappa) * L1.B);
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
        Metric m;
        kerr_schild<false>(g.a, r, t, m);
        return sqrt(m.gd_rr * m.gd_thth);
    };
    const double tot = ((f(rm, tm) + f(rp, tm)) + f(rm, tp)) + f(rp, tp);
    return sqrt(tot * (hr * ht));
}

}  // namespace gr
}  // namespace gcb
