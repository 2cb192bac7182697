// Reverse-mode derivative of one binary64 step of the 3D coupled pusher, with
// the switch decision held at its forward value: the 2D adjoint of
// gcb_adjoint.hpp with the trilinear gather, gradients along x, y and z and
// three-component positions.  The blocks that do not depend on the dimension
// (Gamma, curvature drift, parallel update, local quantities) are the 2D ones.
//   scatter_sample3  node cotangents of one recorded gather point (2x2x2
//                    stencil per component)
//   gather_vjp3      the position cotangent of the trilinear gather,
//                    including the mixed second derivatives of W carried by
//                    the B-gradient cotangents
//   boris_step_vjp3, gca_step_vjp3   the two branches of a step
// State order st[9] = (x, y, z, xp, yp, zp, ux, uy, uz).
#pragma once

#include "gcb_adjoint.hpp"
#include "gcb_math3.hpp"

namespace gcb {
namespace adj3 {

using adj::conserved_mu;
using adj::cross_vjp;
using adj::gamma_vjp;
using adj::kMaxAdjIter;
using adj::LocalBar;
using adj::parallel_vjp;
using adj::vcurv_vjp;
using adj::zero;
using LocalD = Local<double>;
using KD = Consts<double>;
using K3 = Consts3<double>;
using Sample3D = Sample3<double>;

struct SampleBar3 {
    double E[3], B[3];
    double dB[3][3];   // [j][i]: cotangent of d_j B_i, j = x, y, z
};

GCB_HD void zero(SampleBar3& s) {
    for (int i = 0; i < 3; ++i) {
        s.E[i] = s.B[i] = 0.0;
        for (int j = 0; j < 3; ++j) s.dB[j][i] = 0.0;
    }
}

// lattice offset of component k along axis a, in cells
GCB_HD double offset3(const PushConst3& pc, bool yee, int k, int a) {
    if (yee) return ((kYee3Set[k] >> a) & 1) ? 0.5 : 0.0;
    return a < 2 ? pc.b.stagger[k][a] : pc.sz[k];
}

// a runaway point (lattice coordinate NaN or of magnitude kFarLattice or
// more): its sample is a constant NaN, with no node or position cotangent
GCB_HD bool far3(const PushConst3& pc, double X, double Y, double Z) {
    return !(fabs(X * pc.b.inv_dx) < kFarLattice && fabs(Y * pc.b.inv_dy) < kFarLattice &&
             fabs(Z * pc.inv_dz) < kFarLattice);
}

// cell and weights of component k's stencil at (X, Y, Z)
GCB_HD void stencil3(const PushConst3& pc, bool yee, int k, double X, double Y, double Z,
                     int c[3], double w[3]) {
    const double g[3] = {X * pc.b.inv_dx, Y * pc.b.inv_dy, Z * pc.inv_dz};
    for (int a = 0; a < 3; ++a) {
        const double xi = g[a] - offset3(pc, yee, k, a);
        const double f = floor(xi);
        c[a] = (int)f;
        w[a] = xi - f;
    }
}

// the value and gradient cotangents of component k
GCB_HD void comp_bar(const SampleBar3& sb, int k, double& vb, double gb[3]) {
    vb = k < 3 ? sb.E[k] : sb.B[k - 3];
    for (int j = 0; j < 3; ++j) gb[j] = k < 3 ? 0.0 : sb.dB[j][k - 3];
}

// Node cotangents of one gather point: `add(k, i, j, l, g)` for the eight
// nodes of each component's cell (global indices, any periodic image).
template <class Add>
GCB_HD void scatter_sample3(Add& add, const PushConst3& pc, bool yee, double X, double Y,
                            double Z, const SampleBar3& sb) {
    const double id[3] = {pc.b.inv_dx, pc.b.inv_dy, pc.inv_dz};
    if (far3(pc, X, Y, Z)) return;
    for (int k = 0; k < 6; ++k) {
        double vb, gb[3];
        comp_bar(sb, k, vb, gb);
        if (vb == 0.0 && gb[0] == 0.0 && gb[1] == 0.0 && gb[2] == 0.0) continue;
        int c[3];
        double w[3];
        stencil3(pc, yee, k, X, Y, Z, c, w);
        for (int n = 0; n < 8; ++n) {
            const int o[3] = {n & 1, (n >> 1) & 1, n >> 2};
            double W[3], s[3];
            for (int a = 0; a < 3; ++a) {
                W[a] = o[a] ? w[a] : 1.0 - w[a];
                s[a] = o[a] ? id[a] : -id[a];
            }
            const double g = vb * (W[0] * W[1] * W[2]) + gb[0] * (s[0] * W[1] * W[2]) +
                             gb[1] * (W[0] * s[1] * W[2]) + gb[2] * (W[0] * W[1] * s[2]);
            add(k, c[0] + o[0], c[1] + o[1], c[2] + o[2], g);
        }
    }
}

// Position cotangent of the trilinear gather at (X, Y, Z), added to P[3];
// the gather point and its cotangents go to `sink.sample`.
template <class Sink>
GCB_HD void gather_vjp3(const GlobalAcc3<double>& acc, Sink& sink, const PushConst3& pc,
                        bool yee, double X, double Y, double Z, const SampleBar3& sb,
                        double P[3]) {
    sink.sample(X, Y, Z, sb);
    if (far3(pc, X, Y, Z)) return;
    const double id[3] = {pc.b.inv_dx, pc.b.inv_dy, pc.inv_dz};
    for (int k = 0; k < 6; ++k) {
        double vb, gb[3];
        comp_bar(sb, k, vb, gb);
        if (vb == 0.0 && gb[0] == 0.0 && gb[1] == 0.0 && gb[2] == 0.0) continue;
        int c[3];
        double w[3];
        stencil3(pc, yee, k, X, Y, Z, c, w);
        double f[8];
        acc.oct<double>(k, c[0], c[1], c[2], f);
        const double WX[2] = {1.0 - w[0], w[0]}, WY[2] = {1.0 - w[1], w[1]},
                     WZ[2] = {1.0 - w[2], w[2]};
        // first derivatives of the interpolant and its mixed second derivatives
        double vx = 0.0, vy = 0.0, vz = 0.0, vxy = 0.0, vxz = 0.0, vyz = 0.0;
        for (int q = 0; q < 2; ++q)
            for (int r = 0; r < 2; ++r) {
                vx += WY[q] * WZ[r] * (f[r * 4 + q * 2 + 1] - f[r * 4 + q * 2]);
                vy += WX[q] * WZ[r] * (f[r * 4 + 2 + q] - f[r * 4 + q]);
                vz += WX[q] * WY[r] * (f[4 + r * 2 + q] - f[r * 2 + q]);
            }
        for (int q = 0; q < 2; ++q) {
            vxy += WZ[q] * ((f[q * 4 + 3] - f[q * 4 + 2]) - (f[q * 4 + 1] - f[q * 4]));
            vxz += WY[q] * ((f[4 + q * 2 + 1] - f[4 + q * 2]) - (f[q * 2 + 1] - f[q * 2]));
            vyz += WX[q] * ((f[4 + 2 + q] - f[4 + q]) - (f[2 + q] - f[q]));
        }
        vx *= id[0];
        vy *= id[1];
        vz *= id[2];
        vxy *= id[0] * id[1];
        vxz *= id[0] * id[2];
        vyz *= id[1] * id[2];
        P[0] += vb * vx + gb[1] * vxy + gb[2] * vxz;
        P[1] += vb * vy + gb[0] * vxy + gb[2] * vyz;
        P[2] += vb * vz + gb[0] * vxz + gb[1] * vyz;
    }
}

GCB_HD void local_vjp3(const Sample3D& s, const KD& K, const LocalBar& Lb, SampleBar3& sb) {
    const double G[3][3] = {{s.dBx[0], s.dBx[1], s.dBx[2]},
                            {s.dBy[0], s.dBy[1], s.dBy[2]},
                            {s.dBz[0], s.dBz[1], s.dBz[2]}};
    double Eb[3], Bb[3], Gb[3][3];
    adj::local_vjp_nd<3>(s.E, s.B, G, K, Lb, Eb, Bb, Gb);
    for (int i = 0; i < 3; ++i) {
        sb.E[i] += Eb[i];
        sb.B[i] += Bb[i];
        for (int j = 0; j < 3; ++j) sb.dB[j][i] += Gb[j][i];
    }
}

// u_par b/Gamma + v_E + v_c, three components
GCB_HD void drift_vjp3(const LocalD& L, double upn, double mu, double inv_qm, bool curv,
                       const KD& K, const double Fb[3], LocalBar& Lb, double& upnb,
                       double& mub) {
    const double g = gamma_gca(L, upn, conserved_mu(mu), K);
    const double a = upn / g;
    const double ab = (Fb[0] * L.b[0] + Fb[1] * L.b[1]) + Fb[2] * L.b[2];
    for (int i = 0; i < 3; ++i) {
        Lb.b[i] += a * Fb[i];
        Lb.vE[i] += Fb[i];
    }
    double gb = -ab * a / g;
    upnb += ab / g;
    if (curv) vcurv_vjp(L, upn, g, inv_qm, K, Fb, Lb, upnb, gb);
    gamma_vjp(L, upn, mu, K, gb, Lb, upnb, mub);
}

template <bool kYee>
GCB_HD void local_at3(const GlobalAcc3<double>& acc, const PushConst3& pc, const K3& K,
                      const double X[3], Sample3D& s, LocalD& L) {
    gather3<double, true, kYee>(acc, pc, K, X[0], X[1], X[2], s);
    local_from_sample(s, K, L);
}

// Field samples of the forward recomputation taken again in the reverse sweep
// (slots as in 2D: 0 = R^{n-1/2}, 1 = R^n, 1 + k = R^k); NoSamples3 keeps none.
struct NoSamples3 {
    GCB_HD void put(int, const Sample3D&) {}
    GCB_HD bool get(int, Sample3D&) const { return false; }
};

template <bool kYee, class Keep>
GCB_HD void local_again3(const GlobalAcc3<double>& acc, const Keep& keep, int slot,
                         const PushConst3& pc, const K3& K, const double X[3], Sample3D& s,
                         LocalD& L) {
    if (keep.get(slot, s))
        local_from_sample(s, K, L);
    else
        local_at3<kYee>(acc, pc, K, X, s, L);
}

template <bool kYee, class Sink>
GCB_HD void local_bar_to_position3(const GlobalAcc3<double>& acc, Sink& sink,
                                   const PushConst3& pc, const K3& K, const Sample3D& s,
                                   const double X[3], const LocalBar& Lb, double P[3]) {
    SampleBar3 sb;
    zero(sb);
    local_vjp3(s, K, Lb, sb);
    gather_vjp3(acc, sink, pc, kYee, X[0], X[1], X[2], sb, P);
}

template <bool kYee, class Sink>
GCB_HD void boris_step_vjp3(const GlobalAcc3<double>& acc, Sink& sink, const PushConst3& pc,
                            const K3& K, const double st[9], double qm, double lam[9]) {
    const double X[3] = {st[0], st[1], st[2]};
    Sample3D s;
    gather3<double, false, kYee>(acc, pc, K, X[0], X[1], X[2], s);
    const double* E = s.E;
    const double* Bv = s.B;
    const double u[3] = {st[6], st[7], st[8]};
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
    // reverse: x_out = x + dt u_n/Gamma_n, xp_out = x, u_out = u_n
    const double dt = pc.b.dt;
    double unb[3], igb = 0.0;
    for (int i = 0; i < 3; ++i) {
        unb[i] = lam[6 + i] + dt * ig * lam[i];
        igb += dt * un[i] * lam[i];
    }
    const double gnb = -igb * ig * ig;
    for (int i = 0; i < 3; ++i) unb[i] += gnb * un[i] * K.inv_c2 / gn;
    SampleBar3 sb;
    zero(sb);
    for (int i = 0; i < 3; ++i) sb.E[i] += hq * unb[i];
    double umb[3] = {unb[0], unb[1], unb[2]};
    double upb[3] = {0.0, 0.0, 0.0}, svb[3] = {0.0, 0.0, 0.0};
    cross_vjp(up, sv, unb, upb, svb);
    double tb[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 3; ++i) umb[i] += upb[i];
    cross_vjp(um, t, upb, umb, tb);
    const double gb = (svb[0] * t[0] + svb[1] * t[1]) + svb[2] * t[2];
    for (int i = 0; i < 3; ++i) tb[i] += g * svb[i];
    const double t2b = -gb * g * g * 0.5;
    for (int i = 0; i < 3; ++i) tb[i] += 2.0 * t[i] * t2b;
    const double fb = (tb[0] * Bv[0] + tb[1] * Bv[1]) + tb[2] * Bv[2];
    for (int i = 0; i < 3; ++i) sb.B[i] += f * tb[i];
    const double gmb = -fb * f / gm;
    for (int i = 0; i < 3; ++i) umb[i] += gmb * um[i] * K.inv_c2 / gm;
    for (int i = 0; i < 3; ++i) sb.E[i] += hq * umb[i];
    double P[3] = {lam[0] + lam[3], lam[1] + lam[4], lam[2] + lam[5]};
    gather_vjp3(acc, sink, pc, kYee, X[0], X[1], X[2], sb, P);
    for (int i = 0; i < 3; ++i) {
        lam[i] = P[i];
        lam[3 + i] = 0.0;
        lam[6 + i] = umb[i];
    }
}

// Gather points gca_step_vjp3 hands to its sink: as in 2D.
GCB_HD int gca_vjp_samples3(int n_iter) { return adj::gca_vjp_samples(n_iter); }

template <bool kYee, class Sink, class Keep = NoSamples3>
GCB_HD void gca_step_vjp3(const GlobalAcc3<double>& acc, Sink& sink, const PushConst3& pc,
                          const K3& K, const double st[9], double qm, double lam[9],
                          Keep keep = Keep()) {
    const bool curv = pc.b.curvature != 0;
    const double x[3] = {st[0], st[1], st[2]};
    const double box[3] = {pc.b.Lx, pc.b.Ly, pc.Lz};
    const double ux = st[6], uy = st[7], uz = st[8];
    const double inv_qm = 1.0 / qm;
    const double h = K.h;
    const int Kit = pc.b.n_iter < kMaxAdjIter ? pc.b.n_iter : kMaxAdjIter;

    // ---- forward recomputation
    double Rh[3];
    for (int a = 0; a < 3; ++a) Rh[a] = x[a] - 0.5 * min_image(x[a] - st[3 + a], box[a]);
    double upar, mu, gf, nu, up[3], bp[3], vch[3] = {0.0, 0.0, 0.0};
    {
        Sample3D s;
        LocalD L;
        local_at3<kYee>(acc, pc, K, Rh, s, L);
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
    double upn, Fn[3];
    {
        Sample3D s;
        LocalD L;
        local_at3<kYee>(acc, pc, K, x, s, L);
        keep.put(1, s);
        uint32_t fl = 0;
        upn = parallel_update(L, upar, conserved_mu(mu), qm, curv, K, fl);
        drift_terms3(L, upn, conserved_mu(mu), inv_qm, curv, K, Fn);
    }
    double Rk[kMaxAdjIter + 1][3];
    for (int a = 0; a < 3; ++a) Rk[0][a] = x[a];
    for (int k = 0; k < Kit; ++k) {
        double F[3];
        if (k == 0) {
            for (int a = 0; a < 3; ++a) F[a] = Fn[a];
        } else {
            Sample3D s;
            LocalD L;
            local_at3<kYee>(acc, pc, K, Rk[k], s, L);
            keep.put(1 + k, s);
            drift_terms3(L, upn, conserved_mu(mu), inv_qm, curv, K, F);
        }
        for (int a = 0; a < 3; ++a) Rk[k + 1][a] = x[a] + h * (Fn[a] + F[a]);
    }
    double Rm[3];
    for (int a = 0; a < 3; ++a) Rm[a] = x[a] + 0.5 * (Rk[Kit][a] - x[a]);

    // ---- reverse sweep
    double xb[3] = {lam[3], lam[4], lam[5]};   // xp_out = x
    double RKb[3] = {lam[0], lam[1], lam[2]};  // x_out = wrap(R^K)
    const double ub[3] = {lam[6], lam[7], lam[8]};
    double upnb = 0.0, mub = 0.0, bpb[3] = {0.0, 0.0, 0.0};

    // 5. reconstruction at R^{n+1/2}
    {
        Sample3D s;
        LocalD L;
        local_at3<kYee>(acc, pc, K, Rm, s, L);
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
        double Rmb[3] = {0.0, 0.0, 0.0};
        local_bar_to_position3<kYee>(acc, sink, pc, K, s, Rm, Lb, Rmb);
        for (int a = 0; a < 3; ++a) {
            xb[a] += 0.5 * Rmb[a];
            RKb[a] += 0.5 * Rmb[a];
        }
    }

    // 4. fixed-point iterations in reverse order
    double Fnb[3] = {0.0, 0.0, 0.0};
    double Rb[3] = {RKb[0], RKb[1], RKb[2]};
    for (int k = Kit - 1; k >= 0; --k) {
        double Fkb[3];
        for (int a = 0; a < 3; ++a) {
            xb[a] += Rb[a];
            Fnb[a] += h * Rb[a];
            Fkb[a] = h * Rb[a];
        }
        if (k == 0) {
            for (int a = 0; a < 3; ++a) {
                Fnb[a] += Fkb[a];
                Rb[a] = 0.0;
            }
        } else {
            Sample3D s;
            LocalD L;
            local_again3<kYee>(acc, keep, 1 + k, pc, K, Rk[k], s, L);
            LocalBar Lb;
            zero(Lb);
            drift_vjp3(L, upn, mu, inv_qm, curv, K, Fkb, Lb, upnb, mub);
            double nb[3] = {0.0, 0.0, 0.0};
            local_bar_to_position3<kYee>(acc, sink, pc, K, s, Rk[k], Lb, nb);
            for (int a = 0; a < 3; ++a) Rb[a] = nb[a];
        }
    }

    // 3.-2. drift at R^n and the parallel update
    double uparb = 0.0;
    {
        Sample3D s;
        LocalD L;
        local_again3<kYee>(acc, keep, 1, pc, K, x, s, L);
        LocalBar Lb;
        zero(Lb);
        drift_vjp3(L, upn, mu, inv_qm, curv, K, Fnb, Lb, upnb, mub);
        parallel_vjp(L, upar, mu, qm, curv, K, upnb, Lb, uparb, mub);
        local_bar_to_position3<kYee>(acc, sink, pc, K, s, x, Lb, xb);
    }

    // 1. decomposition at R^{n-1/2}
    double uvb[3], xpb[3] = {0.0, 0.0, 0.0};
    {
        Sample3D s;
        LocalD L;
        local_again3<kYee>(acc, keep, 0, pc, K, Rh, s, L);
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
        for (int i = 0; i < 3; ++i) {
            uvb[i] = upb[i];
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
        double Rhb[3] = {0.0, 0.0, 0.0};
        local_bar_to_position3<kYee>(acc, sink, pc, K, s, Rh, Lb, Rhb);
        for (int a = 0; a < 3; ++a) {
            xb[a] += 0.5 * Rhb[a];
            xpb[a] += 0.5 * Rhb[a];
        }
    }
    for (int a = 0; a < 3; ++a) {
        lam[a] = xb[a];
        lam[3 + a] = xpb[a];
        lam[6 + a] = uvb[a];
    }
}

}  // namespace adj3
}  // namespace gcb
