// Per-particle arithmetic of the coupled pusher in three dimensions, templated
// on the bulk type R like gcb_math.hpp (binary64, or the mixed form with
// binary64 positions).  The equations are the 2D ones; what changes is the
// trilinear gather with gradients along z, d_j b over j = x, y, z, and the
// three-component guiding-center position.  The Boris push, the switch, the
// parallel update and the curvature drift are the 2D functions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gcb_access3.hpp"
#include "gcb_math.hpp"

namespace gcb {
// one instance per arithmetic (see gcb_math.hpp)
inline namespace GCB_ARITH_NS {

template <typename R>
struct Consts3 : Consts<R> {
    R inv_dz;
};

template <typename R>
GCB_HD Consts3<R> make_consts3(const PushConst3& pc) {
    Consts3<R> k;
    static_cast<Consts<R>&>(k) = make_consts<R>(pc.b);
    k.inv_dz = (R)pc.inv_dz;
    return k;
}

template <typename R>
struct Regs3 {
    double x, y, z, xp, yp, zp;
    R ux, uy, uz;
    double qm;
};

template <typename R>
struct Sample3 {
    static constexpr bool kGradE = false;
    R E[3], B[3];
    R dBx[3], dBy[3], dBz[3];   // d B_i / dx, dy, dz
};

// with the E gradients as well (the exact frame with curvature)
template <typename R>
struct SampleEG3 : Sample3<R> {
    static constexpr bool kGradE = true;
    R dEx[3], dEy[3], dEz[3];   // d E_i / dx, dy, dz
};

// ---------------------------------------------------------------------------
// Gather (Sec. 4, opening paragraph): linear shape function on the 2x2x2
// nodes of each component's lattice, summed plane by plane (the bilinear
// expression of each z plane, then the two planes weighted along z);
// gradients by differentiating it.  f[dz*4 + dy*2 + dx].

template <typename R>
GCB_HD void trilerp(const R f[8], R wx, R wy, R wz, const Consts3<R>& K, bool grad, R& val,
                    R& ddx, R& ddy, R& ddz) {
    const R ax = (R)1 - wx, ay = (R)1 - wy, az = (R)1 - wz;
    const R v0 = (((ax * ay) * f[0] + (wx * ay) * f[1]) + (ax * wy) * f[2]) + (wx * wy) * f[3];
    const R v1 = (((ax * ay) * f[4] + (wx * ay) * f[5]) + (ax * wy) * f[6]) + (wx * wy) * f[7];
    val = az * v0 + wz * v1;
    if (grad) {
        const R g0 = ay * (f[1] - f[0]) + wy * (f[3] - f[2]);
        const R g1 = ay * (f[5] - f[4]) + wy * (f[7] - f[6]);
        const R h0 = ax * (f[2] - f[0]) + wx * (f[3] - f[1]);
        const R h1 = ax * (f[6] - f[4]) + wx * (f[7] - f[5]);
        ddx = (az * g0 + wz * g1) * K.inv_dx;
        ddy = (az * h0 + wz * h1) * K.inv_dy;
        ddz = (v1 - v0) * K.inv_dz;
    }
}

template <typename R, bool kGrad, class S>
GCB_HD void store_comp(int k, R val, R ddx, R ddy, R ddz, S& s) {
    if (k < 3) {
        s.E[k] = val;
        if constexpr (S::kGradE) {
            s.dEx[k] = ddx;
            s.dEy[k] = ddy;
            s.dEz[k] = ddz;
        }
    } else {
        s.B[k - 3] = val;
        if (kGrad) {
            s.dBx[k - 3] = ddx;
            s.dBy[k - 3] = ddy;
            s.dBz[k - 3] = ddz;
        }
    }
}

// the six components from the located Yee stencils
template <typename R, bool kGrad, class Loader, class S>
GCB_HD void interp3_yee(const Loader& ld, const R wx[2], const R wy[2], const R wz[2],
                        const Consts3<R>& K, S& s) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int set = kYee3Set[k];
        R f[8];
        ld.template load8<R>(set, k, f);
        R val, ddx, ddy, ddz;
        trilerp(f, wx[set & 1], wy[(set >> 1) & 1], wz[set >> 2], K,
                (kGrad && k >= 3) || S::kGradE, val, ddx, ddy, ddz);
        store_comp<R, kGrad>(k, val, ddx, ddy, ddz, s);
    }
}

template <typename R, bool kGrad, typename T, class S>
GCB_HD void yee3_fetch(const GlobalAcc3<T>& acc, const int fl[3][2], const R wx[2],
                       const R wy[2], const R wz[2], const Consts3<R>& K, S& s) {
    typename GlobalAcc3<T>::Loc L;
    acc.locate(fl, L);
    interp3_yee<R, kGrad>(GlobalLoad3<T>{acc, L}, wx, wy, wz, K, s);
}

template <typename R, bool kGrad, typename T, class S>
GCB_HD void yee3_fetch(const TileAcc3<T>& acc, const int fl[3][2], const R wx[2],
                       const R wy[2], const R wz[2], const Consts3<R>& K, S& s) {
    int off[8];
    typename GlobalAcc3<T>::Loc L;
    if (acc.locate(fl, off, L)) {
        const int W = acc.W;
        interp3_yee<R, kGrad>(LdsLoad3<T>{acc.lds, off, W, W * W, W * W * W}, wx, wy, wz, K,
                              s);
    } else {
        interp3_yee<R, kGrad>(GlobalLoad3<T>{acc.g, L}, wx, wy, wz, K, s);
    }
}

// the gather at lattice coordinates g = (X/dx, Y/dy, Z/dz)
template <typename R, bool kGrad, bool kYee, class Acc, class S>
GCB_HD void gather3_at(const Acc& acc, const PushConst3& pc, const Consts3<R>& K,
                       const double g[3], S& s) {
    if constexpr (kYee) {
        // lattice coordinate minus the offset: offset 0 leaves it unchanged
        int fl[3][2];
        R w[3][2];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double h = g[a] - 0.5;
            const double fa = floor(g[a]), fb = floor(h);
            fl[a][0] = (int)fa;
            fl[a][1] = (int)fb;
            w[a][0] = (R)(g[a] - fa);
            w[a][1] = (R)(h - fb);
        }
        yee3_fetch<R, kGrad>(acc, fl, w[0], w[1], w[2], K, s);
    } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double xi = g[0] - pc.b.stagger[k][0];
            const double eta = g[1] - pc.b.stagger[k][1];
            const double zeta = g[2] - pc.sz[k];
            const double fi = floor(xi), fj = floor(eta), fk = floor(zeta);
            R f[8];
            acc.template oct<R>(k, (int)fi, (int)fj, (int)fk, f);
            R val, ddx, ddy, ddz;
            trilerp(f, (R)(xi - fi), (R)(eta - fj), (R)(zeta - fk), K,
                    (kGrad && k >= 3) || S::kGradE, val, ddx, ddy, ddz);
            store_comp<R, kGrad>(k, val, ddx, ddy, ddz, s);
        }
    }
}

// All six components at (X, Y, Z); B gradients when kGrad.  kYee: the 3D Yee
// offsets.  Lattice coordinates and weights in binary64 from the positions.
template <typename R, bool kGrad, bool kYee, class Acc, class S>
GCB_HD void gather3(const Acc& acc, const PushConst3& pc, const Consts3<R>& K, double X,
                    double Y, double Z, S& s) {
    double g[3] = {X * pc.b.inv_dx, Y * pc.b.inv_dy, Z * pc.inv_dz};
    // a runaway point (lattice coordinate NaN or of magnitude kFarLattice or
    // more) is gathered at the origin and its sample replaced by NaN
    const bool far = !(fabs(g[0]) < kFarLattice && fabs(g[1]) < kFarLattice &&
                       fabs(g[2]) < kFarLattice);
    if (__builtin_expect(far, 0)) g[0] = g[1] = g[2] = 0.0;
    gather3_at<R, kGrad, kYee>(acc, pc, K, g, s);
    if (__builtin_expect(far, 0)) {
        const R q = (R)__builtin_nan("");
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            s.E[i] = q;
            s.B[i] = q;
            s.dBx[i] = q;
            s.dBy[i] = q;
            s.dBz[i] = q;
            if constexpr (S::kGradE) {
                s.dEx[i] = q;
                s.dEy[i] = q;
                s.dEz[i] = q;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Local guiding-center quantities (Sec. 2.2) with gradients along x, y, z:
// (b.grad)b = b_x d_x b + b_y d_y b + b_z d_z b, (v_E.grad)b likewise.

template <typename R>
GCB_HD uint32_t local_from_sample(const Sample3<R>& s, const Consts<R>& K, Local<R>& L) {
    const uint32_t flags = local_fields(s.E, s.B, K, L);
    R dbx[3], dby[3], dbz[3];
    L.gB[0] = db_along(L, s.dBx, dbx);
    L.gB[1] = db_along(L, s.dBy, dby);
    L.gB[2] = db_along(L, s.dBz, dbz);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        L.bgb[i] = (L.b[0] * dbx[i] + L.b[1] * dby[i]) + L.b[2] * dbz[i];
        L.vgb[i] = (L.vE[0] * dbx[i] + L.vE[1] * dby[i]) + L.vE[2] * dbz[i];
    }
    curvature_scalars(L);
    return flags;
}

// The exact frame with the curvature scheme in 3D: as the 2D
// local_exact_curv, with d_j b* over j = x, y, z.
template <typename R>
GCB_HD uint32_t local_exact_curv(const SampleEG3<R>& s, const Consts<R>& K, Local<R>& L) {
    const uint32_t flags = local_fields_exact(s.E, s.B, K, L);
    Dual<R, 3> E[3], Bv[3], b[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        E[i].v = s.E[i];
        E[i].d[0] = s.dEx[i];
        E[i].d[1] = s.dEy[i];
        E[i].d[2] = s.dEz[i];
        Bv[i].v = s.B[i];
        Bv[i].d[0] = s.dBx[i];
        Bv[i].d[1] = s.dBy[i];
        Bv[i].d[2] = s.dBz[i];
    }
    bstar_dual<R, 3>(E, Bv, K, b);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        L.bgb[i] = (L.b[0] * b[i].d[0] + L.b[1] * b[i].d[1]) + L.b[2] * b[i].d[2];
        L.vgb[i] = (L.vE[0] * b[i].d[0] + L.vE[1] * b[i].d[1]) + L.vE[2] * b[i].d[2];
        L.gB[i] = (R)0;
    }
    curvature_scalars(L);
    return flags;
}

// u_par b / Gamma + v_E + v_c at a point, three components (v_c with the
// grad-B drift under the mirror option)
template <typename R>
GCB_HD void drift_terms3(const Local<R>& L, R upn, const Gyr<R>& gy, R inv_qm, bool curvature,
                         const Consts<R>& K, R F[3], bool mirror = false) {
    const Gam<R> G = gamma_gca2(L, upn, gy, K);
    const R a = over(upn, G);
    if (curvature) {
        R vc[3];
        if (mirror)
            v_curv_mirror<3>(L, upn, G.g, inv_qm, gy.mu, K, vc);
        else
            v_curv_g(L, upn, G, inv_qm, K, vc);
#pragma unroll
        for (int i = 0; i < 3; ++i) F[i] = (a * L.b[i] + L.vE[i]) + vc[i];
    } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) F[i] = a * L.b[i] + L.vE[i];
    }
}

// ---------------------------------------------------------------------------
// Full-orbit step (Sec. 2.1): u^{n-1/2} -> u^{n+1/2}, x^{n+1} = x^n + dt u/Gamma.
template <typename R>
GCB_HD void boris_step3(const Sample3<R>& s, Regs3<R>& r, const PushConst3& pc,
                        const Consts<R>& K) {
    boris(s.E, s.B, r.ux, r.uy, r.uz, (R)r.qm, K);
    R inv_g;
    if constexpr (kFastD<R>) {
        inv_g = gamma_full2(r.ux, r.uy, r.uz, K).inv;
    } else {
        const R gn = gamma_full(r.ux, r.uy, r.uz, K);
        inv_g = (R)1 / gn;
    }
    const double xn = r.x + pc.b.dt * (double)(r.ux * inv_g);
    const double yn = r.y + pc.b.dt * (double)(r.uy * inv_g);
    const double zn = r.z + pc.b.dt * (double)(r.uz * inv_g);
    r.xp = r.x;
    r.yp = r.y;
    r.zp = r.z;
    r.x = wrap_i<R>(xn, pc.b.Lx, pc.b.inv_Lx);
    r.y = wrap_i<R>(yn, pc.b.Ly, pc.b.inv_Ly);
    r.z = wrap_i<R>(zn, pc.Lz, pc.inv_Lz);
}

// One guiding-center step (Sec. 2.2.1 / 2.2.2 inside the coupled step of
// Sec. 3.1).  sn is the gather (with gradients) at x^n.  Returns status
// flags; res receives |R^K - R^{K-1}|_inf over the three components.
// kExact: the exact frame of Sec. 2.2 (with kExCurv its curvature scheme,
// whose gathers carry the E gradients);
// kMirror: the mirror force and grad-B drift (curvature scheme only).
template <typename R, bool kYee, bool kExact = false, bool kMirror = false, bool kPhase = false,
          bool kExCurv = false, class Acc>
GCB_HD uint32_t gca_step3(const Acc& acc, const Sample3<R>& sn, Regs3<R>& r,
                          const PushConst3& pc, const Consts3<R>& K, double& res) {
    static_assert(!kExCurv || kExact, "kExCurv is a form of the exact frame");
    using Smp = std::conditional_t<kExCurv, SampleEG3<R>, Sample3<R>>;
    uint32_t flags = 0;
    const bool curv = kExCurv || (!kExact && pc.b.curvature != 0);
    // the mirror terms ride on the curvature scheme (the host refuses others)
    const bool mirror = kMirror && curv;
    const double x[3] = {r.x, r.y, r.z};
    const double xprev[3] = {r.xp, r.yp, r.zp};
    const double box[3] = {pc.b.Lx, pc.b.Ly, pc.Lz};
    const double inv_box[3] = {pc.b.inv_Lx, pc.b.inv_Ly, pc.inv_Lz};
    const R ux = r.ux, uy = r.uy, uz = r.uz;
    const R qm = (R)r.qm;
    const R inv_qm = (R)1 / qm;

    // 1. guiding-center variables at R^{n-1/2} = (x^n + x^{n-1})/2
    R upar, bp[3];
    Gyr<R> gy;
    {
        double Rh[3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            Rh[a] = x[a] - 0.5 * min_image_i<R>(x[a] - xprev[a], box[a], inv_box[a]);
        Smp sh;
        gather3<R, true, kYee>(acc, pc, K, Rh[0], Rh[1], Rh[2], sh);
        Local<R> Lh;
        flags |= local_in_frame<kExact, R>(sh, K, Lh);
        upar = (ux * Lh.b[0] + uy * Lh.b[1]) + uz * Lh.b[2];
        const Gam<R> G = gamma_full2(ux, uy, uz, K);
        const R gf = G.g;
        R vc[3] = {(R)0, (R)0, (R)0};
        if (curv) v_curv_g(Lh, upar, G, inv_qm, K, vc);
        const R upx = (ux - upar * Lh.b[0]) - (Lh.vE[0] + vc[0]) * gf;
        const R upy = (uy - upar * Lh.b[1]) - (Lh.vE[1] + vc[1]) * gf;
        const R upz = (uz - upar * Lh.b[2]) - (Lh.vE[2] + vc[2]) * gf;
        const R up2 = (upx * upx + upy * upy) + upz * upz;
        flags |= mirror_check(ux, uy, uz, Lh, vc, up2, gf, pc.b, K);
        R mu;
        if constexpr (kFastD<R>)
            mu = (((R)0.5 * up2) * Lh.inv_B) * Lh.inv_kappa;
        else
            mu = (((R)0.5 * up2) * Lh.inv_B) / Lh.kappa;
        gy.mu = pc.b.gyration == GYR_ZERO ? (R)0 : mu;
        gy.up2 = up2;
        gy.fixed = pc.b.gyration == GYR_UPERP;
        R inv_nu;
        if constexpr (kFastD<R>) {
            inv_nu = up2 > (R)0 ? rsqrt_nr(up2) : (R)0;
        } else {
            const R nu = sqrt(up2);
            inv_nu = nu > (R)0 ? (R)1 / nu : (R)0;
        }
        bp[0] = upx * inv_nu;
        bp[1] = upy * inv_nu;
        bp[2] = upz * inv_nu;
    }

    // 2.-3. local quantities at R^n = x^n and the parallel update
    R upn, Fn[3];
    {
        Local<R> Ln;
        if constexpr (kExCurv) {
            SampleEG3<R> se;
            gather3<R, true, kYee>(acc, pc, K, x[0], x[1], x[2], se);
            flags |= local_in_frame<kExact, R>(se, K, Ln);
        } else {
            flags |= local_in_frame<kExact, R>(sn, K, Ln);
        }
        if (mirror)
            upn = mirror_parallel<3>(Ln, upar, gy, qm, K, flags);
        else
            upn = parallel_update(Ln, upar, gy, qm, curv, K, flags);
        drift_terms3(Ln, upn, gy, inv_qm, curv, K, Fn, mirror);
        if constexpr (kPhase) phase_advance(Ln, upar, upn, gy, qm, K, bp);
    }

    // 4. R^{n+1}: K fixed-point iterations R^{k+1} = R^k - H(R^k), R^0 = R^n
    double Rp[3] = {x[0], x[1], x[2]};
    res = 0.0;
    for (int k = 0; k < pc.b.n_iter; ++k) {
        R Fk[3];
        if (k == 0) {
            Fk[0] = Fn[0];
            Fk[1] = Fn[1];
            Fk[2] = Fn[2];
        } else {
            Smp sk;
            gather3<R, true, kYee>(acc, pc, K, Rp[0], Rp[1], Rp[2], sk);
            Local<R> Lk;
            flags |= local_in_frame<kExact, R>(sk, K, Lk);
            drift_terms3(Lk, upn, gy, inv_qm, curv, K, Fk, mirror);
        }
        double d[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double Rn = x[a] + (double)(K.h * (Fn[a] + Fk[a]));
            d[a] = fabs(Rn - Rp[a]);
            Rp[a] = Rn;
        }
        res = nan_max(nan_max(d[0], d[1]), d[2]);
    }
    if (res > pc.b.fp_tol) flags |= ST_FPRES;

    // 5. particle variables at R^{n+1/2} = (R^n + R^{n+1})/2, gyration
    //    direction held fixed (or advanced, kPhase)
    {
        double Rm[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) Rm[a] = x[a] + 0.5 * (Rp[a] - x[a]);
        Smp sm;
        gather3<R, true, kYee>(acc, pc, K, Rm[0], Rm[1], Rm[2], sm);
        Local<R> Lm;
        flags |= local_in_frame<kExact, R>(sm, K, Lm);
        const Gam<R> G = gamma_gca2(Lm, upn, gy, K);
        const R gr = G.g;
        R vc[3] = {(R)0, (R)0, (R)0};
        if (curv) v_curv_g(Lm, upn, G, inv_qm, K, vc);
        const R um = sqrt(uperp_sq(Lm, gy));
        r.ux = (upn * Lm.b[0] + (Lm.vE[0] + vc[0]) * gr) + um * bp[0];
        r.uy = (upn * Lm.b[1] + (Lm.vE[1] + vc[1]) * gr) + um * bp[1];
        r.uz = (upn * Lm.b[2] + (Lm.vE[2] + vc[2]) * gr) + um * bp[2];
    }

    // 6. store
    r.xp = x[0];
    r.yp = x[1];
    r.zp = x[2];
    r.x = wrap_i<R>(Rp[0], pc.b.Lx, pc.b.inv_Lx);
    r.y = wrap_i<R>(Rp[1], pc.b.Ly, pc.b.inv_Ly);
    r.z = wrap_i<R>(Rp[2], pc.Lz, pc.inv_Lz);
    return flags;
}

template <typename R>
GCB_HD uint32_t finite_flag3(const Regs3<R>& r) {
    const bool ok = __builtin_isfinite(r.x) && __builtin_isfinite(r.y) &&
                    __builtin_isfinite(r.z) && __builtin_isfinite(r.ux) &&
                    __builtin_isfinite(r.uy) && __builtin_isfinite(r.uz);
    return ok ? 0u : (uint32_t)ST_NONFINITE;
}

}  // inline namespace GCB_ARITH_NS
}  // namespace gcb
