"""The coupled guiding-center / Boris pusher, written out plainly (float64).

TEST INFRASTRUCTURE: the definition the HIP path is checked against.

Notation follows the paper (Gaussian units with explicit c; u is the spatial
part of the four-velocity in velocity units, Gamma = sqrt(1 + u^2/c^2)).
Vectorised over particles with torch CPU float64 tensors; every particle is
independent, so this is the per-particle algorithm applied elementwise.

Readings of the paper used here (each is listed with its reason in the
design notes of the repository):
  * 2D3V: positions (x, y); u, E, B have three components; d/dz = 0.
  * Boris push (Sec. 2.1, cited there, formula not printed): the standard
    relativistic form -- half electric kick, magnetic rotation with
    t = (q dt/2m) B/(c Gamma^-), s = 2t/(1+t^2), half electric kick.
  * Simplified guiding-center split u = u_par b + v_E Gamma + u_perp_g with
    v_E = c E x B / B^2 and kappa = (1 - v_E^2/c^2)^(-1/2) (Sec. 2.2, the
    paper's own simplification); magnetic moment mu/m = u_perp_g^2/(2 B kappa).
  * Curvature drift (Sec. 2.2, eq. curvdrift) with d b computed by the chain
    rule from the interpolated gradients of the B components.
  * Switch (Sec. 4.1): guiding center iff B > 0, rho~/dl < f_rho and
    E/B < f_E, with rho~ = c^2 Gamma/(|q/m| B) the gyro-radius of a particle
    whose whole four-velocity Gamma c is perpendicular, Gamma from the full u
    and fields at x^n; dl = sqrt(dx dy) (Sec. 3).
  * Conversions (Sec. 3.1): every guiding-center step decomposes u at
    R^{n-1/2} = (x^n + x^{n-1})/2 (minimum image), with Gamma of the full u,
    and reconstructs at R^{n+1/2} = (R^n + R^{n+1})/2 with the gyration
    direction held fixed.
  * Parallel update with curvature (Sec. 2.2.2): the positive root of the
    quadratic k1 G^2 + k2 G + k3 = 0, evaluated without cancellation.
  * Fixed point for R^{n+1} (Sec. 2.2.1/2.2.2): a fixed number K of
    iterations R^{k+1} = R^k - H(R^k) from R^0 = R^n; the last increment
    |R^K - R^{K-1}| is the reported iteration error.
  * Periodic box; stored positions are wrapped into [0, L).
  * Params.exact_frame: b*, the exact v_E and kappa and E_par = E'/kappa of
    the frame of Sec. 2.2 (frame.py) in place of b, c E x B/B^2 and E.b;
    with the curvature scheme also (b*.grad)b* and (v_E.grad)b* from the
    gradients of b* (frame.py); everything else unchanged.
  * Params.gyration: how the gyration speed enters a guiding-center step.
    GYR_MU (the paper's choice, eq. dmudt): mu is conserved, so wherever
    u_perp_g^2 = 2 mu B kappa/m appears (eq. lfacgca2, k3 of the quadratic,
    the reconstruction) it is evaluated with B and kappa of that point.
    GYR_UPERP (the energy-conserving alternative the paper describes after
    the SRGCA system): u_perp_g keeps the value of the decomposition over
    the whole step.  GYR_ZERO (mu = 0, which the paper allows where
    radiation has removed the gyration, Sec. 2.2 before Sec. 2.2.1): the
    decomposition's gyration is discarded.  GYR_PHASE (mu conserved, and the
    gyration phase evolved by the extra equation Sec. 3.1 allows in place of
    holding the gyration direction): over the step the gyration direction is
    turned about b at R^n by the angle -(q/m) B dt/(c kappa Gamma), the
    gyration frequency of a particle whose guiding center drifts with v_E
    (in the drift frame q B'/(m c gamma') with B' = B/kappa, and the lab time
    runs kappa times faster; Gamma = kappa gamma' is eq. lfacgca2), with
    Gamma at R^n and the mean of u_par before and after the parallel update.
  * Params.mirror (curvature scheme only): the mirror force and the grad-B
    drift, which Sec. 2.2 names and leaves out of the reduced equations, with
    the paper's mu: du_par/dt gains -(mu/(m kappa Gamma)) b.grad|B| and the
    bracket of the curvature drift gains (mu/(m kappa Gamma)) grad|B|.
    grad(B/kappa) is taken as grad|B|/kappa (the gradient of kappa, which
    needs that of E, is left out; with E = 0 both are the textbook
    relativistic terms).  The force is time-centred by one
    predictor-corrector pass on 1/Gamma; the decomposition and the
    reconstruction keep the paper's u_perp_d = Gamma (v_E + v_c).
  * Params.mirror_tol (> 0): the check of the neglect of the mirror terms
    that Sec. 2.2 asks for, as a status bit: ST_MIRROR where
    (v_perp_g/c)^2 = u_perp_g^2/(Gamma^2 c^2) at a decomposition exceeds it.
"""
from __future__ import annotations

from dataclasses import dataclass
from types import SimpleNamespace

import torch

from .ieee import sqrt
from .trig import sincos

F64 = torch.float64

# sticky per-particle status bits
ST_NONFINITE = 1   # a non-finite position or four-velocity was produced
ST_KAPPA = 2       # v_E >= c at a guiding-center evaluation (kappa clamped)
ST_QUAD = 4        # no admissible root of the parallel-update quadratic
ST_BZERO = 8       # B = 0 at a guiding-center evaluation point
ST_FPRES = 16      # fixed-point iteration error above tolerance
ST_MIRROR = 128    # (v_perp_g/c)^2 above Params.mirror_tol at a decomposition

# gyration handling of a guiding-center step (Params.gyration)
GYR_MU = 0      # mu conserved (eq. dmudt)
GYR_UPERP = 1   # u_perp_g constant over the step
GYR_ZERO = 2    # mu = 0
GYR_PHASE = 3   # mu conserved, the gyration phase advanced over the step

KAPPA_FLOOR = 1.0e-12   # lower clamp of 1 - v_E^2/c^2
D_FLOOR = 1.0e-12       # |1 - (dt/2) v_E.(b.grad)b| below this: no division


@dataclass
class Params:
    dt: float = 1.0
    c: float = 0.45
    f_rho: float = 0.4
    f_E: float = 1.0
    curvature: bool = True
    n_iter: int = 4
    fp_tol: float = 1.0e-7
    Lx: float = 0.0
    Ly: float = 0.0
    dl: float = 1.0   # effective cell size sqrt(dx*dy)
    exact_frame: bool = False   # b*, exact v_E and their curvature terms (frame.py)
    gyration: int = GYR_MU      # GYR_MU, GYR_UPERP, GYR_ZERO or GYR_PHASE
    mirror: bool = False        # mirror force and grad-B drift (curvature scheme only)
    mirror_tol: float = 0.0     # > 0: flag ST_MIRROR where (v_perp_g/c)^2 exceeds it

    @property
    def c2(self) -> float:
        return self.c * self.c

    @property
    def inv_c2(self) -> float:
        return 1.0 / (self.c * self.c)


@dataclass
class State:
    x: torch.Tensor
    y: torch.Tensor
    xp: torch.Tensor
    yp: torch.Tensor
    ux: torch.Tensor
    uy: torch.Tensor
    uz: torch.Tensor
    qm: torch.Tensor
    status: torch.Tensor   # uint8

    @staticmethod
    def from_numpy(ens) -> "State":
        t = lambda a: torch.as_tensor(a, dtype=F64).clone()
        return State(t(ens.x), t(ens.y), t(ens.xp), t(ens.yp), t(ens.ux),
                     t(ens.uy), t(ens.uz), t(ens.qm),
                     torch.zeros(ens.x.shape[0], dtype=torch.uint8))

    def clone(self) -> "State":
        return State(*(getattr(self, k).clone() for k in
                       ("x", "y", "xp", "yp", "ux", "uy", "uz", "qm", "status")))

    def subset(self, idx) -> "State":
        return State(*(getattr(self, k)[idx] for k in
                       ("x", "y", "xp", "yp", "ux", "uy", "uz", "qm", "status")))


# --------------------------------------------------------------------------
# geometry of the periodic box


def wrap(x, L: float):
    """Map a coordinate into [0, L)."""
    w = x - L * torch.floor(x / L)
    w = torch.where(w < 0.0, w + L, w)
    return torch.where(w >= L, w - L, w)


def min_image(d, L: float):
    """Shortest periodic representative of a displacement (ties to -L/2)."""
    return d - L * torch.floor(d / L + 0.5)


# --------------------------------------------------------------------------
# local field quantities at a point (Sec. 2.2)


def local(prov, X, Y, p: Params):
    """b, v_E, kappa, E_par and the curvature terms at points (X, Y).

    Returns a namespace with B, inv_B, b=(bx,by,bz), vE, kappa, Epar,
    bgb = (b.grad)b, vgb = (v_E.grad)b, A = v_E.(b.grad)b,
    C = v_E.(v_E.grad)b, gB = grad|B| (x, y), the raw E and B vectors and
    status flags.  With p.exact_frame, the quantities of the exact frame
    (frame.py).
    """
    if p.exact_frame:
        from .frame import local_exact
        return local_exact(prov, X, Y, p)
    s = prov(X, Y)
    Ex, Ey, Ez = s.E
    Bx, By, Bz = s.B
    B2 = (Bx * Bx + By * By) + Bz * Bz
    B = sqrt(B2)
    bzero = B == 0.0
    inv_B = torch.where(bzero, 0.0, 1.0 / torch.where(bzero, 1.0, B))
    bx, by, bz = Bx * inv_B, By * inv_B, Bz * inv_B
    # E x B drift, v_E = c E x B / B^2
    sc = p.c * (inv_B * inv_B)
    vEx = sc * (Ey * Bz - Ez * By)
    vEy = sc * (Ez * Bx - Ex * Bz)
    vEz = sc * (Ex * By - Ey * Bx)
    vE2 = (vEx * vEx + vEy * vEy) + vEz * vEz
    om = 1.0 - vE2 * p.inv_c2
    kflag = om < KAPPA_FLOOR
    om = torch.where(kflag, KAPPA_FLOOR, om)
    kappa = 1.0 / sqrt(om)
    Epar = (Ex * bx + Ey * by) + Ez * bz
    # d_j b_i = (d_j B_i - b_i d_j|B|)/B with d_j|B| = b . d_j B
    db, gB = [], []
    for j in range(2):
        gx, gy, gz = s.dB[j]
        dBn = (bx * gx + by * gy) + bz * gz
        gB.append(dBn)
        db.append(((gx - bx * dBn) * inv_B,
                   (gy - by * dBn) * inv_B,
                   (gz - bz * dBn) * inv_B))
    bgb = tuple(bx * db[0][i] + by * db[1][i] for i in range(3))
    vgb = tuple(vEx * db[0][i] + vEy * db[1][i] for i in range(3))
    A = (vEx * bgb[0] + vEy * bgb[1]) + vEz * bgb[2]
    C = (vEx * vgb[0] + vEy * vgb[1]) + vEz * vgb[2]
    flags = (torch.where(kflag, ST_KAPPA, 0) | torch.where(bzero, ST_BZERO, 0))
    return SimpleNamespace(E=(Ex, Ey, Ez), Bv=(Bx, By, Bz), B=B, inv_B=inv_B,
                           b=(bx, by, bz), vE=(vEx, vEy, vEz), kappa=kappa,
                           Epar=Epar, bgb=bgb, vgb=vgb, A=A, C=C, gB=tuple(gB),
                           flags=flags.to(torch.uint8))


def gyration(up2, Lh, p: Params):
    """Gyration state of a guiding-center step from u_perp_g^2 at the
    decomposition point: mu/m = u_perp_g^2/(2 B kappa), or u_perp_g^2 itself
    when it is held constant (Params.gyration)."""
    mu = ((0.5 * up2) * Lh.inv_B) / Lh.kappa
    if p.gyration == GYR_ZERO:
        mu = torch.zeros_like(mu)
    return SimpleNamespace(mu=mu, up2=up2, fixed=p.gyration == GYR_UPERP)


def rotate_about(b, d, ang):
    """d turned by the angle ang (right-handed) about the unit vector b:
    d cos + (b x d) sin + b (b.d)(1 - cos) (Rodrigues' rotation formula)."""
    sn, cs = sincos(ang)
    bd = (b[0] * d[0] + b[1] * d[1]) + b[2] * d[2]
    cx = b[1] * d[2] - b[2] * d[1]
    cy = b[2] * d[0] - b[0] * d[2]
    cz = b[0] * d[1] - b[1] * d[0]
    w = bd * (1.0 - cs)
    return ((d[0] * cs + cx * sn) + b[0] * w,
            (d[1] * cs + cy * sn) + b[1] * w,
            (d[2] * cs + cz * sn) + b[2] * w)


def phase_advance(Ln, upar, upn, gy, qm, bp, p: Params):
    """The gyration direction bp after one step of the gyro-phase option:
    turned about b at R^n by -(q/m) B dt/(c kappa Gamma), Gamma from eq.
    lfacgca2 at R^n with the mean of u_par^{n-1/2} and u_par^{n+1/2}."""
    gn = gamma_gca(Ln, 0.5 * (upar + upn), gy, p)
    ang = -((qm * Ln.B) * p.dt) / ((p.c * Ln.kappa) * gn)
    return rotate_about(Ln.b, bp, ang)


def mirror_check(up2, gf, p: Params):
    """ST_MIRROR where (v_perp_g/c)^2 = u_perp_g^2/(Gamma^2 c^2) exceeds
    p.mirror_tol (> 0) at the decomposition, Gamma of the full u: the check
    Sec. 2.2 asks for of the neglect of the mirror terms, whose size against
    the curvature terms grows as v_perp_g^2."""
    if not p.mirror_tol > 0.0:
        return torch.zeros_like(up2, dtype=torch.uint8)
    return torch.where(up2 * p.inv_c2 > p.mirror_tol * (gf * gf), ST_MIRROR, 0).to(torch.uint8)


def conserved_mu(mu):
    """The gyration state for a given mu/m, conserved over the step."""
    return SimpleNamespace(mu=mu, up2=None, fixed=False)


def uperp_sq(L, gy):
    """u_perp_g^2 at a point: 2 mu B kappa/m, or the held value."""
    if gy.fixed:
        return gy.up2
    return ((2.0 * gy.mu) * L.B) * L.kappa


def gamma_gca(L, upar, gy, p: Params):
    """Gamma(R, u_par) = kappa sqrt(1 + (u_par^2 + 2 mu B kappa / m)/c^2) (eq. lfacgca2)."""
    uperp2 = uperp_sq(L, gy)
    return L.kappa * sqrt(1.0 + (upar * upar + uperp2) * p.inv_c2)


def v_curv(L, upar, gam, inv_qm, p: Params, gy=None):
    """Curvature drift (eq. curvdrift):
    (m c kappa^2/(q B)) b x [ (u_par^2/Gamma)(b.grad)b + u_par (v_E.grad)b ].

    With a gyration state gy (the mirror option), the grad-B drift joins the
    bracket as (mu/(m kappa Gamma)) grad|B|: with kappa = 1 this is
    c u_perp^2/(2 (q/m) Gamma B^2) b x grad|B|, the relativistic grad-B
    drift.  grad(B/kappa) is taken as grad|B|/kappa (the gradient of kappa,
    which needs that of E, is left out)."""
    pre = ((p.c * L.kappa) * L.kappa) * (L.inv_B * inv_qm)
    a1 = (upar * upar) / gam
    w = [a1 * L.bgb[i] + upar * L.vgb[i] for i in range(3)]
    if gy is not None:
        a3 = (gy.mu / L.kappa) / gam
        for i in range(len(L.gB)):
            w[i] = w[i] + a3 * L.gB[i]
    bx, by, bz = L.b
    return (pre * (by * w[2] - bz * w[1]),
            pre * (bz * w[0] - bx * w[2]),
            pre * (bx * w[1] - by * w[0]))


# --------------------------------------------------------------------------
# switch (Sec. 3 criteria, Sec. 4.1 step function)


def switch_gca(s, ux, uy, uz, qm, p: Params):
    """True where the guiding-center system is used (S = 0).

    s is a FieldSample at x^n.  GCA iff B > 0 and rho~/dl < f_rho and
    E/B < f_E with rho~ = c^2 Gamma / (|q/m| B).
    """
    Ex, Ey, Ez = s.E
    Bx, By, Bz = s.B
    B = sqrt((Bx * Bx + By * By) + Bz * Bz)
    E = sqrt((Ex * Ex + Ey * Ey) + Ez * Ez)
    pos = B > 0.0
    inv_B = torch.where(pos, 1.0 / torch.where(pos, B, 1.0), 0.0)
    gf = sqrt(1.0 + ((ux * ux + uy * uy) + uz * uz) * p.inv_c2)
    inv_absqm = torch.abs(1.0 / qm)
    rho = ((p.c2 * gf) * inv_B) * inv_absqm
    return pos & (rho * (1.0 / p.dl) < p.f_rho) & (E * inv_B < p.f_E)


# --------------------------------------------------------------------------
# full equations of motion: relativistic Boris (Sec. 2.1)


def boris(E, B, ux, uy, uz, qm, p: Params):
    """u^{n-1/2} -> u^{n+1/2} with fields at x^n."""
    Ex, Ey, Ez = E
    Bx, By, Bz = B
    hq = (qm * p.dt) * 0.5
    umx, umy, umz = ux + hq * Ex, uy + hq * Ey, uz + hq * Ez
    gm = sqrt(1.0 + ((umx * umx + umy * umy) + umz * umz) * p.inv_c2)
    f = hq / (p.c * gm)
    tx, ty, tz = f * Bx, f * By, f * Bz
    t2 = (tx * tx + ty * ty) + tz * tz
    g = 2.0 / (1.0 + t2)
    sx, sy, sz = g * tx, g * ty, g * tz
    # u' = u- + u- x t ;  u+ = u- + u' x s
    upx = umx + (umy * tz - umz * ty)
    upy = umy + (umz * tx - umx * tz)
    upz = umz + (umx * ty - umy * tx)
    uqx = umx + (upy * sz - upz * sy)
    uqy = umy + (upz * sx - upx * sz)
    uqz = umz + (upx * sy - upy * sx)
    return uqx + hq * Ex, uqy + hq * Ey, uqz + hq * Ez


def boris_step(s, st: State, p: Params):
    """Full Boris step: new (x, y, u); x^{n+1} = x^n + dt u^{n+1/2}/Gamma^{n+1/2}."""
    ux, uy, uz = boris(s.E, s.B, st.ux, st.uy, st.uz, st.qm, p)
    gn = sqrt(1.0 + ((ux * ux + uy * uy) + uz * uz) * p.inv_c2)
    inv_g = 1.0 / gn
    xn = st.x + p.dt * (ux * inv_g)
    yn = st.y + p.dt * (uy * inv_g)
    return wrap(xn, p.Lx), wrap(yn, p.Ly), ux, uy, uz


# --------------------------------------------------------------------------
# guiding-center leapfrog (Sec. 2.2.1, 2.2.2) inside the coupled step (Sec. 3.1)


def parallel_update(Ln, upar, gy, qm, p: Params, shift=None):
    """u_par^{n-1/2} -> u_par^{n+1/2} at R^n; returns (u_par_new, flags).

    Without curvature: u_par + (q dt/m) E_par.  With curvature: solve
    eq. dupardtcase2disc via the quadratic for Gamma(R^n, u_par^{n+1/2})
    and take its positive root, then eq. dupardtcase2discsol.  `shift`
    (the mirror option) is an explicit change of u_par over the step that is
    subtracted from the known part of the update.
    """
    dtqm = qm * p.dt
    if not p.curvature:
        return upar + dtqm * Ln.Epar, torch.zeros_like(upar, dtype=torch.uint8)
    h = 0.5 * p.dt
    A, C = Ln.A, Ln.C
    G0 = gamma_gca(Ln, upar, gy, p)
    upr = (upar * (1.0 + h * A) + dtqm * Ln.Epar) + (h * G0) * C
    if shift is not None:
        upr = upr - shift
    D = 1.0 - h * A
    DD = D * D
    k1 = (h * h) * (C * C) - (p.c2 * DD) / (Ln.kappa * Ln.kappa)
    k2 = (upr * p.dt) * C
    k3 = upr * upr + (p.c2 + uperp_sq(Ln, gy)) * DD
    disc = k2 * k2 - (4.0 * k1) * k3
    dok = torch.abs(D) >= D_FLOOR
    ok = (k1 < 0.0) & (disc >= 0.0) & dok
    sq = sqrt(torch.where(disc >= 0.0, disc, 0.0))
    # positive root without cancellation: (k2 + sq)/(-2 k1) if k2 >= 0,
    # else 2 k3/(sq - k2)
    pos_k2 = k2 >= 0.0
    num = torch.where(pos_k2, k2 + sq, 2.0 * k3)
    den = torch.where(pos_k2, -2.0 * k1, sq - k2)
    den = torch.where(ok & (den > 0.0), den, 1.0)
    gp = num / den
    ok = ok & (gp > 0.0) & torch.isfinite(gp)
    Ds = torch.where(dok, D, 1.0)
    unew = (upr + (h * gp) * C) / Ds
    # fallbacks: neglect the implicit Gamma term, or the curvature terms
    gfb = gamma_gca(Ln, upr / Ds, gy, p)
    ufb = (upr + (h * gfb) * C) / Ds
    uexp = upar + dtqm * Ln.Epar
    if shift is not None:
        uexp = uexp - shift
    out = torch.where(ok, unew, torch.where(dok, ufb, uexp))
    flags = torch.where(ok, 0, ST_QUAD).to(torch.uint8)
    return out, flags


def mirror_parallel(Ln, upar, gy, qm, p: Params):
    """Parallel update with the mirror force -(mu/(m kappa Gamma)) b.grad|B|
    added to eq. dupardt (the mirror option; with kappa = 1 it is the
    relativistic mirror force, which keeps u_par^2 + 2 mu B/m constant).
    Gamma is centred by one predictor-corrector pass: the predictor takes
    1/Gamma(R^n, u_par^{n-1/2}), the corrector the mean of that and
    1/Gamma(R^n, u_par*) with u_par* the predictor's result.  Returns
    (u_par_new, flags of both passes)."""
    if len(Ln.gB) == 2:
        M = Ln.b[0] * Ln.gB[0] + Ln.b[1] * Ln.gB[1]
    else:
        M = (Ln.b[0] * Ln.gB[0] + Ln.b[1] * Ln.gB[1]) + Ln.b[2] * Ln.gB[2]
    ds = (p.dt * (gy.mu / Ln.kappa)) * M
    G0 = gamma_gca(Ln, upar, gy, p)
    u1, f1 = parallel_update(Ln, upar, gy, qm, p, ds / G0)
    G1 = gamma_gca(Ln, u1, gy, p)
    u2, f2 = parallel_update(Ln, upar, gy, qm, p, ds * (0.5 * (1.0 / G0 + 1.0 / G1)))
    return u2, f1 | f2


def _drift_terms(L, upar_new, gy, inv_qm, p: Params):
    """u_par b/Gamma + v_E + v_c at a point, x and y components."""
    g = gamma_gca(L, upar_new, gy, p)
    a = upar_new / g
    if p.curvature:
        vc = v_curv(L, upar_new, g, inv_qm, p, gy if p.mirror else None)
        return ((a * L.b[0] + L.vE[0]) + vc[0], (a * L.b[1] + L.vE[1]) + vc[1])
    return (a * L.b[0] + L.vE[0], a * L.b[1] + L.vE[1])


def gca_step(prov, st: State, p: Params):
    """One guiding-center step for the particles in `st`.

    Returns (x, y, xp, yp, ux, uy, uz, flags, residual).
    """
    x, y, qm = st.x, st.y, st.qm
    ux, uy, uz = st.ux, st.uy, st.uz
    inv_qm = 1.0 / qm
    assert p.curvature or not p.mirror, "the mirror terms ride on the curvature scheme"
    assert not (p.exact_frame and p.mirror), "the mirror terms go with the reduced frame"
    flags = torch.zeros_like(x, dtype=torch.uint8)

    # 1. switch to guiding-center variables at R^{n-1/2} = (x^n + x^{n-1})/2
    Rhx = x - 0.5 * min_image(x - st.xp, p.Lx)
    Rhy = y - 0.5 * min_image(y - st.yp, p.Ly)
    Lh = local(prov, Rhx, Rhy, p)
    flags |= Lh.flags
    bx, by, bz = Lh.b
    upar = (ux * bx + uy * by) + uz * bz
    gf = sqrt(1.0 + ((ux * ux + uy * uy) + uz * uz) * p.inv_c2)
    if p.curvature:
        vc = v_curv(Lh, upar, gf, inv_qm, p)
    else:
        z = torch.zeros_like(x)
        vc = (z, z, z)
    upx = (ux - upar * bx) - (Lh.vE[0] + vc[0]) * gf
    upy = (uy - upar * by) - (Lh.vE[1] + vc[1]) * gf
    upz = (uz - upar * bz) - (Lh.vE[2] + vc[2]) * gf
    up2 = (upx * upx + upy * upy) + upz * upz
    flags |= mirror_check(up2, gf, p)
    gy = gyration(up2, Lh, p)
    nu = sqrt(up2)
    inv_nu = torch.where(nu > 0.0, 1.0 / torch.where(nu > 0.0, nu, 1.0), 0.0)
    bpx, bpy, bpz = upx * inv_nu, upy * inv_nu, upz * inv_nu

    # 2.-3. fields at R^n = x^n and the parallel four-velocity update
    Ln = local(prov, x, y, p)
    flags |= Ln.flags
    if p.mirror:
        upn, qf = mirror_parallel(Ln, upar, gy, qm, p)
    else:
        upn, qf = parallel_update(Ln, upar, gy, qm, p)
    flags |= qf
    if p.gyration == GYR_PHASE:
        bpx, bpy, bpz = phase_advance(Ln, upar, upn, gy, qm, (bpx, bpy, bpz), p)

    # 4. R^{n+1} by fixed-point iteration R^{k+1} = R^k - H(R^k), R^0 = R^n
    h = 0.5 * p.dt
    Fn = _drift_terms(Ln, upn, gy, inv_qm, p)
    Rx, Ry = x, y
    res = torch.zeros_like(x)
    for k in range(p.n_iter):
        if k == 0:
            Fk = Fn
        else:
            Lk = local(prov, Rx, Ry, p)
            flags |= Lk.flags
            Fk = _drift_terms(Lk, upn, gy, inv_qm, p)
        Rx_new = x + h * (Fn[0] + Fk[0])
        Ry_new = y + h * (Fn[1] + Fk[1])
        res = torch.maximum(torch.abs(Rx_new - Rx), torch.abs(Ry_new - Ry))
        Rx, Ry = Rx_new, Ry_new
    flags |= torch.where(res > p.fp_tol, ST_FPRES, 0).to(torch.uint8)

    # 5. back to particle variables at R^{n+1/2} = (R^n + R^{n+1})/2
    Rmx = x + 0.5 * (Rx - x)
    Rmy = y + 0.5 * (Ry - y)
    Lm = local(prov, Rmx, Rmy, p)
    flags |= Lm.flags
    gr = gamma_gca(Lm, upn, gy, p)
    if p.curvature:
        vcm = v_curv(Lm, upn, gr, inv_qm, p)
    else:
        z = torch.zeros_like(x)
        vcm = (z, z, z)
    um = sqrt(uperp_sq(Lm, gy))
    bmx, bmy, bmz = Lm.b
    uxn = (upn * bmx + (Lm.vE[0] + vcm[0]) * gr) + um * bpx
    uyn = (upn * bmy + (Lm.vE[1] + vcm[1]) * gr) + um * bpy
    uzn = (upn * bmz + (Lm.vE[2] + vcm[2]) * gr) + um * bpz

    # 6. store x^{n+1} (wrapped), x^n as the previous position, u^{n+1/2}
    return (wrap(Rx, p.Lx), wrap(Ry, p.Ly), x, y, uxn, uyn, uzn, flags, res)


# --------------------------------------------------------------------------
# coupled step (Sec. 3.1) and driver


def _finite_flag(*vals):
    ok = torch.ones_like(vals[0], dtype=torch.bool)
    for v in vals:
        ok &= torch.isfinite(v)
    return torch.where(ok, 0, ST_NONFINITE).to(torch.uint8)


def step(prov, st: State, p: Params):
    """Advance every particle by one step. Returns (new_state, S, residual).

    S is a bool tensor, True where the Boris push was used (S = 1).
    """
    s = prov(st.x, st.y)
    gca = switch_gca(s, st.ux, st.uy, st.uz, st.qm, p)
    S = ~gca
    ib = torch.nonzero(S).flatten()
    ig = torch.nonzero(gca).flatten()

    xs = [st.x, st.y, st.xp, st.yp, st.ux, st.uy, st.uz]
    status = st.status.clone()
    res = torch.zeros_like(st.x)
    if ib.numel():
        sb = type(s)(tuple(v[ib] for v in s.E), tuple(v[ib] for v in s.B), s.dB)
        sub = st.subset(ib)
        bx_, by_, bux, buy, buz = boris_step(sb, sub, p)
        vals = [bx_, by_, sub.x, sub.y, bux, buy, buz]
        xs = [a.index_put((ib,), v) for a, v in zip(xs, vals)]
        status = status.index_put((ib,), status[ib] | _finite_flag(*vals[:2], *vals[4:]))
    if ig.numel():
        sub = st.subset(ig)
        out = gca_step(prov, sub, p)
        vals = list(out[:7])
        xs = [a.index_put((ig,), v) for a, v in zip(xs, vals)]
        fl = out[7] | _finite_flag(*vals[:2], *vals[4:])
        status = status.index_put((ig,), status[ig] | fl)
        res = res.index_put((ig,), out[8])
    new = State(*xs, st.qm, status)
    return new, S, res


def push(prov, st: State, p: Params, n_steps: int, trace: bool = False):
    """Run n_steps coupled steps. Returns (state, S_trace or None, max residual).

    S_trace has shape (n_steps, n), dtype uint8, 1 where Boris was used.
    """
    tr = [] if trace else None
    maxres = torch.zeros_like(st.x)
    for _ in range(n_steps):
        st, S, res = step(prov, st, p)
        maxres = torch.maximum(maxres, res)
        if trace:
            tr.append(S.to(torch.uint8))
    return st, (torch.stack(tr) if trace else None), maxres
