"""The general-relativistic coupled pusher, written out plainly (float64).

TEST INFRASTRUCTURE: the definition the HIP path's curved-spacetime push is
checked against.

Notation follows the paper's 3+1 split (Sec. 2.3): geometrized units
(c = G = 1, M = 1), positions x^i = (r, theta, phi) in spherical Kerr-Schild
coordinates, covariant spatial four-velocity u_i = (u_r, u_theta, u_phi),
lapse alpha, shift beta^i, spatial metric gamma_ij (inverse gamma^ij),
fields D^i, B^i (contravariant), Gamma = sqrt(1 + gamma^ij u_i u_j).
Position and four-velocity are not staggered (Sec. 3.2).  Vectorised over
particles with torch CPU float64 tensors.

Readings of the paper used here (each is listed with its reason in the
design notes of the repository):
  * Spacetime: Kerr in Kerr-Schild form; axisymmetric, so d/dphi = 0 for the
    metric and the fields, and the geodesic force G_phi vanishes.
  * Fields: D^i and B^i on the nodes of a uniform (r, theta) grid, all six
    components collocated, interpolated with the linear shape function
    (Sec. 4, opening paragraph); points beyond the grid take the value at
    the nearest edge.
  * Local inertial frame (Sec. 2.3, steps 1 and 3): the orthonormal triad of
    the normal observer from the Cholesky factor L of gamma_ij
    (gamma = L L^T): u^ = L^-1 u for covariant, V^ = L^T V for contravariant
    vectors.  There the Lorentz force is alpha q/m (D^ + u^ x B^/Gamma), so a
    half push over dt/2 is the special-relativistic Boris push (c = 1) with
    time step alpha dt/2.  Any other orthonormal triad of the same
    orientation gives the same result up to rounding (the Boris step is
    rotation invariant); the triad is not given in the paper.
  * Geodesic step (Sec. 2.3 step 2; Sec. 2.4 step 2): implicit midpoint rule
    solved by a fixed number K of fixed-point iterations from x^n, u'
    (R^n, u_par'); the reported iteration error is the last increment of
    the position.  Metric functions and their derivatives are analytic.
  * Guiding center (Sec. 2.4): u = u_par b + v_E Gamma + u_perp_g with
    covariant b_i = B_i/B, v_E,i = e_ijk D^j B^k/B^2, kappa from
    gamma^ij v_E,i v_E,j, mu = gamma^ij u_perp_g,i u_perp_g,j/(2 B kappa)
    (m = 1).  The decomposition at R^n = x^n takes Gamma of the full u (as
    in Sec. 3.1); the parallel half pushes add alpha (q/m)(dt/2) D.b (the
    parallel acceleration in the local frame, times the lapse); inside the
    iteration Gamma is eq. grgcalfac and the full four-velocity for G is
    rebuilt with the gyration direction of the step start; the final u
    is rebuilt at R^{n+1} in the same way.
  * Switch (Sec. 3, Sec. 4.2): guiding center iff B > 0,
    rho~/dl < f_rho and D/B < f_E, rho~ = Gamma/(|q/m| B) with Gamma of the
    full u, magnitudes in the metric, and dl the square root of the proper
    area of the particle's (r, theta) cell (eq. volint with n = 2 and the
    2-metric of those coordinates), by 2 x 2 Gauss-Legendre quadrature.
  * A particle whose new position leaves r_min <= r < r_max,
    0 <= theta <= pi is marked GR_ST_OUT and is not advanced again.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from types import SimpleNamespace

import torch

from .ieee import sqrt
from .trig import sincos

F64 = torch.float64

ST_NONFINITE = 1
ST_KAPPA = 2
ST_BZERO = 8
ST_FPRES = 16
GR_ST_OUT = 64      # left the (r, theta) domain; no longer advanced
ST_MIRROR = 128     # (v_perp_g/c)^2 above GRParams.mirror_tol at a decomposition

KAPPA_FLOOR = 1.0e-12
TWO_PI = 2.0 * math.pi

# ---------------------------------------------------------------------------
# metric


class KerrSchild:
    """Kerr spacetime (M = 1, spin a) in spherical Kerr-Schild coordinates.

    With rho^2 = r^2 + a^2 cos^2(theta) and z = 2r/rho^2:
      alpha = (1+z)^-1/2, beta^r = z/(1+z), beta^theta = beta^phi = 0,
      gamma_rr = 1+z, gamma_rphi = -a (1+z) sin^2, gamma_thth = rho^2,
      gamma_phph = sin^2 (rho^2 + a^2 (1+z) sin^2),
      gamma^rr = 1/(1+z) + a^2 sin^2/rho^2, gamma^rphi = a/rho^2,
      gamma^thth = 1/rho^2, gamma^phph = 1/(rho^2 sin^2),
      sqrt(gamma) = sqrt(1+z) rho^2 sin.
    """

    def __init__(self, a: float):
        self.a = float(a)

    def at(self, r, th, derivs: bool = False):
        a = self.a
        a2 = a * a
        sn, cs = sincos(th)
        s2 = sn * sn
        c2 = cs * cs
        rho2 = r * r + a2 * c2
        z = (2.0 * r) / rho2
        opz = 1.0 + z
        sq = sqrt(opz)
        m = SimpleNamespace()
        m.sin, m.cos, m.s2 = sn, cs, s2
        m.alpha = 1.0 / sq
        m.beta_r = z / opz
        m.gu_rr = 1.0 / opz + (a2 * s2) / rho2
        # torch divides a float by a tensor as reciprocal-then-multiply (two
        # roundings); a tensor numerator gives the IEEE quotient
        m.gu_rph = torch.full_like(rho2, a) / rho2
        m.gu_thth = 1.0 / rho2
        m.gu_phph = 1.0 / (rho2 * s2)
        m.gd_rr = opz
        m.gd_rph = -(a * opz) * s2
        m.gd_thth = rho2
        m.gd_phph = s2 * (rho2 + (a2 * opz) * s2)
        m.sqrtg = (sq * rho2) * sn
        if derivs:
            # d/dr and d/dtheta (index 0 and 1) of alpha, beta^r and gamma^ij
            sc = sn * cs
            drho2 = (2.0 * r, -2.0 * (a2 * sc))
            rho4 = rho2 * rho2
            dz = ((2.0 * (a2 * c2 - r * r)) / rho4, (4.0 * (r * (a2 * sc))) / rho4)
            opz2 = opz * opz
            m.dalpha = tuple(-0.5 * (m.alpha / opz) * dz[i] for i in range(2))
            m.dbeta_r = tuple(dz[i] / opz2 for i in range(2))
            m.dgu_rr = (-(dz[0] / opz2) - (a2 * s2) * drho2[0] / rho4,
                        (-(dz[1] / opz2) + (a2 * (2.0 * sc)) / rho2) - (a2 * s2) * drho2[1] / rho4)
            m.dgu_rph = tuple(-(a * drho2[i]) / rho4 for i in range(2))
            m.dgu_thth = tuple(-drho2[i] / rho4 for i in range(2))
            rs2 = rho2 * s2
            m.dgu_phph = (-(drho2[0] * s2) / (rs2 * rs2),
                          -(drho2[1] * s2 + rho2 * (2.0 * sc)) / (rs2 * rs2))
        return m


class FlatSpherical:
    """Flat space in spherical coordinates (alpha = 1, beta = 0), for the pins."""

    a = 0.0

    def at(self, r, th, derivs: bool = False):
        sn, cs = sincos(th)
        s2 = sn * sn
        one = torch.ones_like(r)
        zero = torch.zeros_like(r)
        r2 = r * r
        m = SimpleNamespace()
        m.sin, m.cos, m.s2 = sn, cs, s2
        m.alpha = one
        m.beta_r = zero
        m.gu_rr, m.gu_rph, m.gu_thth, m.gu_phph = one, zero, 1.0 / r2, 1.0 / (r2 * s2)
        m.gd_rr, m.gd_rph, m.gd_thth, m.gd_phph = one, zero, r2, r2 * s2
        m.sqrtg = r2 * sn
        if derivs:
            sc = sn * cs
            m.dalpha = (zero, zero)
            m.dbeta_r = (zero, zero)
            m.dgu_rr = (zero, zero)
            m.dgu_rph = (zero, zero)
            m.dgu_thth = (-2.0 / (r2 * r), zero)
            m.dgu_phph = (-2.0 / (r2 * r * s2), -(2.0 * sc) / (r2 * s2 * s2))
        return m


# ---------------------------------------------------------------------------
# fields on the (r, theta) grid


class GRGrid:
    """D^i, B^i on the nodes of a uniform (r, theta) grid.

    F[k, j, i] is component k (D^r, D^th, D^ph, B^r, B^th, B^ph) at
    r = r_min + i dr, theta = j dth, with dr = (r_max - r_min)/nr and
    dth = pi/nth (nodes i = 0..nr, j = 0..nth).  The value at a point is the
    bilinear interpolation on the surrounding cell; coordinates beyond the
    grid are moved to its edge first.
    """

    def __init__(self, F, r_min: float, r_max: float):
        F = torch.as_tensor(F, dtype=F64)
        assert F.ndim == 3 and F.shape[0] == 6
        self.F = F
        self.nth, self.nr = int(F.shape[1]) - 1, int(F.shape[2]) - 1
        self.r_min, self.r_max = float(r_min), float(r_max)
        self.dr = (self.r_max - self.r_min) / self.nr
        self.dth = math.pi / self.nth
        self.inv_dr = 1.0 / self.dr
        self.inv_dth = 1.0 / self.dth

    def cell(self, r, th):
        """Clamped cell indices and weights of points (r, theta); a NaN
        coordinate is taken at the lower edge."""
        rc = torch.clamp(r, self.r_min, self.r_max)
        tc = torch.clamp(th, 0.0, math.pi)
        rc = torch.where(torch.isnan(rc), self.r_min, rc)
        tc = torch.where(torch.isnan(tc), 0.0, tc)
        xi = (rc - self.r_min) * self.inv_dr
        eta = tc * self.inv_dth
        i = torch.clamp(torch.floor(xi), max=self.nr - 1)
        j = torch.clamp(torch.floor(eta), max=self.nth - 1)
        return i.to(torch.int64), j.to(torch.int64), xi - i, eta - j

    def sample(self, r, th):
        i, j, wx, wy = self.cell(r, th)
        ax, ay = 1.0 - wx, 1.0 - wy
        out = []
        for k in range(6):
            Fk = self.F[k]
            f00, f10 = Fk[j, i], Fk[j, i + 1]
            f01, f11 = Fk[j + 1, i], Fk[j + 1, i + 1]
            out.append(ay * (ax * f00 + wx * f10) + wy * (ax * f01 + wx * f11))
        return tuple(out[:3]), tuple(out[3:])

    def inside(self, r, th):
        return (r >= self.r_min) & (r < self.r_max) & (th >= 0.0) & (th <= math.pi)


def cell_lengths(metric, grid: GRGrid) -> torch.Tensor:
    """dl[j, i] = sqrt(proper area of cell (i, j)) = sqrt(int sqrt(g_rr g_thth) dr dth),
    2 x 2 Gauss-Legendre points per cell (nodes at the centre +- h/sqrt(3))."""
    i = torch.arange(grid.nr, dtype=F64)
    j = torch.arange(grid.nth, dtype=F64)
    J, I = torch.meshgrid(j, i, indexing="ij")
    hr = 0.5 * grid.dr
    ht = 0.5 * grid.dth
    g = 1.0 / math.sqrt(3.0)
    rc = grid.r_min + (I + 0.5) * grid.dr
    tc = (J + 0.5) * grid.dth
    rm, rp = rc - hr * g, rc + hr * g
    tm, tp = tc - ht * g, tc + ht * g

    def f(r, t):
        m = metric.at(r, t)
        return sqrt(m.gd_rr * m.gd_thth)

    tot = ((f(rm, tm) + f(rp, tm)) + f(rm, tp)) + f(rp, tp)
    return sqrt(tot * (hr * ht))


# ---------------------------------------------------------------------------
# pieces of the step


def lower(m, V):
    """gamma_ij V^j."""
    return (m.gd_rr * V[0] + m.gd_rph * V[2], m.gd_thth * V[1], m.gd_rph * V[0] + m.gd_phph * V[2])


def raise_(m, w):
    """gamma^ij w_j."""
    return (m.gu_rr * w[0] + m.gu_rph * w[2], m.gu_thth * w[1], m.gu_rph * w[0] + m.gu_phph * w[2])


def norm2_cov(m, w):
    """gamma^ij w_i w_j."""
    up = raise_(m, w)
    return (w[0] * up[0] + w[1] * up[1]) + w[2] * up[2]


def norm2_con(m, V):
    """gamma_ij V^i V^j."""
    lo = lower(m, V)
    return (V[0] * lo[0] + V[1] * lo[1]) + V[2] * lo[2]


def gamma_of(m, u):
    return sqrt(1.0 + norm2_cov(m, u))


def cross_cov(m, V, W):
    """e_ijk V^j W^k with e_ijk = sqrt(gamma) epsilon_ijk."""
    return (m.sqrtg * (V[1] * W[2] - V[2] * W[1]),
            m.sqrtg * (V[2] * W[0] - V[0] * W[2]),
            m.sqrtg * (V[0] * W[1] - V[1] * W[0]))


def triad(m):
    """Cholesky factor of gamma_ij in the order (r, theta, phi): L11, L22, L31, L33."""
    L11 = sqrt(m.gd_rr)
    L22 = sqrt(m.gd_thth)
    L31 = m.gd_rph / L11
    L33 = sqrt(m.gd_phph - L31 * L31)
    return L11, L22, L31, L33


def half_push(m, D, B, u, qm, dt):
    """Lorentz force over dt/2 in the local frame (Boris, time step alpha dt/2)."""
    L11, L22, L31, L33 = triad(m)
    u1 = u[0] / L11
    u2 = u[1] / L22
    u3 = (u[2] - L31 * u1) / L33
    D1, D2, D3 = L11 * D[0] + L31 * D[2], L22 * D[1], L33 * D[2]
    B1, B2, B3 = L11 * B[0] + L31 * B[2], L22 * B[1], L33 * B[2]
    hq = (qm * (m.alpha * (0.5 * dt))) * 0.5
    umx, umy, umz = u1 + hq * D1, u2 + hq * D2, u3 + hq * D3
    gm = sqrt(1.0 + ((umx * umx + umy * umy) + umz * umz))
    f = hq / gm
    tx, ty, tz = f * B1, f * B2, f * B3
    t2 = (tx * tx + ty * ty) + tz * tz
    g = 2.0 / (1.0 + t2)
    sx, sy, sz = g * tx, g * ty, g * tz
    upx = umx + (umy * tz - umz * ty)
    upy = umy + (umz * tx - umx * tz)
    upz = umz + (umx * ty - umy * tx)
    uqx = umx + (upy * sz - upz * sy)
    uqy = umy + (upz * sx - upx * sz)
    uqz = umz + (upx * sy - upy * sx)
    v1, v2, v3 = uqx + hq * D1, uqy + hq * D2, uqz + hq * D3
    return (L11 * v1, L22 * v2, L31 * v1 + L33 * v3)


def geo_V(m, u, Gam):
    """V^i = alpha gamma^ij u_j / Gamma - beta^i."""
    up = raise_(m, u)
    ag = m.alpha / Gam
    return (ag * up[0] - m.beta_r, ag * up[1], ag * up[2])


def geo_G(m, u, Gam):
    """G_i = -Gamma d_i alpha + u_j d_i beta^j - alpha u_j u_k d_i gamma^jk / (2 Gamma),
    for i = r, theta (G_phi = 0)."""
    ur, ut, up = u
    out = []
    h = m.alpha / (2.0 * Gam)
    for i in range(2):
        q = ((ur * ur) * m.dgu_rr[i] + (2.0 * (ur * up)) * m.dgu_rph[i]) + \
            ((ut * ut) * m.dgu_thth[i] + (up * up) * m.dgu_phph[i])
        out.append((-(Gam * m.dalpha[i]) + ur * m.dbeta_r[i]) - h * q)
    return out[0], out[1]


def gc_local(m, D, B):
    """b (both index positions), B, v_E (covariant), kappa, D_par at a point."""
    flags = torch.zeros(B[0].shape, dtype=torch.uint8)
    Bl = lower(m, B)
    B2 = (B[0] * Bl[0] + B[1] * Bl[1]) + B[2] * Bl[2]
    Bm = sqrt(B2)
    bzero = Bm == 0.0
    inv_B = torch.where(bzero, 0.0, 1.0 / torch.where(bzero, 1.0, Bm))
    flags = flags | torch.where(bzero, ST_BZERO, 0).to(torch.uint8)
    L = SimpleNamespace()
    L.B = Bm
    L.b_up = (B[0] * inv_B, B[1] * inv_B, B[2] * inv_B)
    L.b_dn = (Bl[0] * inv_B, Bl[1] * inv_B, Bl[2] * inv_B)
    DxB = cross_cov(m, D, B)
    ib2 = inv_B * inv_B
    L.vE = (DxB[0] * ib2, DxB[1] * ib2, DxB[2] * ib2)
    om = 1.0 - norm2_cov(m, L.vE)
    low = om < KAPPA_FLOOR
    flags = flags | torch.where(low, ST_KAPPA, 0).to(torch.uint8)
    om = torch.where(low, KAPPA_FLOOR, om)
    L.kappa = 1.0 / sqrt(om)
    L.Dpar = (D[0] * L.b_dn[0] + D[1] * L.b_dn[1]) + D[2] * L.b_dn[2]
    L.flags = flags
    return L


def gamma_gc(L, upar, mu):
    """eq. grgcalfac with m = 1."""
    return L.kappa * sqrt((1.0 + upar * upar) + ((2.0 * mu) * L.B) * L.kappa)


def switch_gca(m, D, B, u, qm, dl, p):
    Bm = sqrt(norm2_con(m, B))
    Dm = sqrt(norm2_con(m, D))
    Gam = gamma_of(m, u)
    safe = torch.where(Bm > 0.0, Bm, 1.0)
    rho = Gam / (torch.abs(qm) * safe)
    return (Bm > 0.0) & (rho / dl < p.f_rho) & (Dm / safe < p.f_E)


def wrap_phi(ph):
    w = ph - TWO_PI * torch.floor(ph / TWO_PI)
    w = torch.where(w < 0.0, w + TWO_PI, w)
    return torch.where(w >= TWO_PI, w - TWO_PI, w)


@dataclass
class GRParams:
    dt: float = 0.04
    f_rho: float = 1.0
    f_E: float = 1.0
    n_iter: int = 4
    fp_tol: float = 1.0e-7
    mirror_tol: float = 0.0   # > 0: ST_MIRROR where (v_perp_g/c)^2 exceeds it


@dataclass
class GRState:
    r: torch.Tensor
    th: torch.Tensor
    ph: torch.Tensor
    ur: torch.Tensor
    uth: torch.Tensor
    uph: torch.Tensor
    qm: torch.Tensor
    status: torch.Tensor

    @staticmethod
    def from_numpy(e) -> "GRState":
        t = lambda a: torch.as_tensor(a, dtype=F64).clone()
        n = len(e.r)
        return GRState(t(e.r), t(e.th), t(e.ph), t(e.ur), t(e.uth), t(e.uph), t(e.qm),
                       torch.zeros(n, dtype=torch.uint8))

    def clone(self) -> "GRState":
        return GRState(*[getattr(self, k).clone() for k in
                         ("r", "th", "ph", "ur", "uth", "uph", "qm", "status")])


def greom_step(metric, grid, x, u, qm, p: GRParams):
    """Strang-split full-orbit step (Sec. 2.3): half push, IMR geodesic, half push."""
    m0 = metric.at(x[0], x[1])
    D0, B0 = grid.sample(x[0], x[1])
    u1 = half_push(m0, D0, B0, u, qm, p.dt)
    xk, uk = x, u1
    res = torch.zeros_like(x[0])
    for _ in range(p.n_iter):
        xb = tuple(0.5 * (xk[i] + x[i]) for i in range(3))
        ub = tuple(0.5 * (uk[i] + u1[i]) for i in range(3))
        mb = metric.at(xb[0], xb[1], derivs=True)
        Gam = gamma_of(mb, ub)
        V = geo_V(mb, ub, Gam)
        G = geo_G(mb, ub, Gam)
        xn = tuple(x[i] + p.dt * V[i] for i in range(3))
        un = (u1[0] + p.dt * G[0], u1[1] + p.dt * G[1], u1[2])
        res = torch.maximum(torch.maximum(torch.abs(xn[0] - xk[0]), torch.abs(xn[1] - xk[1])),
                            torch.abs(xn[2] - xk[2]))
        xk, uk = xn, un
    m1 = metric.at(xk[0], xk[1])
    D1, B1 = grid.sample(xk[0], xk[1])
    u2 = half_push(m1, D1, B1, uk, qm, p.dt)
    return xk, u2, res, torch.zeros_like(x[0], dtype=torch.uint8)


def grgca_step(metric, grid, x, u, qm, p: GRParams):
    """Guiding-center step (Sec. 2.4) inside the coupled step (Sec. 3.2)."""
    m0 = metric.at(x[0], x[1])
    D0, B0 = grid.sample(x[0], x[1])
    L0 = gc_local(m0, D0, B0)
    flags = L0.flags
    Gf = gamma_of(m0, u)
    upar = (L0.b_up[0] * u[0] + L0.b_up[1] * u[1]) + L0.b_up[2] * u[2]
    uperp = tuple((u[i] - upar * L0.b_dn[i]) - L0.vE[i] * Gf for i in range(3))
    up2 = norm2_cov(m0, uperp)
    # the check of the neglect of the mirror terms (Sec. 2.2), c = 1:
    # (v_perp_g/c)^2 = gamma^ij u_perp_g,i u_perp_g,j / Gamma^2 above mirror_tol
    if p.mirror_tol > 0.0:
        flags = flags | torch.where(up2 > p.mirror_tol * (Gf * Gf), ST_MIRROR, 0).to(torch.uint8)
    mu = ((0.5 * up2) / L0.B) / L0.kappa
    mu = torch.where(L0.B > 0.0, mu, 0.0)
    nu = sqrt(up2)
    inv_nu = torch.where(nu > 0.0, 1.0 / torch.where(nu > 0.0, nu, 1.0), 0.0)
    bperp = tuple(uperp[i] * inv_nu for i in range(3))
    # first half push of u_par
    p1 = upar + (qm * (m0.alpha * (0.5 * p.dt))) * L0.Dpar
    Rk, pk = x, p1
    res = torch.zeros_like(x[0])
    for _ in range(p.n_iter):
        Rb = tuple(0.5 * (Rk[i] + x[i]) for i in range(3))
        pb = 0.5 * (pk + p1)
        mb = metric.at(Rb[0], Rb[1], derivs=True)
        Db, Bb = grid.sample(Rb[0], Rb[1])
        Lb = gc_local(mb, Db, Bb)
        flags = flags | Lb.flags
        Gam = gamma_gc(Lb, pb, mu)
        # V~ = alpha (u_par gamma^ij b_j / Gamma + gamma^ij v_E,j) - beta, with
        # gamma^ij b_j = b^i
        vu = raise_(mb, Lb.vE)
        V = (mb.alpha * (pb * (Lb.b_up[0] / Gam) + vu[0]) - mb.beta_r,
             mb.alpha * (pb * (Lb.b_up[1] / Gam) + vu[1]),
             mb.alpha * (pb * (Lb.b_up[2] / Gam) + vu[2]))
        upg = sqrt(((2.0 * mu) * Lb.kappa) * Lb.B)
        ub = tuple((pb * Lb.b_dn[i] + Lb.vE[i] * Gam) + upg * bperp[i] for i in range(3))
        G = geo_G(mb, ub, Gam)
        Gb = G[0] * Lb.b_up[0] + G[1] * Lb.b_up[1]
        Rn = tuple(x[i] + p.dt * V[i] for i in range(3))
        pn = p1 + p.dt * Gb
        res = torch.maximum(torch.maximum(torch.abs(Rn[0] - Rk[0]), torch.abs(Rn[1] - Rk[1])),
                            torch.abs(Rn[2] - Rk[2]))
        Rk, pk = Rn, pn
    m1 = metric.at(Rk[0], Rk[1])
    D1, B1 = grid.sample(Rk[0], Rk[1])
    L1 = gc_local(m1, D1, B1)
    flags = flags | L1.flags
    upar1 = pk + (qm * (m1.alpha * (0.5 * p.dt))) * L1.Dpar
    Gam1 = gamma_gc(L1, upar1, mu)
    upg1 = sqrt(((2.0 * mu) * L1.kappa) * L1.B)
    un = tuple((upar1 * L1.b_dn[i] + L1.vE[i] * Gam1) + upg1 * bperp[i] for i in range(3))
    return Rk, un, res, flags


def step(metric, grid, dl, st: GRState, p: GRParams):
    """One coupled step (Sec. 3.2) of every particle; returns (state, S, res).
    S: 0 guiding center, 1 full orbit, 2 not advanced (outside the domain)."""
    x = (st.r, st.th, st.ph)
    u = (st.ur, st.uth, st.uph)
    active = ((st.status & GR_ST_OUT) == 0) & grid.inside(st.r, st.th)
    m = metric.at(st.r, st.th)
    D, B = grid.sample(st.r, st.th)
    i, j, _, _ = grid.cell(st.r, st.th)
    dlp = dl[j, i]
    gca = switch_gca(m, D, B, u, st.qm, dlp, p)
    xg, ug, rg, fg = grgca_step(metric, grid, x, u, st.qm, p)
    xb, ub, rb, fb = greom_step(metric, grid, x, u, st.qm, p)
    xn = tuple(torch.where(gca, xg[k], xb[k]) for k in range(3))
    un = tuple(torch.where(gca, ug[k], ub[k]) for k in range(3))
    res = torch.where(gca, rg, rb)
    fl = torch.where(gca, fg, fb)
    fl = fl | torch.where(res > p.fp_tol, ST_FPRES, 0).to(torch.uint8)
    fin = torch.isfinite(xn[0]) & torch.isfinite(xn[1]) & torch.isfinite(xn[2]) & \
        torch.isfinite(un[0]) & torch.isfinite(un[1]) & torch.isfinite(un[2])
    fl = fl | torch.where(fin, 0, ST_NONFINITE).to(torch.uint8)
    out = ~grid.inside(xn[0], xn[1])
    fl = fl | torch.where(out, GR_ST_OUT, 0).to(torch.uint8)
    new = GRState(torch.where(active, xn[0], st.r), torch.where(active, xn[1], st.th),
                  torch.where(active, wrap_phi(xn[2]), st.ph),
                  torch.where(active, un[0], st.ur), torch.where(active, un[1], st.uth),
                  torch.where(active, un[2], st.uph), st.qm,
                  torch.where(active, st.status | fl,
                              st.status | torch.where(grid.inside(st.r, st.th), 0,
                                                      GR_ST_OUT).to(torch.uint8)))
    S = torch.where(active, torch.where(gca, 0, 1), 2).to(torch.uint8)
    return new, S, torch.where(active, res, 0.0)


def push(metric, grid, st: GRState, p: GRParams, n_steps: int, trace: bool = False):
    dl = cell_lengths(metric, grid)
    S_all = []
    res = torch.zeros_like(st.r)
    for _ in range(n_steps):
        st, S, r = step(metric, grid, dl, st, p)
        res = torch.maximum(res, r)
        if trace:
            S_all.append(S)
    return st, (torch.stack(S_all) if trace else None), res
