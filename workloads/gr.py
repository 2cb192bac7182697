"""Seeded synthetic inputs for the curved-spacetime push: a black-hole
magnetosphere shaped like the paper's Sec. 4.2 snapshot (which is not
available), on a uniform (r, theta) grid of spherical Kerr-Schild coordinates.

Fields (contravariant D^i, B^i on the nodes r_i = r_min + i dr,
theta_j = j pi/nth, all six components at the nodes), in geometrized units:
  * a split monopole, B^r = B0 tanh(cos(theta)/w)/r^2, whose sign flips across
    an equatorial current sheet of angular half-width w;
  * the toroidal field of field lines rotating at Omega_F = Omega_H/2
    (Omega_H = a/(2 r_+) for the horizon r_+ = 1 + sqrt(1 - a^2)), taken from
    the flat-space rotating monopole: B^phi = -Omega_F B^r (Omega_F times
    `rotation`, 1 by default, for weakly rotating variants);
  * the matching rotational electric field of the same flat-space solution,
    D^theta = -Omega_F sin(theta) B^r (so D.B = 0 away from the sheet),
    plus a reconnection field in the sheet, D^r = E_rec B0 / r^2 * sech^2
    (cos(theta)/w), which gives particles there a parallel electric field;
  * optionally (`inflow` > 0) a toroidal electric field D^phi = inflow B0/r^3,
    whose drift D x B carries field lines of both hemispheres toward the
    sheet at a speed of about inflow sin(theta) c, and which exceeds B inside
    the sheet (the stand-in of the near-sheet test of Sec. 4.2).
These are closed-form samples; none of the pusher's arithmetic is used.

Particles: positions uniform in r and in cos(theta) over a band away from the
poles, phi uniform; four-velocities drawn as for the flat-space workloads
(half Maxwell-Juttner theta_MJ = 1, half a Gamma^-2 power law to 1e4,
isotropic) in the local orthonormal directions (r^, theta^, phi^) and turned
into covariant coordinate components with the flat-space scale factors
(u_r = u^r, u_theta = r u^theta, u_phi = r sin(theta) u^phi).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .particles import isotropic_dirs, maxwell_juttner_u, power_law_gamma

GR_COMPONENTS = ("D^r", "D^th", "D^ph", "B^r", "B^th", "B^ph")


def magnetosphere_fields(nr: int, nth: int, r_min: float, r_max: float, a: float,
                         B0: float, width: float, E_rec: float,
                         rotation: float = 1.0, inflow: float = 0.0) -> np.ndarray:
    """F[k, j, i] = component k at (r_i, theta_j), shape (6, nth+1, nr+1)."""
    r = r_min + (r_max - r_min) * np.arange(nr + 1) / nr
    th = np.pi * np.arange(nth + 1) / nth
    TH, R = np.meshgrid(th, r, indexing="ij")
    r_plus = 1.0 + np.sqrt(1.0 - a * a)
    omega_f = rotation * 0.5 * a / (2.0 * r_plus)
    ct = np.cos(TH)
    sheet = np.tanh(ct / width)
    Br = B0 * sheet / (R * R)
    F = np.zeros((6, nth + 1, nr + 1))
    F[0] = E_rec * B0 / (R * R) / np.cosh(ct / width) ** 2
    F[1] = -omega_f * np.sin(TH) * Br
    F[2] = inflow * B0 / (R * R * R)
    F[3] = Br
    F[5] = -omega_f * Br
    return F


@dataclass
class GREnsemble:
    r: np.ndarray
    th: np.ndarray
    ph: np.ndarray
    ur: np.ndarray
    uth: np.ndarray
    uph: np.ndarray
    qm: np.ndarray
    id: np.ndarray

    @property
    def n(self) -> int:
        return int(self.r.shape[0])

    def subset(self, idx) -> "GREnsemble":
        return GREnsemble(*[getattr(self, k)[idx] for k in
                            ("r", "th", "ph", "ur", "uth", "uph", "qm", "id")])


def magnetosphere_particles(n: int, seed: int, r_lo: float, r_hi: float, cos_max: float,
                            qm: float) -> GREnsemble:
    rng = np.random.default_rng(seed)
    r = rng.uniform(r_lo, r_hi, n)
    th = np.arccos(rng.uniform(-cos_max, cos_max, n))
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    half = n // 2
    g_mj = maxwell_juttner_u(rng, half, 1.0)
    gam = power_law_gamma(rng, n - half, 1.0e4)
    mag = np.concatenate([g_mj, np.sqrt(gam * gam - 1.0)])
    rng.shuffle(mag)
    d = isotropic_dirs(rng, n)
    uhat = d * mag
    ur = uhat[0]
    uth = r * uhat[1]
    uph = r * np.sin(th) * uhat[2]
    return GREnsemble(r, th, ph, ur, uth, uph, np.full(n, float(qm)),
                      np.arange(n, dtype=np.int32))


@dataclass(frozen=True)
class GRConfig:
    name: str
    nr: int
    nth: int
    n: int
    steps: int
    seed: int
    a: float = 0.9
    r_min: float = 1.5
    r_max: float = 50.0
    B0: float = 1.0
    width: float = 0.05
    E_rec: float = 0.02
    qm: float = -4000.0
    dt: float = 0.02
    f_rho: float = 1.0
    f_E: float = 1.0
    n_iter: int = 4
    r_lo: float = 2.5
    r_hi: float = 30.0
    cos_max: float = 0.9
    rotation: float = 1.0
    inflow: float = 0.0

    def fields(self) -> np.ndarray:
        return magnetosphere_fields(self.nr, self.nth, self.r_min, self.r_max, self.a,
                                    self.B0, self.width, self.E_rec, self.rotation,
                                    self.inflow)

    def particles(self, n: int | None = None, seed_offset: int = 0) -> GREnsemble:
        return magnetosphere_particles(self.n if n is None else n, self.seed + seed_offset,
                                       self.r_lo, self.r_hi, self.cos_max, self.qm)


# Named curved-spacetime workloads.  q/m = -4000 with B0 = 1 makes about 70 %
# of the initial particles of grbh512 take the guiding-center branch under
# the switch with f_rho = f_E = 1 (the thresholds of Sec. 4.2).
GR_CONFIGS = {
    # Kerr a = 0.9, r in [1.5, 50], 512 x 512 (r, theta) grid, 1e7 particles,
    # 200 steps of dt = 0.02 r_g/c
    "grbh512": GRConfig("grbh512", 512, 512, 10_000_000, 200, 20071),
    # small grid for fast tests
    "grbh64": GRConfig("grbh64", 64, 64, 4096, 40, 20072),
}


def make_gr_config(name: str, **overrides) -> GRConfig:
    from dataclasses import replace
    return replace(GR_CONFIGS[name], **overrides)
