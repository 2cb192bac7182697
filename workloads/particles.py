"""Seeded particle ensembles.

The state of a particle is the staggered leapfrog state of Sec. 2.1: position
x^n at an integer time level, the previous position x^{n-1}, and the spatial
part of the four-velocity u^{n-1/2} (velocity units, u = Gamma v) at the half
level.  Positions are 2D (x, y); u has three components.

Momentum distributions:
  * Maxwell-Juettner with temperature theta (in m c^2): the density of
    g = |u|/c is proportional to g^2 exp(-(sqrt(1+g^2) - 1)/theta); drawn by
    inverting a tabulated cumulative distribution on a fine grid;
  * a power law dN/dGamma ~ Gamma^-2 on [1, gmax], drawn by inverting its
    cumulative distribution, Gamma = 1/(1 - xi (1 - 1/gmax)).
Directions are isotropic.  The previous position is the start of a straight
move at the initial velocity, x^{-1} = x^0 - dt u/sqrt(1 + u^2/c^2), wrapped
into the box.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def isotropic_dirs(rng: np.random.Generator, n: int) -> np.ndarray:
    """Unit vectors uniformly distributed on the sphere, shape (3, n)."""
    cos_t = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    return np.stack([sin_t * np.cos(phi), sin_t * np.sin(phi), cos_t])


def maxwell_juttner_u(rng: np.random.Generator, n: int, theta: float,
                      table: int = 200001) -> np.ndarray:
    """|u|/c magnitudes drawn from a Maxwell-Juttner distribution."""
    gmax = 1.0 + 60.0 * theta
    umax = np.sqrt(gmax * gmax - 1.0)
    g = np.linspace(0.0, umax, table)
    pdf = g * g * np.exp(-(np.sqrt(1.0 + g * g) - 1.0) / theta)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]))])
    cdf /= cdf[-1]
    return np.interp(rng.uniform(0.0, 1.0, n), cdf, g)


def power_law_gamma(rng: np.random.Generator, n: int, gmax: float) -> np.ndarray:
    """Lorentz factors with dN/dGamma ~ Gamma^-2 on [1, gmax]."""
    xi = rng.uniform(0.0, 1.0, n)
    return 1.0 / (1.0 - xi * (1.0 - 1.0 / gmax))


@dataclass
class Ensemble:
    """Structure-of-arrays particle state (numpy, float64)."""
    x: np.ndarray
    y: np.ndarray
    xp: np.ndarray
    yp: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray
    qm: np.ndarray           # per-particle charge-to-mass ratio (signed)
    id: np.ndarray = field(default=None)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def subset(self, idx) -> "Ensemble":
        return Ensemble(*(getattr(self, k)[idx] for k in
                          ("x", "y", "xp", "yp", "ux", "uy", "uz", "qm", "id")))

    def arrays(self):
        return dict(x=self.x, y=self.y, xp=self.xp, yp=self.yp, ux=self.ux,
                    uy=self.uy, uz=self.uz, qm=self.qm, id=self.id)


def initial_state(rng: np.random.Generator, umag_over_c: np.ndarray, *,
                  Lx: float, Ly: float, c: float, dt: float,
                  qm) -> Ensemble:
    """Uniform positions in the box, isotropic directions, given |u|/c."""
    n = umag_over_c.shape[0]
    x = rng.uniform(0.0, Lx, n)
    y = rng.uniform(0.0, Ly, n)
    d = isotropic_dirs(rng, n)
    u = c * umag_over_c[None, :] * d
    gam = np.sqrt(1.0 + (u * u).sum(axis=0) / (c * c))
    xp = np.mod(x - dt * u[0] / gam, Lx)
    yp = np.mod(y - dt * u[1] / gam, Ly)
    qm = np.broadcast_to(np.asarray(qm, dtype=np.float64), (n,)).copy()
    return Ensemble(x=x, y=y, xp=xp, yp=yp, ux=u[0].copy(), uy=u[1].copy(),
                    uz=u[2].copy(), qm=qm, id=np.arange(n, dtype=np.int32))
