"""Named 3D workloads (code units: dx = dy = dz = 1 cell, dt = 1, c = 0.45
cells/step), fully determined by their seeds.

  harris3d128  128^3 grid, the 3D Harris family with reconnection E_z along
               the oblique X lines, 1e7 electrons (about 4.8 per cell): half
               Maxwell-Juttner theta = 1, half a Gamma^-2 power law up to
               Gamma = 1e4, the scalar q/m of the 2D mixed ensembles; 100 steps.
  harris3d32   32^3 grid, same family and mix, 4096 particles, 20 steps
               (parity cases the CPU oracle finishes in seconds).

The state of a particle is the leapfrog state of the 2D ensembles with a
third coordinate: x^n = (x, y, z), the previous position (xp, yp, zp) and
u^{n-1/2}.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

from .configs import MIX_QM
from .harris3d import YEE3_STAGGER, harris3d_fields
from .particles import isotropic_dirs, maxwell_juttner_u, power_law_gamma


@dataclass
class Ensemble3:
    """Structure-of-arrays 3D particle state (numpy, float64)."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    xp: np.ndarray
    yp: np.ndarray
    zp: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray
    qm: np.ndarray
    id: np.ndarray = field(default=None)

    KEYS = ("x", "y", "z", "xp", "yp", "zp", "ux", "uy", "uz", "qm", "id")

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def subset(self, idx) -> "Ensemble3":
        return Ensemble3(*(getattr(self, k)[idx] for k in self.KEYS))


def initial_state3(rng: np.random.Generator, umag_over_c: np.ndarray, *, Lx: float,
                   Ly: float, Lz: float, c: float, dt: float, qm) -> Ensemble3:
    """Uniform positions in the box, isotropic directions, given |u|/c; the
    previous position is the start of a straight move at the initial velocity."""
    n = umag_over_c.shape[0]
    x = rng.uniform(0.0, Lx, n)
    y = rng.uniform(0.0, Ly, n)
    z = rng.uniform(0.0, Lz, n)
    d = isotropic_dirs(rng, n)
    u = c * umag_over_c[None, :] * d
    gam = np.sqrt(1.0 + (u * u).sum(axis=0) / (c * c))
    xp = np.mod(x - dt * u[0] / gam, Lx)
    yp = np.mod(y - dt * u[1] / gam, Ly)
    zp = np.mod(z - dt * u[2] / gam, Lz)
    qm = np.broadcast_to(np.asarray(qm, dtype=np.float64), (n,)).copy()
    return Ensemble3(x=x, y=y, z=z, xp=xp, yp=yp, zp=zp, ux=u[0].copy(), uy=u[1].copy(),
                     uz=u[2].copy(), qm=qm, id=np.arange(n, dtype=np.int32))


@dataclass(frozen=True)
class Config3:
    name: str
    nx: int
    ny: int
    nz: int
    n: int
    steps: int
    seed: int
    dx: float = 1.0
    dy: float = 1.0
    dz: float = 1.0
    c: float = 0.45
    dt: float = 1.0
    B0: float = 1.0
    delta: float = 4.0
    guide: float = 0.1
    eps: float = 0.01
    vin: float = 0.1
    E_rec: float = 0.15
    qm: float = MIX_QM
    f_rho: float = 0.4
    f_E: float = 1.0
    curvature: int = 1
    n_iter: int = 4
    stagger: tuple = field(default_factory=lambda: tuple(map(tuple, YEE3_STAGGER)))

    @property
    def Lx(self) -> float:
        return self.nx * self.dx

    @property
    def Ly(self) -> float:
        return self.ny * self.dy

    @property
    def Lz(self) -> float:
        return self.nz * self.dz

    @property
    def dl(self) -> float:
        """Effective cell size (dx dy dz)^(1/3) of the switch (Sec. 3), by the C
        library's cube root."""
        return float(np.cbrt((self.dx * self.dy) * self.dz))

    def fields(self, dtype=np.float64) -> np.ndarray:
        return harris3d_fields(self.nx, self.ny, self.nz, self.dx, self.dy, self.dz,
                               B0=self.B0, delta=self.delta, guide=self.guide, eps=self.eps,
                               vin=self.vin, c=self.c, E_rec=self.E_rec,
                               stagger=np.array(self.stagger), dtype=dtype)

    def particles(self, n: int | None = None, seed_offset: int = 0) -> Ensemble3:
        """Half Maxwell-Juttner theta = 1, half a Gamma^-2 power law up to 1e4."""
        n = self.n if n is None else n
        rng = np.random.default_rng(self.seed + seed_offset)
        h = n // 2
        g_mj = maxwell_juttner_u(rng, h, 1.0)
        gam = power_law_gamma(rng, n - h, 1.0e4)
        g = np.concatenate([g_mj, np.sqrt(gam * gam - 1.0)])
        g = g[rng.permutation(n)]
        return initial_state3(rng, g, Lx=self.Lx, Ly=self.Ly, Lz=self.Lz, c=self.c,
                              dt=self.dt, qm=self.qm)

    def with_(self, **kw) -> "Config3":
        return replace(self, **kw)


CONFIGS3 = {
    "harris3d128": Config3("harris3d128", 128, 128, 128, 10_000_000, 100, seed=14410),
    "harris3d32": Config3("harris3d32", 32, 32, 32, 4096, 20, seed=14411),
}


def make_config3(name: str, **overrides) -> Config3:
    return CONFIGS3[name].with_(**overrides)
