"""Named workloads (code units: dx = dy = 1 cell, dt = 1, c = 0.45 cells/step).

Every config is fully determined by its seed.  Sizes:

  harris256   256^2 grid, 1e4 electrons, Maxwell-Juttner theta = 0.1, per-
              particle |q/m| log-uniform so that Omega_c0 dt = |q/m| B0 dt / c
              spans 1e-1 .. 1e3; 1000 steps; ideal fields (E.B = 0, E/B <= 0.1).
  harris4096  4096^2 grid with reconnection E_z at the two X points, 1e7
              electrons: half Maxwell-Juttner theta = 1, half a Gamma^-2 power
              law up to Gamma = 1e4; one scalar q/m chosen so that about 70 % of
              the initial particles take the guiding-center branch; 100 steps.
  harris1024  1024^2 grid, same field family and particle mix as harris4096,
              1e6 particles, 512 steps (differentiation workload).
  harris64    64^2 grid, small mixed ensemble for fast tests.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

from .harris import YEE_STAGGER, harris_fields
from .particles import (Ensemble, initial_state, maxwell_juttner_u,
                        power_law_gamma)

# Scalar q/m of the mixed (Maxwell-Juttner + power-law) electron ensembles.
# Chosen with the CPU oracle's switch on the harris4096 initial state so that
# 70 % of the particles start in the guiding-center regime
# (oracle/calibrate_qm.py prints the fraction for a given value).
MIX_QM = -1.89


@dataclass(frozen=True)
class Config:
    name: str
    nx: int
    ny: int
    n: int
    steps: int
    seed: int
    dx: float = 1.0
    dy: float = 1.0
    c: float = 0.45
    dt: float = 1.0
    B0: float = 1.0
    delta: float = 4.0
    guide: float = 0.1
    eps: float = 0.01
    vin: float = 0.1
    E_rec: float = 0.0
    recipe: str = "mj_logqm"      # or "mix"
    theta: float = 0.1
    qm: float = MIX_QM
    f_rho: float = 0.4
    f_E: float = 1.0
    curvature: int = 1
    n_iter: int = 4
    stagger: tuple = field(default_factory=lambda: tuple(map(tuple, YEE_STAGGER)))

    @property
    def Lx(self) -> float:
        return self.nx * self.dx

    @property
    def Ly(self) -> float:
        return self.ny * self.dy

    def fields(self, dtype=np.float64) -> np.ndarray:
        return harris_fields(self.nx, self.ny, self.dx, self.dy, B0=self.B0,
                             delta=self.delta, guide=self.guide, eps=self.eps,
                             vin=self.vin, c=self.c, E_rec=self.E_rec,
                             stagger=np.array(self.stagger), dtype=dtype)

    def particles(self, n: int | None = None, seed_offset: int = 0) -> Ensemble:
        n = self.n if n is None else n
        rng = np.random.default_rng(self.seed + seed_offset)
        if self.recipe == "mj_logqm":
            g = maxwell_juttner_u(rng, n, self.theta)
            omega_dt = 10.0 ** rng.uniform(-1.0, 3.0, n)
            qm = -omega_dt * self.c / (self.B0 * self.dt)
        elif self.recipe == "mix":
            h = n // 2
            g_mj = maxwell_juttner_u(rng, h, 1.0)
            gam = power_law_gamma(rng, n - h, 1.0e4)
            g_pl = np.sqrt(gam * gam - 1.0)
            g = np.concatenate([g_mj, g_pl])
            g = g[rng.permutation(n)]
            qm = self.qm
        else:
            raise ValueError(f"unknown recipe {self.recipe!r}")
        return initial_state(rng, g, Lx=self.Lx, Ly=self.Ly, c=self.c,
                             dt=self.dt, qm=qm)

    def with_(self, **kw) -> "Config":
        return replace(self, **kw)


CONFIGS = {
    "harris256": Config("harris256", 256, 256, 10_000, 1000, seed=14401),
    "harris4096": Config("harris4096", 4096, 4096, 10_000_000, 100,
                         seed=14402, E_rec=0.15, recipe="mix"),
    "harris1024": Config("harris1024", 1024, 1024, 1_000_000, 512,
                         seed=14404, E_rec=0.15, recipe="mix"),
    "harris64": Config("harris64", 64, 64, 4096, 50, seed=14400,
                       E_rec=0.15, recipe="mix"),
}


def make_config(name: str, **overrides) -> Config:
    return CONFIGS[name].with_(**overrides)
