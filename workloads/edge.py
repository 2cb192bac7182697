"""A small crafted field and particle set on which every status outcome of the
coupled step occurs (test input; no arithmetic of the method).

Grid: 48 x 48 periodic cells, dx = dy = 1, 2D Yee lattice, c = 0.5.  Node
values (component k at node (i, j) of its own lattice) by vertical band:

  band A, i in [0, 16): smooth field lines that curve on the scale of the
      band, with an electric field (E.B != 0, E < B);
  band B, i in [16, 32): a uniform Bz = 1, E = 0 background, with
      * a block i in [20, 30), j in [2, 12) where all six components vanish
        (B = 0 at every point whose stencils lie inside it),
      * a block i in [20, 30), j in [14, 22) with Bz = 0.4, Ey = 0.8
        (E = 2 B: the drift speed c E/B exceeds c),
      * for j in [24, 48), Ey alternating 0.5 + 2^-14 and 0.5 - 2^-14 with
        the parity of i (E/B crosses 0.5 exactly halfway between nodes);
  band C, i in [32, 48): node values drawn uniformly at random (|B_k| <= 1,
      |E_k| <= 0.7): gradients on the cell scale, E > B at some points.

All node values of bands B are exact in binary32, and the particles of the
threshold groups sit at positions whose interpolation weights are multiples
of 1/64, so their field samples are exact in binary32 and binary64 alike.

Particle groups (`EdgeSet.groups` names the slots of each):
  general     random positions, Maxwell-Juttner |u| (theta 0.3), per-particle
              |q/m| log-uniform with Omega_c dt in [0.1, 1e3], x_prev from a
              straight move at the initial velocity
  bzero       x^n just right of the zero block (B = 1 there, guiding center),
              x^{n-1} ten cells to the left: the midpoint R^{n-1/2} of the
              conversion lies where B = 0
  kappa       the same next to the E = 2B block: the drift speed at
              R^{n-1/2} exceeds c
  far_prev    guiding center in band A with x^{n-1} half a box away:
              R^{n-1/2} outside the LDS window of the tiled kernel
  nonfinite   a NaN or infinite component of u
  rho_edge    u = 0, B = 1, E = 0, q/m = -0.5 (1 + j 2^-52), j in [-8, 8]:
              rho~/dl = c^2/(|q/m| B) lies at, and a few ulp either side of,
              f_rho = 0.5
  e_edge      |q/m| = 5 (rho~/dl << f_rho), E/B = 0.5 + 2^-13 (1 - 2w) with
              w = k/64: at (k = 32) and either side of f_E = 0.5
  in_zero     x^n inside the zero block (the switch sees B = 0)
  in_e_gt_b   x^n inside the E = 2B block (the switch sees E > B)
  rough       band C, |q/m| log-uniform with Omega_c dt in [1, 1e3], moderate
              |u|: curvature and drift terms on the cell scale
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .particles import Ensemble, initial_state, maxwell_juttner_u

NX = NY = 48
C_LIGHT = 0.5
F_RHO = 0.5
F_E = 0.5
SEED = 14480


def edge_fields(seed: int = SEED) -> np.ndarray:
    """Node arrays, shape (6, NY, NX), order Ex, Ey, Ez, Bx, By, Bz."""
    rng = np.random.default_rng(seed)
    F = np.zeros((6, NY, NX))
    i = np.arange(NX)[None, :]
    j = np.arange(NY)[:, None]
    # band A
    a = (slice(None), slice(0, 16))
    F[3][a] = (0.6 * np.sin(2 * np.pi * j / 16.0) + 0.0 * i)[a]
    F[4][a] = (0.6 * np.cos(2 * np.pi * i / 16.0) + 0.0 * j)[a]
    F[5][a] = 1.0
    F[0][a] = (0.2 * np.cos(2 * np.pi * j / 16.0) + 0.0 * i)[a]
    F[1][a] = (0.3 * np.sin(2 * np.pi * i / 16.0) + 0.0 * j)[a]
    F[2][a] = 0.15
    # band B
    F[5][:, 16:32] = 1.0
    F[:, 2:12, 20:30] = 0.0
    F[5][14:22, 20:30] = 0.4
    F[1][14:22, 20:30] = 0.8
    d = 2.0 ** -14
    par = np.where(np.arange(16, 32) % 2 == 0, d, -d)
    F[1][24:48, 16:32] = 0.5 + par[None, :]
    # band C
    F[3:, :, 32:48] = rng.uniform(-1.0, 1.0, (3, NY, 16))
    F[:3, :, 32:48] = rng.uniform(-0.7, 0.7, (3, NY, 16))
    return F


@dataclass
class EdgeSet:
    ens: Ensemble
    groups: dict   # group name -> slice of particle slots


def _ens(x, y, xp, yp, u, qm):
    n = x.shape[0]
    return Ensemble(x=np.asarray(x, float), y=np.asarray(y, float),
                    xp=np.asarray(xp, float), yp=np.asarray(yp, float),
                    ux=np.asarray(u[0], float).copy(), uy=np.asarray(u[1], float).copy(),
                    uz=np.asarray(u[2], float).copy(),
                    qm=np.broadcast_to(np.asarray(qm, float), (n,)).copy(),
                    id=np.arange(n, dtype=np.int32))


def edge_particles(dt: float = 1.0, seed: int = SEED, n_general: int = 2000,
                   n_rough: int = 1500) -> EdgeSet:
    rng = np.random.default_rng(seed + 1)
    c, L = C_LIGHT, float(NX)
    parts, groups = [], {}

    def add(name, e):
        start = sum(p.n for p in parts)
        parts.append(e)
        groups[name] = slice(start, start + e.n)

    g = maxwell_juttner_u(rng, n_general, 0.3)
    qm = -(10.0 ** rng.uniform(-1.0, 3.0, n_general)) * c / dt
    add("general", initial_state(rng, g, Lx=L, Ly=L, c=c, dt=dt, qm=qm))

    def beside(n, y0, y1):
        x = rng.uniform(30.6, 31.4, n)
        y = rng.uniform(y0, y1, n)
        u = 0.1 * c * rng.standard_normal((3, n))
        return x, y, np.mod(x - 10.0, L), y.copy(), u

    x, y, xp, yp, u = beside(64, 4.0, 10.0)
    add("bzero", _ens(x, y, xp, yp, u, -5.0))
    x, y, xp, yp, u = beside(64, 16.0, 20.0)
    add("kappa", _ens(x, y, xp, yp, u, -5.0))

    # x^{n-1} half a box away: R^{n-1/2} lies 11.75 cells from x^n, outside
    # the LDS window of any tile of up to 16 cells that holds x^n (x^n sits
    # in the first 6 cells of its tile)
    n = 64
    x = rng.uniform(1.0, 5.9, n)
    y = rng.uniform(0.0, L, n)
    u = 0.1 * c * rng.standard_normal((3, n))
    add("far_prev", _ens(x, y, np.mod(x + 24.5, L), y.copy(), u, -5.0))

    nan, inf = float("nan"), float("inf")
    u = np.array([[nan, inf, 0.0, 0.0, -inf, 0.1],
                  [0.0, 0.0, -inf, 0.0, 0.0, nan],
                  [0.0, 0.0, 0.0, nan, 0.0, 0.0]])
    x = np.array([5.5, 6.25, 24.0, 40.5, 17.75, 10.0])
    y = np.array([5.5, 30.0, 30.5, 20.0, 8.0, 40.0])
    add("nonfinite", _ens(x, y, x, y, u, -3.0))

    js = np.arange(-8, 9)
    k = np.arange(js.size)
    x = 17.5 + (k % 4) / 64.0 * 8.0
    y = 2.0 + (7 * k % 64) / 64.0
    qm = -0.5 * (1.0 + js * 2.0 ** -52)
    add("rho_edge", _ens(x, y, x, y, np.zeros((3, js.size)), qm))

    k = np.arange(24, 41)
    x = 20.0 + k / 64.0
    y = 30.0 + (k % 8) / 64.0 * 32.0
    add("e_edge", _ens(x, y, x, y, np.zeros((3, k.size)), -5.0))

    n = 32
    x = rng.uniform(22.0, 28.0, n)
    y = rng.uniform(4.0, 10.0, n)
    u = 0.2 * c * rng.standard_normal((3, n))
    add("in_zero", _ens(x, y, np.mod(x - 0.1, L), y, u, -5.0))
    x = rng.uniform(22.0, 28.0, n)
    y = rng.uniform(16.0, 20.0, n)
    add("in_e_gt_b", _ens(x, y, np.mod(x - 0.1, L), y, u, -5.0))

    g = maxwell_juttner_u(rng, n_rough, 0.05)
    qm = -(10.0 ** rng.uniform(0.0, 3.0, n_rough)) * c / dt
    e = initial_state(rng, g, Lx=L, Ly=L, c=c, dt=dt, qm=qm)
    e.x = rng.uniform(33.0, 47.0, n_rough)
    e.y = rng.uniform(0.0, L, n_rough)
    gam = np.sqrt(1.0 + (e.ux ** 2 + e.uy ** 2 + e.uz ** 2) / (c * c))
    e.xp = np.mod(e.x - dt * e.ux / gam, L)
    e.yp = np.mod(e.y - dt * e.uy / gam, L)
    add("rough", e)

    cat = {k2: np.concatenate([getattr(p, k2) for p in parts])
           for k2 in ("x", "y", "xp", "yp", "ux", "uy", "uz", "qm")}
    n = cat["x"].shape[0]
    ens = Ensemble(**cat, id=np.arange(n, dtype=np.int32))
    return EdgeSet(ens, groups)


NZ = 8


def edge_fields3(seed: int = SEED, nz: int = NZ) -> np.ndarray:
    """The 2D edge field extruded along z: shape (6, nz, NY, NX).  The 3D Yee
    lattice places each component at the same (x, y) offsets as the 2D one,
    so every (x, y) feature is where it is in 2D, at every z."""
    F = edge_fields(seed)
    return np.ascontiguousarray(np.broadcast_to(F[:, None], (6, nz, NY, NX)))


def edge_particles3(dt: float = 1.0, seed: int = SEED, nz: int = NZ):
    """The 2D edge set with z positions on the 1/64 lattice (so the z weights
    keep the threshold groups' samples exact); x_{n-1} at the same z for the
    constructed groups, from a straight move for the random ones."""
    from .configs3d import Ensemble3
    es = edge_particles(dt=dt, seed=seed)
    e = es.ens
    rng = np.random.default_rng(seed + 2)
    z = rng.integers(0, nz * 64, e.n) / 64.0
    zp = z.copy()
    for name in ("general", "rough"):
        sl = es.groups[name]
        gam = np.sqrt(1.0 + (e.ux[sl] ** 2 + e.uy[sl] ** 2 + e.uz[sl] ** 2) / C_LIGHT ** 2)
        zp[sl] = np.mod(z[sl] - dt * e.uz[sl] / gam, float(nz))
    ens3 = Ensemble3(x=e.x, y=e.y, z=z, xp=e.xp, yp=e.yp, zp=zp, ux=e.ux, uy=e.uy, uz=e.uz,
                     qm=e.qm, id=e.id)
    return EdgeSet(ens3, es.groups)
