"""Field providers for the oracle (test infrastructure, float64, torch CPU).

A provider is called with particle positions (X, Y) and returns a
`FieldSample`: E and B (three components each) and the in-plane gradient of
each B component, dB[j][i] = d B_i / d x_j for j in (x, y).  The problem is
2D3V, so d/dz is identically zero.  `e_gradient(X, Y)` gives the E
gradients in the same layout (only the exact guiding-center frame with
curvature needs them).

`GridFields` is the grid gather of the paper: a field value at a particle is
the sum over the surrounding nodes of node value times a linear shape
function W, and gradients come from differentiating W (Sec. 4, opening
paragraph).  In 2D with a linear W this is bilinear interpolation on the
2 x 2 nodes around the point, per component, on each component's own
(staggered) lattice, with periodic node indices.

The closed-form providers (uniform, linear, circular) are used by the pins:
bilinear interpolation reproduces fields linear in x and y exactly.
"""
from __future__ import annotations

from typing import NamedTuple

import numpy as np
import torch

from .ieee import sqrt

F64 = torch.float64

YEE = ((0.5, 0.0), (0.0, 0.5), (0.0, 0.0), (0.0, 0.5), (0.5, 0.0), (0.5, 0.5))
COLLOCATED = ((0.0, 0.0),) * 6


# Lattice coordinates (position / cell size) of magnitude FAR or more have no
# field: the gather returns NaN there.  Periodicity defines the field at any
# finite point, but no step of the method moves a particle that far from the
# box unless an iteration diverged (e.g. with the drift speed clamped where
# it reaches c), and node indices of such points do not fit a 32-bit integer.
FAR = float(2 ** 30)


def far_points(*lattice_coords):
    """True where any lattice coordinate is NaN or of magnitude >= FAR."""
    ok = None
    for g in lattice_coords:
        o = torch.abs(g) < FAR
        ok = o if ok is None else ok & o
    return ~ok


def nan_where(far, sample):
    """The sample with every value replaced by NaN where `far`."""
    if not bool(far.any()):
        return sample
    f = lambda v: torch.where(far, float("nan"), v)
    return type(sample)(*(tuple(f(v) for v in part) if not isinstance(part[0], tuple)
                          else tuple(tuple(f(v) for v in row) for row in part)
                          for part in sample))


class FieldSample(NamedTuple):
    E: tuple   # (Ex, Ey, Ez)
    B: tuple   # (Bx, By, Bz)
    dB: tuple  # ((dBx/dx, dBy/dx, dBz/dx), (dBx/dy, dBy/dy, dBz/dy))


class GridFields:
    """Bilinear gather from a periodic staggered grid.

    F[k, j, i] is component k (Ex, Ey, Ez, Bx, By, Bz) at
    ((i + s[k][0]) dx, (j + s[k][1]) dy).  For a point X the component's
    fractional node coordinate is xi = X/dx - s; with i = floor(xi),
    w = xi - i, the value is
        (1-wx)(1-wy) F[j,i] + wx(1-wy) F[j,i+1] + (1-wx)wy F[j+1,i] + wx wy F[j+1,i+1]
    and its x derivative is [(1-wy)(F[j,i+1]-F[j,i]) + wy(F[j+1,i+1]-F[j+1,i])]/dx
    (y symmetric).  Node indices are taken modulo nx, ny.
    """

    def __init__(self, F, dx: float = 1.0, dy: float = 1.0, stagger=YEE):
        F = torch.as_tensor(F, dtype=F64)
        assert F.ndim == 3 and F.shape[0] == 6
        self.F = F
        self.ny, self.nx = int(F.shape[1]), int(F.shape[2])
        self.dx, self.dy = float(dx), float(dy)
        self.inv_dx, self.inv_dy = 1.0 / self.dx, 1.0 / self.dy
        self.stagger = tuple((float(a), float(b)) for a, b in
                             np.asarray(stagger, dtype=np.float64))
        self.Lx, self.Ly = self.nx * self.dx, self.ny * self.dy

    def component(self, k: int, X, Y, grad: bool):
        sx, sy = self.stagger[k]
        xi = X * self.inv_dx - sx
        eta = Y * self.inv_dy - sy
        fi = torch.floor(xi)
        fj = torch.floor(eta)
        wx = xi - fi
        wy = eta - fj
        i = fi.to(torch.int64)
        j = fj.to(torch.int64)
        i0 = torch.remainder(i, self.nx)
        i1 = torch.remainder(i + 1, self.nx)
        j0 = torch.remainder(j, self.ny)
        j1 = torch.remainder(j + 1, self.ny)
        Fk = self.F[k]
        F00 = Fk[j0, i0]
        F10 = Fk[j0, i1]
        F01 = Fk[j1, i0]
        F11 = Fk[j1, i1]
        ax = 1.0 - wx
        ay = 1.0 - wy
        val = (((ax * ay) * F00 + (wx * ay) * F10) + (ax * wy) * F01) + (wx * wy) * F11
        if not grad:
            return val, None, None
        ddx = (ay * (F10 - F00) + wy * (F11 - F01)) * self.inv_dx
        ddy = (ax * (F01 - F00) + wx * (F11 - F10)) * self.inv_dy
        return val, ddx, ddy

    def __call__(self, X, Y) -> FieldSample:
        # a point 2^30 cells or more from the origin (or not a number): a
        # fixed-point iteration that ran away; its fields are NaN
        far = far_points(X * self.inv_dx, Y * self.inv_dy)
        X = torch.where(far, 0.0, X)
        Y = torch.where(far, 0.0, Y)
        E = tuple(self.component(k, X, Y, False)[0] for k in range(3))
        Bs = [self.component(k, X, Y, True) for k in range(3, 6)]
        B = tuple(b[0] for b in Bs)
        dB = (tuple(b[1] for b in Bs), tuple(b[2] for b in Bs))
        return nan_where(far, FieldSample(E, B, dB))

    def e_gradient(self, X, Y):
        """dE[j][i] = d E_i / d x_j (j = x, y) by differentiating W on each E
        component's own lattice, as for B; NaN where the sample is."""
        far = far_points(X * self.inv_dx, Y * self.inv_dy)
        X = torch.where(far, 0.0, X)
        Y = torch.where(far, 0.0, Y)
        Es = [self.component(k, X, Y, True) for k in range(3)]
        nan = lambda v: torch.where(far, float("nan"), v)
        return (tuple(nan(e[1]) for e in Es), tuple(nan(e[2]) for e in Es))


def _full(X, v):
    return torch.full_like(X, float(v))


class UniformFields:
    """Spatially constant E and B (zero gradients)."""

    def __init__(self, E, B):
        self.E = tuple(float(v) for v in E)
        self.B = tuple(float(v) for v in B)

    def __call__(self, X, Y) -> FieldSample:
        z = torch.zeros_like(X)
        return FieldSample(tuple(_full(X, v) for v in self.E),
                           tuple(_full(X, v) for v in self.B),
                           ((z, z, z), (z, z, z)))

    def e_gradient(self, X, Y):
        z = torch.zeros_like(X)
        return ((z, z, z), (z, z, z))


class LinearFields:
    """E(x) = E0 + GE @ (x, y), B(x) = B0 + GB @ (x, y) with 3x2 gradient matrices."""

    def __init__(self, E0, GE, B0, GB):
        self.E0 = np.asarray(E0, dtype=np.float64)
        self.GE = np.asarray(GE, dtype=np.float64).reshape(3, 2)
        self.B0 = np.asarray(B0, dtype=np.float64)
        self.GB = np.asarray(GB, dtype=np.float64).reshape(3, 2)

    def __call__(self, X, Y) -> FieldSample:
        E = tuple(self.E0[i] + self.GE[i, 0] * X + self.GE[i, 1] * Y for i in range(3))
        B = tuple(self.B0[i] + self.GB[i, 0] * X + self.GB[i, 1] * Y for i in range(3))
        dB = (tuple(_full(X, self.GB[i, 0]) for i in range(3)),
              tuple(_full(X, self.GB[i, 1]) for i in range(3)))
        return FieldSample(E, B, dB)

    def e_gradient(self, X, Y):
        return (tuple(_full(X, self.GE[i, 0]) for i in range(3)),
                tuple(_full(X, self.GE[i, 1]) for i in range(3)))

    def sample_grid(self, nx, ny, dx=1.0, dy=1.0, stagger=YEE):
        """The same fields sampled on each component's staggered nodes."""
        F = np.empty((6, ny, nx))
        G = np.concatenate([self.GE, self.GB])
        C = np.concatenate([self.E0, self.B0])
        for k in range(6):
            xs = (np.arange(nx) + stagger[k][0]) * dx
            ys = (np.arange(ny) + stagger[k][1]) * dy
            F[k] = C[k] + G[k, 0] * xs[None, :] + G[k, 1] * ys[:, None]
        return F


class CircularFields:
    """B = B0 e_phi around (xc, yc) plus a uniform Bz; E = 0.

    With Bz = 0 the field lines are circles of radius r and the curvature
    vector is (b.grad)b = -r_hat / r.  Gradients are analytic: with
    (dx, dy) = (X - xc, Y - yc) and r = |(dx, dy)|, Bx = -B0 dy/r and
    By = B0 dx/r.
    """

    def __init__(self, B0: float, xc: float, yc: float, Bz: float = 0.0):
        self.B0, self.xc, self.yc, self.Bz = float(B0), float(xc), float(yc), float(Bz)

    def __call__(self, X, Y) -> FieldSample:
        dx = X - self.xc
        dy = Y - self.yc
        r2 = dx * dx + dy * dy
        r = sqrt(r2)
        r3 = r2 * r
        Bx = -self.B0 * dy / r
        By = self.B0 * dx / r
        Bz = _full(X, self.Bz)
        z = torch.zeros_like(X)
        # d(dy/r)/dx = -dx dy / r^3 ; d(dy/r)/dy = dx^2 / r^3
        dBx_dx = self.B0 * dx * dy / r3
        dBx_dy = -self.B0 * dx * dx / r3
        dBy_dx = self.B0 * dy * dy / r3
        dBy_dy = -self.B0 * dx * dy / r3
        return FieldSample((z, z, z), (Bx, By, Bz),
                           ((dBx_dx, dBy_dx, z), (dBx_dy, dBy_dy, z)))

    def e_gradient(self, X, Y):
        z = torch.zeros_like(X)
        return ((z, z, z), (z, z, z))
