"""3D field providers for the oracle (test infrastructure, float64, torch CPU).

A 3D provider is called with particle positions (X, Y, Z) and returns a
`FieldSample3`: E and B (three components each) and the gradient of each B
component, dB[j][i] = d B_i / d x_j for j in (x, y, z).

`GridFields3` is the grid gather of the paper in three dimensions: the value
at a particle is the sum over the surrounding nodes of node value times the
linear shape function W(x - x_N) = W(dx) W(dy) W(dz), and the gradient
differentiates W (Sec. 4, opening paragraph).  On each component's own
(staggered) lattice that is trilinear interpolation on the 2 x 2 x 2 nodes
around the point, with periodic node indices.  The sum is grouped by z plane:
the bilinear sum of each of the two planes (the 2D provider's expression),
then the two planes weighted by W along z.

The closed-form providers serve the pins: trilinear interpolation reproduces
fields linear in x, y and z exactly.
"""
from __future__ import annotations

from typing import NamedTuple

import numpy as np
import torch

from .fields import far_points, nan_where
from .ieee import sqrt

F64 = torch.float64

YEE3 = ((0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5),
        (0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0))
COLLOCATED3 = ((0.0, 0.0, 0.0),) * 6


class FieldSample3(NamedTuple):
    E: tuple   # (Ex, Ey, Ez)
    B: tuple   # (Bx, By, Bz)
    dB: tuple  # (d/dx, d/dy, d/dz), each (dBx, dBy, dBz)


class GridFields3:
    """Trilinear gather from a periodic staggered 3D grid.

    F[k, l, j, i] is component k at ((i + s[k][0]) dx, (j + s[k][1]) dy,
    (l + s[k][2]) dz).  For a point X the component's fractional node
    coordinates are (xi, eta, zeta) = (X/dx, Y/dy, Z/dz) - s; with
    (i, j, l) their floors and (wx, wy, wz) the remainders, a = 1 - w,
        v_l  = ax ay F[l,j,i] + wx ay F[l,j,i+1] + ax wy F[l,j+1,i] + wx wy F[l,j+1,i+1]
        value = az v_l + wz v_{l+1}
        d/dx  = (az g_l + wz g_{l+1})/dx,  g_l = ay (F[l,j,i+1]-F[l,j,i]) + wy (F[l,j+1,i+1]-F[l,j+1,i])
        d/dy  = (az h_l + wz h_{l+1})/dy,  h_l = ax (F[l,j+1,i]-F[l,j,i]) + wx (F[l,j+1,i+1]-F[l,j,i+1])
        d/dz  = (v_{l+1} - v_l)/dz.
    Node indices are taken modulo nx, ny, nz.
    """

    def __init__(self, F, dx: float = 1.0, dy: float = 1.0, dz: float = 1.0,
                 stagger=YEE3):
        F = torch.as_tensor(F, dtype=F64)
        assert F.ndim == 4 and F.shape[0] == 6
        self.F = F
        self.nz, self.ny, self.nx = int(F.shape[1]), int(F.shape[2]), int(F.shape[3])
        self.dx, self.dy, self.dz = float(dx), float(dy), float(dz)
        self.inv_dx, self.inv_dy, self.inv_dz = 1.0 / self.dx, 1.0 / self.dy, 1.0 / self.dz
        self.stagger = tuple(tuple(float(v) for v in s) for s in
                             np.asarray(stagger, dtype=np.float64))
        self.Lx, self.Ly, self.Lz = self.nx * self.dx, self.ny * self.dy, self.nz * self.dz

    def component(self, k: int, X, Y, Z, grad: bool):
        sx, sy, sz = self.stagger[k]
        xi = X * self.inv_dx - sx
        eta = Y * self.inv_dy - sy
        zeta = Z * self.inv_dz - sz
        fi, fj, fl = torch.floor(xi), torch.floor(eta), torch.floor(zeta)
        wx, wy, wz = xi - fi, eta - fj, zeta - fl
        i, j, l = fi.to(torch.int64), fj.to(torch.int64), fl.to(torch.int64)
        i0, i1 = torch.remainder(i, self.nx), torch.remainder(i + 1, self.nx)
        j0, j1 = torch.remainder(j, self.ny), torch.remainder(j + 1, self.ny)
        l0, l1 = torch.remainder(l, self.nz), torch.remainder(l + 1, self.nz)
        Fk = self.F[k]
        ax, ay, az = 1.0 - wx, 1.0 - wy, 1.0 - wz

        def plane(lz):
            f00, f10 = Fk[lz, j0, i0], Fk[lz, j0, i1]
            f01, f11 = Fk[lz, j1, i0], Fk[lz, j1, i1]
            v = (((ax * ay) * f00 + (wx * ay) * f10) + (ax * wy) * f01) + (wx * wy) * f11
            g = ay * (f10 - f00) + wy * (f11 - f01)
            h = ax * (f01 - f00) + wx * (f11 - f10)
            return v, g, h

        v0, g0, h0 = plane(l0)
        v1, g1, h1 = plane(l1)
        val = az * v0 + wz * v1
        if not grad:
            return val, None, None, None
        ddx = (az * g0 + wz * g1) * self.inv_dx
        ddy = (az * h0 + wz * h1) * self.inv_dy
        ddz = (v1 - v0) * self.inv_dz
        return val, ddx, ddy, ddz

    def __call__(self, X, Y, Z) -> FieldSample3:
        # a point 2^30 cells or more from the origin (or not a number) has NaN
        # fields, as in 2D
        far = far_points(X * self.inv_dx, Y * self.inv_dy, Z * self.inv_dz)
        X = torch.where(far, 0.0, X)
        Y = torch.where(far, 0.0, Y)
        Z = torch.where(far, 0.0, Z)
        E = tuple(self.component(k, X, Y, Z, False)[0] for k in range(3))
        Bs = [self.component(k, X, Y, Z, True) for k in range(3, 6)]
        B = tuple(b[0] for b in Bs)
        dB = tuple(tuple(b[j + 1] for b in Bs) for j in range(3))
        return nan_where(far, FieldSample3(E, B, dB))

    def e_gradient(self, X, Y, Z):
        """dE[j][i] = d E_i / d x_j (j = x, y, z), differentiating W on each E
        component's own lattice; NaN where the sample is."""
        far = far_points(X * self.inv_dx, Y * self.inv_dy, Z * self.inv_dz)
        X = torch.where(far, 0.0, X)
        Y = torch.where(far, 0.0, Y)
        Z = torch.where(far, 0.0, Z)
        Es = [self.component(k, X, Y, Z, True) for k in range(3)]
        nan = lambda v: torch.where(far, float("nan"), v)
        return tuple(tuple(nan(e[j + 1]) for e in Es) for j in range(3))


def _full(X, v):
    return torch.full_like(X, float(v))


class UniformFields3:
    """Spatially constant E and B (zero gradients)."""

    def __init__(self, E, B):
        self.E = tuple(float(v) for v in E)
        self.B = tuple(float(v) for v in B)

    def __call__(self, X, Y, Z) -> FieldSample3:
        z = torch.zeros_like(X)
        return FieldSample3(tuple(_full(X, v) for v in self.E),
                            tuple(_full(X, v) for v in self.B),
                            ((z, z, z), (z, z, z), (z, z, z)))

    def e_gradient(self, X, Y, Z):
        z = torch.zeros_like(X)
        return ((z, z, z), (z, z, z), (z, z, z))


class LinearFields3:
    """E(x) = E0 + GE @ (x, y, z), B(x) = B0 + GB @ (x, y, z) with 3x3 gradients."""

    def __init__(self, E0, GE, B0, GB):
        self.E0 = np.asarray(E0, dtype=np.float64)
        self.GE = np.asarray(GE, dtype=np.float64).reshape(3, 3)
        self.B0 = np.asarray(B0, dtype=np.float64)
        self.GB = np.asarray(GB, dtype=np.float64).reshape(3, 3)

    def __call__(self, X, Y, Z) -> FieldSample3:
        E = tuple(self.E0[i] + self.GE[i, 0] * X + self.GE[i, 1] * Y + self.GE[i, 2] * Z
                  for i in range(3))
        B = tuple(self.B0[i] + self.GB[i, 0] * X + self.GB[i, 1] * Y + self.GB[i, 2] * Z
                  for i in range(3))
        dB = tuple(tuple(_full(X, self.GB[i, j]) for i in range(3)) for j in range(3))
        return FieldSample3(E, B, dB)

    def e_gradient(self, X, Y, Z):
        return tuple(tuple(_full(X, self.GE[i, j]) for i in range(3)) for j in range(3))

    def sample_grid(self, nx, ny, nz, dx=1.0, dy=1.0, dz=1.0, stagger=YEE3):
        """The same fields sampled on each component's staggered nodes, (6, nz, ny, nx)."""
        F = np.empty((6, nz, ny, nx))
        G = np.concatenate([self.GE, self.GB])
        C = np.concatenate([self.E0, self.B0])
        for k in range(6):
            xs = (np.arange(nx) + stagger[k][0]) * dx
            ys = (np.arange(ny) + stagger[k][1]) * dy
            zs = (np.arange(nz) + stagger[k][2]) * dz
            F[k] = (C[k] + G[k, 0] * xs[None, None, :] + G[k, 1] * ys[None, :, None]
                    + G[k, 2] * zs[:, None, None])
        return F


class CircularFieldsXZ:
    """B = B0 e_phi around the line x = xc, z = zc (parallel to y), plus a
    uniform By; E = 0.  Field lines are circles in planes of constant y, so the
    curvature (b.grad)b = -r_hat/r (By = 0) lies in the (x, z) plane and is
    built from x and z derivatives.  With (ex, ez) = (X - xc, Z - zc) and
    r = |(ex, ez)|: Bx = B0 ez/r, Bz = -B0 ex/r (counter-clockwise seen from +y).
    """

    def __init__(self, B0: float, xc: float, zc: float, By: float = 0.0):
        self.B0, self.xc, self.zc, self.By = float(B0), float(xc), float(zc), float(By)

    def __call__(self, X, Y, Z) -> FieldSample3:
        ex = X - self.xc
        ez = Z - self.zc
        r2 = ex * ex + ez * ez
        r = sqrt(r2)
        r3 = r2 * r
        Bx = self.B0 * ez / r
        Bz = -self.B0 * ex / r
        By = _full(X, self.By)
        z = torch.zeros_like(X)
        # d(ez/r)/dx = -ex ez/r^3, d(ez/r)/dz = ex^2/r^3
        # d(ex/r)/dx = ez^2/r^3,   d(ex/r)/dz = -ex ez/r^3
        dBx_dx = -self.B0 * ex * ez / r3
        dBx_dz = self.B0 * ex * ex / r3
        dBz_dx = -self.B0 * ez * ez / r3
        dBz_dz = self.B0 * ex * ez / r3
        return FieldSample3((z, z, z), (Bx, By, Bz),
                            ((dBx_dx, z, dBz_dx), (z, z, z), (dBx_dz, z, dBz_dz)))

    def e_gradient(self, X, Y, Z):
        z = torch.zeros_like(X)
        return ((z, z, z), (z, z, z), (z, z, z))
