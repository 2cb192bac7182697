"""Harris-family static field snapshots on a periodic 3D staggered grid.

Component order everywhere is (Ex, Ey, Ez, Bx, By, Bz).  Each component lives
on its own lattice, offset from the cell corner (i dx, j dy, l dz) by a
fraction of a cell given by a stagger table; the default is the 3D Yee
arrangement of explicit PiC codes (E on cell edges, B on cell faces).  Its
(x, y) offsets are those of the 2D Yee lattice, so a field that does not
depend on z samples to the same values as on the 2D grid.

Field family (closed form, sampled at each component's own nodes):
  * the periodic double Harris sheet of the 2D family,
      Bx0(y) = B0 [tanh((y - Ly/4)/d) - tanh((y - 3Ly/4)/d) - 1];
  * a uniform guide field Bz = guide * B0;
  * an oblique tearing perturbation from the vector potential psi z_hat,
      psi = eps B0 cos(kx x + kz z) sin(ky y) / ky,
    dBx = d psi/dy = eps B0 cos(kx x + kz z) cos(ky y),
    dBy = -d psi/dx = eps B0 (kx/ky) sin(kx x + kz z) sin(ky y)
    (divergence free; with kz = 0 and Lx = Ly it is the 2D perturbation), so
    the X lines run obliquely through the box along kx x + kz z = 0;
  * the ideal inflow field E = -v_in x B / c with
      v_in = (0, -vin*c*sin(4pi (y - Ly/4)/Ly), 0);
  * optionally a reconnection field Ez += E_rec B0 exp(-d^2/(2 d_sheet^2)),
    d the distance in the (x, y) plane to the X line of each sheet.
"""
from __future__ import annotations

import numpy as np

# (x, y, z) offsets of each component's nodes, in cells
YEE3_STAGGER = np.array([
    [0.5, 0.0, 0.0],   # Ex on x-edges
    [0.0, 0.5, 0.0],   # Ey on y-edges
    [0.0, 0.0, 0.5],   # Ez on z-edges
    [0.0, 0.5, 0.5],   # Bx on x-faces
    [0.5, 0.0, 0.5],   # By on y-faces
    [0.5, 0.5, 0.0],   # Bz on z-faces
], dtype=np.float64)


def _component(k, X, Y, Z, Lx, Ly, Lz, B0, delta, guide, eps, vin, c, E_rec):
    """Analytic component k (0..5 = Ex, Ey, Ez, Bx, By, Bz) at points (X, Y, Z)."""
    kx = 2.0 * np.pi / Lx
    ky = 2.0 * np.pi / Ly
    kz = 2.0 * np.pi / Lz
    shape = np.broadcast(X, Y, Z).shape

    def bx():
        v = B0 * (np.tanh((Y - 0.25 * Ly) / delta)
                  - np.tanh((Y - 0.75 * Ly) / delta) - 1.0)
        return v + eps * B0 * np.cos(kx * X + kz * Z) * np.cos(ky * Y)

    def vy():
        return -vin * c * np.sin(4.0 * np.pi * (Y - 0.25 * Ly) / Ly)

    if k == 3:
        return np.broadcast_to(bx(), shape)
    if k == 4:
        return np.broadcast_to(eps * B0 * (kx / ky) * np.sin(kx * X + kz * Z)
                               * np.sin(ky * Y), shape)
    if k == 5:
        return np.full(shape, guide * B0)
    if k == 0:
        return np.broadcast_to(-vy() * (guide * B0) / c, shape)
    if k == 1:
        return np.zeros(shape)
    ez = np.broadcast_to(vy() * bx() / c, shape)
    if E_rec != 0.0:
        # X line of each sheet: kx x + kz z = 0 (mod 2 pi), i.e. x = -z Lx/Lz
        for y0 in (0.25 * Ly, 0.75 * Ly):
            ddx = X + Z * (Lx / Lz)
            ddx = ddx - Lx * np.round(ddx / Lx)
            ddy = Y - y0
            ddy = ddy - Ly * np.round(ddy / Ly)
            ez = ez + E_rec * B0 * np.exp(-(ddx * ddx + ddy * ddy)
                                         / (2.0 * delta * delta))
    return ez


def harris3d_fields(nx: int, ny: int, nz: int, dx: float = 1.0, dy: float = 1.0,
                    dz: float = 1.0, *, B0: float = 1.0, delta: float = 4.0,
                    guide: float = 0.1, eps: float = 0.01, vin: float = 0.1,
                    c: float = 0.45, E_rec: float = 0.0, stagger=YEE3_STAGGER,
                    dtype=np.float64) -> np.ndarray:
    """Sample the field family on an nx x ny x nz periodic grid.

    Returns F of shape (6, nz, ny, nx): F[k, l, j, i] is component k at
    ((i + s[k,0]) dx, (j + s[k,1]) dy, (l + s[k,2]) dz).
    """
    stagger = np.asarray(stagger, dtype=np.float64)
    Lx, Ly, Lz = nx * dx, ny * dy, nz * dz
    out = np.empty((6, nz, ny, nx), dtype=dtype)
    ii = np.arange(nx, dtype=np.float64)
    jj = np.arange(ny, dtype=np.float64)
    ll = np.arange(nz, dtype=np.float64)
    for k in range(6):
        X = ((ii + stagger[k, 0]) * dx)[None, None, :]
        Y = ((jj + stagger[k, 1]) * dy)[None, :, None]
        Z = ((ll + stagger[k, 2]) * dz)[:, None, None]
        out[k] = _component(k, X, Y, Z, Lx, Ly, Lz, B0, delta, guide, eps, vin, c, E_rec)
    return out
