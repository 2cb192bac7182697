"""Harris-family static field snapshots on a periodic 2D staggered grid.

Component order everywhere is (Ex, Ey, Ez, Bx, By, Bz).  Each component lives
on its own lattice, offset from the cell corner (i*dx, j*dy) by a fraction of
a cell given by a stagger table.  The default is the 2D Yee arrangement used
by explicit PiC codes (E on edges, B on faces); the paper only states that
fields are interpolated from the surrounding grid points with a linear shape
function (Sec. 4, opening paragraph), so the lattice offsets are an input.

Field family (all closed form, sampled at each component's own nodes):
  * a periodic double Harris sheet,
      Bx(y) = B0 [tanh((y - L/4)/d) - tanh((y - 3L/4)/d) - 1],
    so Bx = -B0 far from the sheets near y = 0 and +B0 between them;
  * a uniform guide field Bz = guide * B0;
  * a divergence-free tearing perturbation with flux
      psi = eps B0 (L/2pi) cos(2pi x/L) sin(2pi y/L),
    giving dBx = eps B0 cos(kx) cos(ky), dBy = eps B0 sin(kx) sin(ky)
    (one X point at x = 0 on each sheet, an O point at x = L/2);
  * an ideal inflow electric field E = -v_in x B / c with
      v_in = (0, -vin*c*sin(4pi (y - L/4)/L), 0)
    that points toward both sheets (E.B = 0, E/B <= vin);
  * optionally a reconnection field Ez += E_rec * sum_X exp(-|x - x_X|^2/(2 d^2))
    centred on the two X points, which makes E > B there.
"""
from __future__ import annotations

import numpy as np

COMPONENTS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")

# (x, y) offsets of each component's nodes, in cells
YEE_STAGGER = np.array([
    [0.5, 0.0],   # Ex on x-edges
    [0.0, 0.5],   # Ey on y-edges
    [0.0, 0.0],   # Ez on nodes
    [0.0, 0.5],   # Bx on x-faces
    [0.5, 0.0],   # By on y-faces
    [0.5, 0.5],   # Bz on cell centres
], dtype=np.float64)

COLLOCATED = np.zeros((6, 2), dtype=np.float64)


def _component(k, X, Y, Lx, Ly, B0, delta, guide, eps, vin, c, E_rec):
    """Analytic component k (0..5 = Ex, Ey, Ez, Bx, By, Bz) at points (X, Y)."""
    kx = 2.0 * np.pi / Lx
    ky = 2.0 * np.pi / Ly

    def bx():
        v = B0 * (np.tanh((Y - 0.25 * Ly) / delta)
                  - np.tanh((Y - 0.75 * Ly) / delta) - 1.0)
        return v + eps * B0 * np.cos(kx * X) * np.cos(ky * Y)

    def vy():
        return -vin * c * np.sin(4.0 * np.pi * (Y - 0.25 * Ly) / Ly)

    if k == 3:
        return bx()
    if k == 4:
        return eps * B0 * np.sin(kx * X) * np.sin(ky * Y)
    if k == 5:
        return np.full(np.broadcast(X, Y).shape, guide * B0)
    # E = -(v x B)/c with v = (0, vy, 0):  v x B = (vy Bz, 0, -vy Bx)
    if k == 0:
        return -vy() * (guide * B0) / c + 0.0 * X
    if k == 1:
        return np.zeros(np.broadcast(X, Y).shape)
    ez = vy() * bx() / c
    if E_rec != 0.0:
        for (x0, y0) in ((0.0, 0.25 * Ly), (0.0, 0.75 * Ly)):
            ddx = X - x0
            ddx = ddx - Lx * np.round(ddx / Lx)
            ddy = Y - y0
            ddy = ddy - Ly * np.round(ddy / Ly)
            ez = ez + E_rec * B0 * np.exp(-(ddx * ddx + ddy * ddy)
                                         / (2.0 * delta * delta))
    return ez


def harris_fields(nx: int, ny: int, dx: float = 1.0, dy: float = 1.0, *,
                  B0: float = 1.0, delta: float = 4.0, guide: float = 0.1,
                  eps: float = 0.01, vin: float = 0.1, c: float = 0.45,
                  E_rec: float = 0.0, stagger=YEE_STAGGER,
                  dtype=np.float64) -> np.ndarray:
    """Sample the field family on an nx x ny periodic grid.

    Returns an array F of shape (6, ny, nx): F[k, j, i] is component k at
    ((i + stagger[k,0]) dx, (j + stagger[k,1]) dy).  `delta` is in length
    units (cells when dx = 1); `E_rec` is in units of B0.
    """
    stagger = np.asarray(stagger, dtype=np.float64)
    Lx, Ly = nx * dx, ny * dy
    out = np.empty((6, ny, nx), dtype=dtype)
    ii = np.arange(nx, dtype=np.float64)
    jj = np.arange(ny, dtype=np.float64)
    for k in range(6):
        X = ((ii + stagger[k, 0]) * dx)[None, :]
        Y = ((jj + stagger[k, 1]) * dy)[:, None]
        out[k] = np.broadcast_to(
            _component(k, X, Y, Lx, Ly, B0, delta, guide, eps, vin, c, E_rec),
            (ny, nx))
    return out
