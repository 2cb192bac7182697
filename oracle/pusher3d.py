"""The coupled guiding-center / Boris pusher in three dimensions (float64).

TEST INFRASTRUCTURE: the definition the 3D HIP path is checked against.

The equations are those of the 2D oracle (`pusher.py`, same notation and
readings); only the geometry changes:
  * 3D3V: positions (x, y, z) in a periodic box, every field component and
    gradient depends on all three coordinates;
  * the gather is trilinear with gradients in x, y and z (`fields3d.py`);
  * d_j b_i runs over j = x, y, z, so (b.grad)b = b_x d_x b + b_y d_y b +
    b_z d_z b and (v_E.grad)b likewise (summed in that order);
  * the guiding-center position R, its midpoints, the fixed-point iteration
    and the iteration error |R^K - R^{K-1}|_inf have three components;
  * the effective cell size of the switch is dl = (dx dy dz)^(1/3) (Sec. 3).
The Boris push, the switch, the parallel update and the curvature drift are
the 2D oracle's functions, which never depended on the number of dimensions.
"""
from __future__ import annotations

from dataclasses import dataclass
from types import SimpleNamespace

import torch

from .ieee import sqrt
from .pusher import (D_FLOOR, GYR_PHASE, KAPPA_FLOOR, ST_BZERO, ST_FPRES, ST_KAPPA,
                     ST_NONFINITE, Params, boris, gamma_gca, gyration, min_image, mirror_check,
                     mirror_parallel, parallel_update, phase_advance, switch_gca, uperp_sq,
                     v_curv, wrap)

F64 = torch.float64

__all__ = ["Params3", "State3", "local3", "boris_step3", "gca_step3", "step3", "push3",
           "D_FLOOR"]


@dataclass
class Params3(Params):
    Lz: float = 0.0
    # dl (inherited) is the effective cell size (dx dy dz)^(1/3)


_KEYS = ("x", "y", "z", "xp", "yp", "zp", "ux", "uy", "uz", "qm", "status")


@dataclass
class State3:
    x: torch.Tensor
    y: torch.Tensor
    z: torch.Tensor
    xp: torch.Tensor
    yp: torch.Tensor
    zp: torch.Tensor
    ux: torch.Tensor
    uy: torch.Tensor
    uz: torch.Tensor
    qm: torch.Tensor
    status: torch.Tensor   # uint8

    @staticmethod
    def from_numpy(ens) -> "State3":
        t = lambda a: torch.as_tensor(a, dtype=F64).clone()
        return State3(*(t(getattr(ens, k)) for k in _KEYS[:-1]),
                      torch.zeros(ens.x.shape[0], dtype=torch.uint8))

    def clone(self) -> "State3":
        return State3(*(getattr(self, k).clone() for k in _KEYS))

    def subset(self, idx) -> "State3":
        return State3(*(getattr(self, k)[idx] for k in _KEYS))


# --------------------------------------------------------------------------
# local field quantities at a point (Sec. 2.2)


def local3(prov, X, Y, Z, p: Params3):
    """b, v_E, kappa, E_par and the curvature terms at points (X, Y, Z); the
    same namespace as the 2D oracle's `local` (with p.exact_frame, the exact
    frame of frame.py)."""
    if p.exact_frame:
        from .frame import local_exact
        return local_exact(prov, X, Y, p, Z)
    s = prov(X, Y, Z)
    Ex, Ey, Ez = s.E
    Bx, By, Bz = s.B
    B2 = (Bx * Bx + By * By) + Bz * Bz
    B = sqrt(B2)
    bzero = B == 0.0
    inv_B = torch.where(bzero, 0.0, 1.0 / torch.where(bzero, 1.0, B))
    bx, by, bz = Bx * inv_B, By * inv_B, Bz * inv_B
    sc = p.c * (inv_B * inv_B)
    vEx = sc * (Ey * Bz - Ez * By)
    vEy = sc * (Ez * Bx - Ex * Bz)
    vEz = sc * (Ex * By - Ey * Bx)
    vE2 = (vEx * vEx + vEy * vEy) + vEz * vEz
    om = 1.0 - vE2 * p.inv_c2
    kflag = om < KAPPA_FLOOR
    om = torch.where(kflag, KAPPA_FLOOR, om)
    kappa = 1.0 / sqrt(om)
    Epar = (Ex * bx + Ey * by) + Ez * bz
    # d_j b_i = (d_j B_i - b_i d_j|B|)/B with d_j|B| = b . d_j B, j = x, y, z
    db, gB = [], []
    for j in range(3):
        gx, gy, gz = s.dB[j]
        dBn = (bx * gx + by * gy) + bz * gz
        gB.append(dBn)
        db.append(((gx - bx * dBn) * inv_B,
                   (gy - by * dBn) * inv_B,
                   (gz - bz * dBn) * inv_B))
    bgb = tuple((bx * db[0][i] + by * db[1][i]) + bz * db[2][i] for i in range(3))
    vgb = tuple((vEx * db[0][i] + vEy * db[1][i]) + vEz * db[2][i] for i in range(3))
    A = (vEx * bgb[0] + vEy * bgb[1]) + vEz * bgb[2]
    C = (vEx * vgb[0] + vEy * vgb[1]) + vEz * vgb[2]
    flags = (torch.where(kflag, ST_KAPPA, 0) | torch.where(bzero, ST_BZERO, 0))
    return SimpleNamespace(E=(Ex, Ey, Ez), Bv=(Bx, By, Bz), B=B, inv_B=inv_B,
                           b=(bx, by, bz), vE=(vEx, vEy, vEz), kappa=kappa,
                           Epar=Epar, bgb=bgb, vgb=vgb, A=A, C=C, gB=tuple(gB),
                           flags=flags.to(torch.uint8))


# --------------------------------------------------------------------------
# full equations of motion: relativistic Boris (Sec. 2.1)


def boris_step3(s, st: State3, p: Params3):
    """Full Boris step: new (x, y, z, u); x^{n+1} = x^n + dt u^{n+1/2}/Gamma^{n+1/2}."""
    ux, uy, uz = boris(s.E, s.B, st.ux, st.uy, st.uz, st.qm, p)
    gn = sqrt(1.0 + ((ux * ux + uy * uy) + uz * uz) * p.inv_c2)
    inv_g = 1.0 / gn
    xn = st.x + p.dt * (ux * inv_g)
    yn = st.y + p.dt * (uy * inv_g)
    zn = st.z + p.dt * (uz * inv_g)
    return wrap(xn, p.Lx), wrap(yn, p.Ly), wrap(zn, p.Lz), ux, uy, uz


# --------------------------------------------------------------------------
# guiding-center leapfrog (Sec. 2.2.1, 2.2.2) inside the coupled step (Sec. 3.1)


def _drift_terms3(L, upar_new, gy, inv_qm, p: Params3):
    """u_par b/Gamma + v_E + v_c at a point, all three components."""
    g = gamma_gca(L, upar_new, gy, p)
    a = upar_new / g
    if p.curvature:
        vc = v_curv(L, upar_new, g, inv_qm, p, gy if p.mirror else None)
        return tuple((a * L.b[i] + L.vE[i]) + vc[i] for i in range(3))
    return tuple(a * L.b[i] + L.vE[i] for i in range(3))


def gca_step3(prov, st: State3, p: Params3):
    """One guiding-center step. Returns (x, y, z, xp, yp, zp, ux, uy, uz, flags, residual)."""
    pos = (st.x, st.y, st.z)
    prev = (st.xp, st.yp, st.zp)
    assert p.curvature or not p.mirror, "the mirror terms ride on the curvature scheme"
    assert not (p.exact_frame and p.mirror), "the mirror terms go with the reduced frame"
    box = (p.Lx, p.Ly, p.Lz)
    qm = st.qm
    ux, uy, uz = st.ux, st.uy, st.uz
    inv_qm = 1.0 / qm
    flags = torch.zeros_like(st.x, dtype=torch.uint8)

    # 1. guiding-center variables at R^{n-1/2} = (x^n + x^{n-1})/2
    Rh = tuple(c - 0.5 * min_image(c - cp, L) for c, cp, L in zip(pos, prev, box))
    Lh = local3(prov, *Rh, p)
    flags |= Lh.flags
    bx, by, bz = Lh.b
    upar = (ux * bx + uy * by) + uz * bz
    gf = sqrt(1.0 + ((ux * ux + uy * uy) + uz * uz) * p.inv_c2)
    if p.curvature:
        vc = v_curv(Lh, upar, gf, inv_qm, p)
    else:
        zr = torch.zeros_like(st.x)
        vc = (zr, zr, zr)
    upx = (ux - upar * bx) - (Lh.vE[0] + vc[0]) * gf
    upy = (uy - upar * by) - (Lh.vE[1] + vc[1]) * gf
    upz = (uz - upar * bz) - (Lh.vE[2] + vc[2]) * gf
    up2 = (upx * upx + upy * upy) + upz * upz
    flags |= mirror_check(up2, gf, p)
    gy = gyration(up2, Lh, p)
    nu = sqrt(up2)
    inv_nu = torch.where(nu > 0.0, 1.0 / torch.where(nu > 0.0, nu, 1.0), 0.0)
    bpx, bpy, bpz = upx * inv_nu, upy * inv_nu, upz * inv_nu

    # 2.-3. fields at R^n = x^n and the parallel four-velocity update
    Ln = local3(prov, *pos, p)
    flags |= Ln.flags
    if p.mirror:
        upn, qf = mirror_parallel(Ln, upar, gy, qm, p)
    else:
        upn, qf = parallel_update(Ln, upar, gy, qm, p)
    flags |= qf
    if p.gyration == GYR_PHASE:
        bpx, bpy, bpz = phase_advance(Ln, upar, upn, gy, qm, (bpx, bpy, bpz), p)

    # 4. R^{n+1} by fixed-point iteration R^{k+1} = R^k - H(R^k), R^0 = R^n
    h = 0.5 * p.dt
    Fn = _drift_terms3(Ln, upn, gy, inv_qm, p)
    R = pos
    res = torch.zeros_like(st.x)
    for k in range(p.n_iter):
        if k == 0:
            Fk = Fn
        else:
            Lk = local3(prov, *R, p)
            flags |= Lk.flags
            Fk = _drift_terms3(Lk, upn, gy, inv_qm, p)
        Rn = tuple(c + h * (a + b) for c, a, b in zip(pos, Fn, Fk))
        d = [torch.abs(a - b) for a, b in zip(Rn, R)]
        res = torch.maximum(torch.maximum(d[0], d[1]), d[2])
        R = Rn
    flags |= torch.where(res > p.fp_tol, ST_FPRES, 0).to(torch.uint8)

    # 5. back to particle variables at R^{n+1/2} = (R^n + R^{n+1})/2
    Rm = tuple(c + 0.5 * (r - c) for c, r in zip(pos, R))
    Lm = local3(prov, *Rm, p)
    flags |= Lm.flags
    gr = gamma_gca(Lm, upn, gy, p)
    if p.curvature:
        vcm = v_curv(Lm, upn, gr, inv_qm, p)
    else:
        zr = torch.zeros_like(st.x)
        vcm = (zr, zr, zr)
    um = sqrt(uperp_sq(Lm, gy))
    bmx, bmy, bmz = Lm.b
    uxn = (upn * bmx + (Lm.vE[0] + vcm[0]) * gr) + um * bpx
    uyn = (upn * bmy + (Lm.vE[1] + vcm[1]) * gr) + um * bpy
    uzn = (upn * bmz + (Lm.vE[2] + vcm[2]) * gr) + um * bpz

    # 6. store x^{n+1} (wrapped), x^n as the previous position, u^{n+1/2}
    return (wrap(R[0], p.Lx), wrap(R[1], p.Ly), wrap(R[2], p.Lz), st.x, st.y, st.z,
            uxn, uyn, uzn, flags, res)


# --------------------------------------------------------------------------
# coupled step (Sec. 3.1) and driver


def _finite_flag(*vals):
    ok = torch.ones_like(vals[0], dtype=torch.bool)
    for v in vals:
        ok &= torch.isfinite(v)
    return torch.where(ok, 0, ST_NONFINITE).to(torch.uint8)


def step3(prov, st: State3, p: Params3):
    """Advance every particle by one step. Returns (new_state, S, residual);
    S is True where the Boris push was used (S = 1)."""
    s = prov(st.x, st.y, st.z)
    gca = switch_gca(s, st.ux, st.uy, st.uz, st.qm, p)
    S = ~gca
    ib = torch.nonzero(S).flatten()
    ig = torch.nonzero(gca).flatten()

    xs = [st.x, st.y, st.z, st.xp, st.yp, st.zp, st.ux, st.uy, st.uz]
    status = st.status.clone()
    res = torch.zeros_like(st.x)
    if ib.numel():
        sb = SimpleNamespace(E=tuple(v[ib] for v in s.E), B=tuple(v[ib] for v in s.B))
        sub = st.subset(ib)
        bx_, by_, bz_, bux, buy, buz = boris_step3(sb, sub, p)
        vals = [bx_, by_, bz_, sub.x, sub.y, sub.z, bux, buy, buz]
        xs = [a.index_put((ib,), v) for a, v in zip(xs, vals)]
        status = status.index_put((ib,), status[ib] | _finite_flag(*vals[:3], *vals[6:]))
    if ig.numel():
        sub = st.subset(ig)
        out = gca_step3(prov, sub, p)
        vals = list(out[:9])
        xs = [a.index_put((ig,), v) for a, v in zip(xs, vals)]
        fl = out[9] | _finite_flag(*vals[:3], *vals[6:])
        status = status.index_put((ig,), status[ig] | fl)
        res = res.index_put((ig,), out[10])
    new = State3(*xs, st.qm, status)
    return new, S, res


def push3(prov, st: State3, p: Params3, n_steps: int, trace: bool = False):
    """Run n_steps coupled steps. Returns (state, S_trace or None, max residual)."""
    tr = [] if trace else None
    maxres = torch.zeros_like(st.x)
    for _ in range(n_steps):
        st, S, res = step3(prov, st, p)
        maxres = torch.maximum(maxres, res)
        if trace:
            tr.append(S.to(torch.uint8))
    return st, (torch.stack(tr) if trace else None), maxres
