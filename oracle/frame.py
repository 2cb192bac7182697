"""The exact guiding-center frame of Sec. 2.2 (float64, torch CPU).

TEST INFRASTRUCTURE: the definition the exact-frame option of the HIP path is
checked against.

The paper splits u along b*, the direction of the magnetic field in the frame
that moves with v_E and in which E and B are parallel, and gives that frame
in closed form:
  w_E = c E x B/(E^2 + B^2),  v_E = w_E (1 - s)/(2 w_E^2/c^2),
  s = sqrt(1 - 4 w_E^2/c^2),  kappa = (1 - v_E^2/c^2)^(-1/2),
  B' = sqrt((B^2 - E^2 + (B^2 + E^2) s)/2),  E' = E.B/B',
  E_perp = E - (E.B) B/B^2,  Psi = E'(B^2 - B'^2)/(B' E_perp^2),
  eta = 1/(B sqrt(Psi^2 E_perp^2/B^2 + 1)),  xi = eta Psi,
  b* = xi E_perp + eta B.
It then replaces them by b = B/B and v_E = c E x B/B^2 for its schemes.

Readings used here (each listed with its reason in the design notes):
  * Two algebraically identical forms free of 0/0 where E x B -> 0:
    v_E = 2 w_E/(1 + s), and, since B^2 - B'^2 = (E^2 + B^2)(1 - s)/2 and
    |E x B| = E_perp B,  Psi = 2 E' B^2/(B'(E^2 + B^2)(1 + s)).
  * Parallel equation: in the moving frame the only force along b* is q E';
    u_par = u.b* is unchanged by the boost (b* is perpendicular to v_E) and
    the moving frame's clock runs slow by kappa, so du_par/dt = (q/m) E'/kappa
    (equal to (q/m)(E + v_E x B/c).b*; it reduces to (q/m) E.b when E.B = 0).
  * The local namespace keeps the lab-frame B in mu = m u_perp_g^2/(2 B kappa)
    and eq. lfacgca2, with the exact kappa.
  * With the curvature scheme (Sec. 2.2.2) b* stands for b in eq. curvdrift
    and eq. dupardt, in the cross product and in both directional derivatives,
    (b*.grad)b* and (v_E.grad)b*, with the exact v_E; the prefactor
    m c kappa^2/(q B) keeps the lab B, as mu does.  b* is a function of the
    local E and B only, so its gradient is the chain rule
    d_j b*_i = sum_c (d b*_i/d F_c) d_j F_c over the six components, with the
    gather gradients d_j F_c (the E components differentiated through W on
    their own lattices, as the B components are).  The partial derivatives
    d b*_i/d F_c are taken by reverse-mode differentiation of `exact_frame`
    (torch autograd, a library primitive).  Where B = 0, b* = 0 and its
    gradient is 0.
  * B = 0: b* = 0, v_E = 0 and the B = 0 flag, as for the reduced frame;
    B' = 0 (E x B with E > B and E.B = 0): E' = 0 and Psi = 0.
"""
from __future__ import annotations

from types import SimpleNamespace

import torch

from .ieee import sqrt

KAPPA_FLOOR = 1.0e-12
ST_KAPPA = 2
ST_BZERO = 8


def exact_frame(E, B, p):
    """The frame quantities of Sec. 2.2 from lab-frame E and B (tuples of
    three tensors).  Returns a namespace with vE, kappa, Bp (B'), Ep (E'),
    Eperp, Psi, eta, xi, bstar, Epar (= E'/kappa), B, inv_B and flags."""
    Ex, Ey, Ez = E
    Bx, By, Bz = B
    E2 = (Ex * Ex + Ey * Ey) + Ez * Ez
    B2 = (Bx * Bx + By * By) + Bz * Bz
    EB = (Ex * Bx + Ey * By) + Ez * Bz
    S = E2 + B2
    Bm = sqrt(B2)
    bzero = Bm == 0.0
    inv_B = torch.where(bzero, 0.0, 1.0 / torch.where(bzero, 1.0, Bm))
    # w_E = c E x B/(E^2 + B^2)
    szero = S == 0.0
    f = torch.where(szero, 0.0, torch.full_like(S, p.c) / torch.where(szero, 1.0, S))
    wx = f * (Ey * Bz - Ez * By)
    wy = f * (Ez * Bx - Ex * Bz)
    wz = f * (Ex * By - Ey * Bx)
    w2 = (wx * wx + wy * wy) + wz * wz
    s_arg = 1.0 - (4.0 * w2) * p.inv_c2
    s = sqrt(torch.where(s_arg > 0.0, s_arg, 0.0))
    # v_E = w_E (1 - s)/(2 w_E^2/c^2) = 2 w_E/(1 + s)
    g = 2.0 / (1.0 + s)
    vE = (g * wx, g * wy, g * wz)
    vE2 = (vE[0] * vE[0] + vE[1] * vE[1]) + vE[2] * vE[2]
    om = 1.0 - vE2 * p.inv_c2
    kflag = om < KAPPA_FLOOR
    om = torch.where(kflag, KAPPA_FLOOR, om)
    kappa = 1.0 / sqrt(om)
    # B' and E' in the moving frame
    Bp2 = 0.5 * ((B2 - E2) + S * s)
    Bp = sqrt(torch.where(Bp2 > 0.0, Bp2, 0.0))
    bpzero = Bp == 0.0
    Ep = torch.where(bpzero, 0.0, EB / torch.where(bpzero, 1.0, Bp))
    # E_perp = E - (E.B) B/B^2
    a = torch.where(bzero, 0.0, EB / torch.where(bzero, 1.0, B2))
    Eperp = (Ex - a * Bx, Ey - a * By, Ez - a * Bz)
    Eperp2 = (Eperp[0] * Eperp[0] + Eperp[1] * Eperp[1]) + Eperp[2] * Eperp[2]
    # Psi = E'(B^2 - B'^2)/(B' E_perp^2) = 2 E' B^2/(B' (E^2 + B^2)(1 + s))
    Psi = torch.where(bpzero, 0.0,
                      ((2.0 * Ep) * B2) / torch.where(bpzero, 1.0, (Bp * S) * (1.0 + s)))
    q = torch.where(bzero, 0.0, ((Psi * Psi) * Eperp2) / torch.where(bzero, 1.0, B2))
    eta = torch.where(bzero, 0.0, 1.0 / torch.where(bzero, 1.0, Bm * sqrt(q + 1.0)))
    xi = eta * Psi
    bstar = tuple(xi * e + eta * b for e, b in zip(Eperp, (Bx, By, Bz)))
    flags = torch.where(kflag, ST_KAPPA, 0) | torch.where(bzero, ST_BZERO, 0)
    return SimpleNamespace(vE=vE, kappa=kappa, Bp=Bp, Ep=Ep, Eperp=Eperp, Psi=Psi,
                           eta=eta, xi=xi, bstar=bstar, Epar=Ep / kappa, B=Bm, inv_B=inv_B,
                           flags=flags.to(torch.uint8), E=(Ex, Ey, Ez), Bv=(Bx, By, Bz))


def bstar_jacobian(E, B, p):
    """J[i][c] = d b*_i / d F_c, F = (Ex, Ey, Ez, Bx, By, Bz), per particle:
    reverse-mode differentiation of `exact_frame` (each particle's b* depends
    on its own E and B only, so the gradient of the sum over particles is the
    per-particle derivative).  Zero where B = 0."""
    leaves = [v.detach().clone().requires_grad_(True) for v in (*E, *B)]
    with torch.enable_grad():
        fr = exact_frame(tuple(leaves[:3]), tuple(leaves[3:]), p)
        J = []
        for i in range(3):
            g = torch.autograd.grad(fr.bstar[i].sum(), leaves, retain_graph=i < 2,
                                    allow_unused=True)
            J.append([torch.zeros_like(E[0]) if gi is None else gi.detach() for gi in g])
    bzero = fr.B.detach() == 0.0
    return [[torch.where(bzero, 0.0, v) for v in row] for row in J]


def curvature_terms(fr, dF, p):
    """(b*.grad)b*, (v_E.grad)b*, A = v_E.(b*.grad)b*, C = v_E.(v_E.grad)b*
    from the frame `fr` and the field gradients dF[j][c] = d_j F_c
    (j over the dimensions of the provider, c over the six components)."""
    J = bstar_jacobian(fr.E, fr.Bv, p)
    nd = len(dF)
    # d_j b*_i = sum_c J[i][c] d_j F_c
    db = [[sum(J[i][c] * dF[j][c] for c in range(6)) for i in range(3)] for j in range(nd)]
    bs, vE = fr.bstar, fr.vE
    bgb = tuple(sum(bs[j] * db[j][i] for j in range(nd)) for i in range(3))
    vgb = tuple(sum(vE[j] * db[j][i] for j in range(nd)) for i in range(3))
    A = (vE[0] * bgb[0] + vE[1] * bgb[1]) + vE[2] * bgb[2]
    C = (vE[0] * vgb[0] + vE[1] * vgb[1]) + vE[2] * vgb[2]
    return bgb, vgb, A, C


def local_exact(prov, X, Y, p, Z=None):
    """The local namespace of the guiding-center step (see `pusher.local`)
    with b = b*, the exact v_E and kappa, and E_par = E'/kappa; with
    p.curvature the curvature terms of b* (`curvature_terms`).  Z for a 3D
    provider."""
    s = prov(X, Y) if Z is None else prov(X, Y, Z)
    fr = exact_frame(s.E, s.B, p)
    z = torch.zeros_like(X)
    if p.curvature:
        dE = prov.e_gradient(X, Y) if Z is None else prov.e_gradient(X, Y, Z)
        dF = [tuple(dE[j]) + tuple(s.dB[j]) for j in range(len(s.dB))]
        bgb, vgb, A, C = curvature_terms(fr, dF, p)
    else:
        bgb, vgb, A, C = (z, z, z), (z, z, z), z, z
    return SimpleNamespace(E=fr.E, Bv=fr.Bv, B=fr.B, inv_B=fr.inv_B, b=fr.bstar, vE=fr.vE,
                           kappa=fr.kappa, Epar=fr.Epar, bgb=bgb, vgb=vgb, A=A, C=C,
                           flags=fr.flags)
