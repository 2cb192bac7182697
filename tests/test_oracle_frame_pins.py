"""Pins of the exact guiding-center frame (Sec. 2.2) in the oracle against
the Lorentz transformation of the fields, its invariants, the limits the
paper states, and a gyro-resolved Boris trajectory.  No GPU."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from oracle.frame import exact_frame

F64 = torch.float64


def T(*v):
    return torch.tensor(v, dtype=F64)


def _fields(rng, n, e_scale):
    E = rng.normal(size=(3, n)) * e_scale
    B = rng.normal(size=(3, n))
    return E, B


def _frame(E, B, c):
    fr = exact_frame(tuple(torch.as_tensor(v) for v in E), tuple(torch.as_tensor(v) for v in B),
                     O.Params(c=c))
    arr = lambda t: np.stack([v.numpy() for v in t])
    return fr, arr(fr.vE), arr(fr.bstar)


@pytest.mark.parametrize("c,e_scale", [(0.45, 0.3), (1.0, 1.5)])
def test_bstar_is_the_boosted_magnetic_field_direction(c, e_scale):
    """Boosting by v_E (perpendicular to E and B) gives E' = kappa (E + v_E x B/c)
    and B' = kappa (B - v_E x E/c) (textbook field transformation): they are
    parallel, |B'| and E'.b* equal the paper's B' and E', and b* = B'/|B'|.
    Fields with E > B (and E.B != 0) included."""
    rng = np.random.default_rng(41)
    E, B = _fields(rng, 400, e_scale)
    # the paper's B' cancels where E > B and E.B -> 0 (B' -> 0, no magnetized
    # frame): keep frames with B' above 5 % of |(E, B)|
    fr, _, _ = _frame(E, B, c)
    keep = fr.Bp.numpy() > 0.05 * np.sqrt((E * E).sum(0) + (B * B).sum(0))
    assert keep.mean() > 0.8
    E, B = E[:, keep], B[:, keep]
    fr, vE, bs = _frame(E, B, c)
    kap = fr.kappa.numpy()
    assert np.all(np.linalg.norm(vE, axis=0) < c)
    Ep = kap * (E + np.cross(vE.T, B.T).T / c)
    Bp = kap * (B - np.cross(vE.T, E.T).T / c)
    nB = np.linalg.norm(Bp, axis=0)
    nE = np.linalg.norm(Ep, axis=0)
    assert np.all(np.linalg.norm(np.cross(Ep.T, Bp.T).T, axis=0) <= 1e-12 * nE * nB + 1e-15)
    assert np.allclose(nB, fr.Bp.numpy(), rtol=1e-12)
    assert np.allclose((Ep * bs).sum(axis=0), fr.Ep.numpy(), rtol=1e-11, atol=1e-14)
    assert np.allclose(bs, Bp / nB, rtol=0, atol=1e-12)
    # v_E is perpendicular to E and B, b* to v_E
    assert np.allclose((vE * E).sum(axis=0), 0, atol=1e-14)
    assert np.allclose((vE * bs).sum(axis=0), 0, atol=1e-14)


def test_lorentz_invariants():
    """B'^2 - E'^2 = B^2 - E^2 and E' B' = E.B (frames with B' above 5 % of
    |(E, B)|, as above)."""
    rng = np.random.default_rng(42)
    E, B = _fields(rng, 400, 0.8)
    fr, _, _ = _frame(E, B, 0.45)
    keep = fr.Bp.numpy() > 0.05 * np.sqrt((E * E).sum(0) + (B * B).sum(0))
    assert keep.mean() > 0.8
    E, B = E[:, keep], B[:, keep]
    fr, _, _ = _frame(E, B, 0.45)
    Bp, Ep = fr.Bp.numpy(), fr.Ep.numpy()
    assert np.allclose(Bp ** 2 - Ep ** 2, (B * B).sum(0) - (E * E).sum(0), rtol=1e-12, atol=1e-13)
    assert np.allclose(Ep * Bp, (E * B).sum(0), rtol=1e-12, atol=1e-14)


def test_limits_for_perpendicular_fields():
    """E.B = 0 (Sec. 2.2), E < B: b* = b, v_E = c E x B/B^2 and kappa =
    (1 - E^2/B^2)^(-1/2); E > B: |v_E| = c B/E (there B' = 0: the moving
    frame holds no magnetic field and b* is not defined)."""
    rng = np.random.default_rng(43)
    c = 0.45
    B = rng.normal(size=(3, 200))
    d = rng.normal(size=(3, 200))
    Eu = np.cross(B.T, d.T).T                       # perpendicular to B
    Eu /= np.linalg.norm(Eu, axis=0)
    Bm = np.linalg.norm(B, axis=0)
    for ratio in (0.3, 2.5):
        E = Eu * ratio * Bm
        fr, vE, bs = _frame(E, B, c)
        if ratio < 1:
            assert np.allclose(bs, B / Bm, rtol=0, atol=1e-14)
            assert np.allclose(vE, c * np.cross(E.T, B.T).T / Bm ** 2, rtol=1e-13, atol=1e-16)
            assert np.allclose(fr.kappa.numpy(), 1 / np.sqrt(1 - ratio ** 2), rtol=1e-13)
        else:
            assert np.allclose(np.linalg.norm(vE, axis=0), c / ratio, rtol=1e-13)


def test_first_order_form_for_small_parallel_field():
    """E.B -> 0: b* -> (B + E_perp (E.B)/B'^2)/B (the relativistic drift term of
    Sec. 2.2) with a remainder of second order in E.B."""
    rng = np.random.default_rng(44)
    B = rng.normal(size=(3, 50))
    Bm = np.linalg.norm(B, axis=0)
    Eperp = np.cross(B.T, rng.normal(size=(3, 50)).T).T
    Eperp *= 0.3 * Bm / np.linalg.norm(Eperp, axis=0)
    errs = []
    for eps in (1e-2, 5e-3):
        E = Eperp + eps * B
        fr, _, bs = _frame(E, B, 1.0)
        EB = (E * B).sum(0)
        Bp2 = Bm ** 2 * (1 - (Eperp * Eperp).sum(0) / Bm ** 2)
        approx = (B + Eperp * EB / Bp2) / Bm
        errs.append(np.max(np.linalg.norm(bs - approx, axis=0)))
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_exact_frame_guiding_center_step_closed_form():
    """One zero-curvature step with the exact frame in uniform fields:
    u_par += (q/m) dt E'/kappa along b*, R += dt (u_par b*/Gamma + v_E)."""
    c, dt, qm = 0.45, 1.0, -3.0
    E = np.array([0.03, -0.05, 0.02])
    B = np.array([0.2, 0.4, 0.8])
    u = np.array([0.05, 0.1, -0.02])
    p = O.Params(dt=dt, c=c, f_rho=1e9, f_E=1e9, curvature=False, exact_frame=True,
                 Lx=1e6, Ly=1e6)
    st = O.State(T(7.0), T(9.0), T(7.0), T(9.0), T(u[0]), T(u[1]), T(u[2]), T(qm),
                 torch.zeros(1, dtype=torch.uint8))
    st2, S, _ = O.step(O.UniformFields(E, B), st, p)
    assert not bool(S[0])
    fr, vE, bs = _frame(E[:, None], B[:, None], c)
    vE, bs = vE[:, 0], bs[:, 0]
    kap, Ep = float(fr.kappa), float(fr.Ep)
    gf = math.sqrt(1 + u @ u / c ** 2)
    upar = u @ bs
    uperp = u - upar * bs - vE * gf
    upn = upar + qm * dt * Ep / kap
    gam = kap * math.sqrt(1 + (upn ** 2 + uperp @ uperp) / c ** 2)
    dR = dt * (upn * bs / gam + vE)
    assert abs(float(st2.x) - 7.0 - dR[0]) < 1e-14
    assert abs(float(st2.y) - 9.0 - dR[1]) < 1e-14
    got = np.array([float(st2.ux), float(st2.uy), float(st2.uz)])
    assert np.allclose(got, upn * bs + vE * gam + uperp, rtol=0, atol=1e-14)


def test_exact_frame_follows_the_resolved_orbit():
    """Uniform fields with E.B != 0 and a particle without gyration in the
    moving frame (u = u_par b* + v_E Gamma): the gyro-resolved Boris orbit is
    the guiding-center orbit itself.  The exact-frame scheme with a step 200
    times larger stays on it; the reduced frame (b, c E x B/B^2) drifts off
    along the tilt between b and b*."""
    c, qm = 0.45, -2.0
    E = np.array([0.12, 0.0, 0.05])
    B = np.array([0.0, 0.0, 1.0])
    fr, vE, bs = _frame(E[:, None], B[:, None], c)
    vE, bs, kap = vE[:, 0], bs[:, 0], float(fr.kappa)
    upar0 = 0.1
    u0 = upar0 * bs + vE * kap * math.sqrt(1 + upar0 ** 2 / c ** 2)
    prov = O.UniformFields(E, B)

    def run(p, n):
        g = math.sqrt(1 + u0 @ u0 / c ** 2)
        st = O.State(T(100.0), T(100.0), T(100.0 - p.dt * u0[0] / g),
                     T(100.0 - p.dt * u0[1] / g), T(u0[0]), T(u0[1]), T(u0[2]), T(qm),
                     torch.zeros(1, dtype=torch.uint8))
        for _ in range(n):
            st, _, _ = O.step(prov, st, p)
        return (np.array([float(st.x), float(st.y)]),
                np.array([float(st.ux), float(st.uy), float(st.uz)]))

    t_end, dtb = 40.0, 0.005
    xb, ub = run(O.Params(c=c, dt=dtb, f_rho=0.0, Lx=1e6, Ly=1e6), int(t_end / dtb))
    res = {}
    for exact in (False, True):
        p = O.Params(c=c, dt=1.0, f_rho=1e9, f_E=1e9, curvature=False, exact_frame=exact,
                     Lx=1e6, Ly=1e6)
        res[exact] = run(p, int(t_end))
    dx_red = np.linalg.norm(res[False][0] - xb)
    dx_ex = np.linalg.norm(res[True][0] - xb)
    du_red = np.linalg.norm(res[False][1] - ub) / np.linalg.norm(ub)
    du_ex = np.linalg.norm(res[True][1] - ub) / np.linalg.norm(ub)
    assert dx_red > 0.05 and dx_ex < 0.05 * dx_red
    assert du_red > 1e-3 and du_ex < 1e-6


def test_exact_frame_equals_reduced_frame_when_fields_are_perpendicular():
    """Fields perpendicular in floating point at every point (B along z, E in
    the plane; E < B): the exact frame is the reduced one, and a
    zero-curvature run agrees to rounding with identical decisions."""
    rng = np.random.default_rng(45)
    prov = O.LinearFields(E0=[0.02, -0.01, 0.0], GE=[[1e-3, 2e-3], [-1e-3, 5e-4], [0.0, 0.0]],
                          B0=[0.0, 0.0, 1.0], GB=[[0.0, 0.0], [0.0, 0.0], [2e-3, -1e-3]])
    n = 200
    x, y = rng.uniform(0, 50, n), rng.uniform(0, 50, n)
    u = 0.2 * rng.normal(size=(3, n))
    qm = -np.where(np.arange(n) % 3 == 0, 0.05, 50.0)       # some Boris, most GCA
    st0 = O.State(*(torch.as_tensor(v) for v in (x, y, x.copy(), y.copy(), *u, qm)),
                  torch.zeros(n, dtype=torch.uint8))
    kw = dict(c=0.45, curvature=False, Lx=1e6, Ly=1e6, dl=1.0)
    a, Sa, _ = O.push(prov, st0.clone(), O.Params(**kw), 10, trace=True)
    b, Sb, _ = O.push(prov, st0.clone(), O.Params(exact_frame=True, **kw), 10, trace=True)
    assert torch.equal(Sa, Sb) and 0 < int(Sa.sum()) < Sa.numel()
    for k in ("x", "y", "ux", "uy", "uz"):
        assert torch.allclose(getattr(a, k), getattr(b, k), rtol=1e-12, atol=1e-14), k
