"""Pins of the exact guiding-center frame (Sec. 2.2) in the oracle against
the Lorentz transformation of the fields, its invariants, the limits the
paper states, and a gyro-resolved Boris trajectory.  No GPU."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from oracle.frame import exact_frame, local_exact

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


# ---------------------------------------------------------------------------
# the exact frame with the curvature scheme (Sec. 2.2 with Sec. 2.2.2): the
# curvature terms are built from the gradient of b*, which depends on E too


def _bstar_at(prov, p, *X):
    s = prov(*X)
    return exact_frame(s.E, s.B, p).bstar


@pytest.mark.parametrize("nd", [2, 3])
def test_exact_frame_curvature_terms_match_finite_differences(nd):
    """(b*.grad)b*, (v_E.grad)b*, A and C of the oracle against central
    differences of b* itself, evaluated from the fields at displaced points,
    for fields linear in position with E.B != 0 (so b* differs from b and
    depends on the gradients of both E and B)."""
    rng = np.random.default_rng(47 + nd)
    n = 64
    E0 = np.array([0.06, -0.04, 0.09])[:, None] + 0.0 * rng.normal(size=(3, 1))
    B0 = np.array([0.3, 0.5, 0.8])
    GE = rng.normal(0.0, 0.004, (3, nd))
    GB = rng.normal(0.0, 0.01, (3, nd))
    if nd == 2:
        prov = O.LinearFields(E0[:, 0], GE, B0, GB)
        p = O.Params(c=0.45, curvature=True, exact_frame=True, Lx=1e6, Ly=1e6)
    else:
        prov = O.LinearFields3(E0[:, 0], GE, B0, GB)
        p = O.Params3(c=0.45, curvature=True, exact_frame=True, Lx=1e6, Ly=1e6, Lz=1e6)
    X = [torch.as_tensor(rng.uniform(0.0, 6.0, n)) for _ in range(nd)]
    L = local_exact(prov, *X[:2], p, *X[2:])
    h = 1e-5
    db = []
    for j in range(nd):
        Xp = [x + (h if k == j else 0.0) for k, x in enumerate(X)]
        Xm = [x - (h if k == j else 0.0) for k, x in enumerate(X)]
        db.append([(a - b) / (2 * h) for a, b in
                   zip(_bstar_at(prov, p, *Xp), _bstar_at(prov, p, *Xm))])
    bgb = [sum(L.b[j] * db[j][i] for j in range(nd)) for i in range(3)]
    vgb = [sum(L.vE[j] * db[j][i] for j in range(nd)) for i in range(3)]
    scale = max(float(torch.stack(bgb).abs().max()), float(torch.stack(vgb).abs().max()))
    assert scale > 1e-4   # the terms are not trivially small
    for i in range(3):
        assert float((L.bgb[i] - bgb[i]).abs().max()) < 1e-7 * scale
        assert float((L.vgb[i] - vgb[i]).abs().max()) < 1e-7 * scale
    A = (L.vE[0] * bgb[0] + L.vE[1] * bgb[1]) + L.vE[2] * bgb[2]
    C = (L.vE[0] * vgb[0] + L.vE[1] * vgb[1]) + L.vE[2] * vgb[2]
    assert float((L.A - A).abs().max()) < 1e-7 * scale
    assert float((L.C - C).abs().max()) < 1e-7 * scale
    # b* itself differs from b by much more than the tolerance
    s = prov(*X)
    Bm = torch.sqrt(sum(v * v for v in s.B))
    assert float(max((bs - Bv / Bm).abs().max() for bs, Bv in zip(L.b, s.B))) > 1e-3


@pytest.mark.parametrize("nd", [2, 3])
def test_grid_e_gradient_is_the_derivative_of_the_gather(nd):
    """The gather's E gradients (differentiated W on each E lattice) equal the
    slope of the gathered E along each axis inside a cell, where the
    interpolant is linear along the axis."""
    rng = np.random.default_rng(53 + nd)
    shape = (6,) + (8,) * nd
    prov = (O.GridFields(rng.normal(size=shape)) if nd == 2
            else O.GridFields3(rng.normal(size=shape)))
    n = 100
    # points at least 0.1 cell from every lattice line of every component
    X = [torch.as_tensor(np.floor(rng.uniform(0, 8, n)) + rng.uniform(0.1, 0.4, n))
         for _ in range(nd)]
    dE = prov.e_gradient(*X)
    h = 1e-6
    for j in range(nd):
        Xp = [x + (h if k == j else 0.0) for k, x in enumerate(X)]
        Xm = [x - (h if k == j else 0.0) for k, x in enumerate(X)]
        for i in range(3):
            fd = (prov(*Xp).E[i] - prov(*Xm).E[i]) / (2 * h)
            assert torch.allclose(dE[j][i], fd, rtol=1e-7, atol=1e-8)


def test_exact_frame_curvature_equals_reduced_frame_for_ideal_fields():
    """Ideal fields E = -v x B/c with uniform v (E.B = 0 up to rounding at every
    point, E < B): b* = b and the exact v_E is c E x B/B^2, and the gradient of
    b* reduces to that of b (its E-dependent part is proportional to the
    gradient of E.B).  The curvature scheme in both frames then agrees to
    rounding over a multi-step run, with identical switch decisions."""
    rng = np.random.default_rng(59)
    c = 0.45
    v = np.array([0.02, -0.03, 0.01])
    B0 = np.array([0.3, 0.2, 1.0])
    GB = rng.normal(0.0, 0.02, (3, 2))
    E0 = -np.cross(v, B0) / c
    GE = np.stack([-np.cross(v, GB[:, j]) / c for j in range(2)], axis=1)
    prov = O.LinearFields(E0, GE, B0, GB)
    n = 200
    # inside the box, away from its edges: no wrap over the run
    x, y = rng.uniform(20, 40, n), rng.uniform(20, 40, n)
    u = 0.2 * rng.normal(size=(3, n))
    qm = -np.where(np.arange(n) % 3 == 0, 0.05, 20.0)
    st0 = O.State(*(torch.as_tensor(w) for w in (x, y, x.copy(), y.copy(), *u, qm)),
                  torch.zeros(n, dtype=torch.uint8))
    kw = dict(c=c, curvature=True, Lx=1e6, Ly=1e6, dl=1.0)
    Lr = O.local(prov, st0.x, st0.y, O.Params(**kw))
    Le = O.local(prov, st0.x, st0.y, O.Params(exact_frame=True, **kw))
    for k in ("b", "vE", "bgb", "vgb"):
        for a, b in zip(getattr(Lr, k), getattr(Le, k)):
            assert torch.allclose(a, b, rtol=1e-12, atol=1e-15), k
    for k in ("kappa", "A", "C", "Epar"):
        assert torch.allclose(getattr(Lr, k), getattr(Le, k), rtol=1e-12, atol=1e-15), k
    assert float(torch.stack(Lr.bgb).abs().max()) > 1e-3
    a, Sa, _ = O.push(prov, st0.clone(), O.Params(**kw), 10, trace=True)
    b, Sb, _ = O.push(prov, st0.clone(), O.Params(exact_frame=True, **kw), 10, trace=True)
    assert torch.equal(Sa, Sb) and 0 < int(Sa.sum()) < Sa.numel()
    for k in ("x", "y", "ux", "uy", "uz"):
        assert torch.allclose(getattr(a, k), getattr(b, k), rtol=1e-11, atol=1e-13), k


def test_exact_frame_curvature_in_uniform_fields_is_the_zero_curvature_step():
    """Uniform fields with E.B != 0: the gradient of b* vanishes, so the
    curvature scheme in the exact frame takes exactly (bit for bit) the step
    of the zero-curvature scheme: the quadratic's root reduces to the explicit
    parallel update and the curvature drift to zero."""
    rng = np.random.default_rng(61)
    E = [0.05, -0.02, 0.07]
    B = [0.2, 0.4, 0.8]
    prov = O.UniformFields(E, B)
    n = 100
    x, y = rng.uniform(0, 20, n), rng.uniform(0, 20, n)
    u = 0.2 * rng.normal(size=(3, n))
    qm = -np.full(n, 20.0)
    st0 = O.State(*(torch.as_tensor(w) for w in (x, y, x - 0.01, y + 0.02, *u, qm)),
                  torch.zeros(n, dtype=torch.uint8))
    kw = dict(c=0.45, exact_frame=True, Lx=1e6, Ly=1e6, dl=1.0)
    a, Sa, _ = O.push(prov, st0.clone(), O.Params(curvature=False, **kw), 5, trace=True)
    b, Sb, _ = O.push(prov, st0.clone(), O.Params(curvature=True, **kw), 5, trace=True)
    assert not bool(Sa.any()) and torch.equal(Sa, Sb)
    for k in ("x", "y", "xp", "yp", "ux", "uy", "uz"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
