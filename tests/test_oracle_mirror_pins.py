"""Pins of the oracle's mirror option (Params.mirror): the mirror force and
the grad-B drift that Sec. 2.2 names and then leaves out of the reduced
equations, added to the curvature scheme of Sec. 2.2.2.  No GPU.

The paper prints no formula for these terms, so the pins use what the
physics fixes when E = 0 (kappa = 1, where every reading of the terms
agrees):
  * the mirror force -(mu/(m Gamma)) b.grad|B| keeps u_par^2 + 2 mu B/m = |u|^2
    constant along the guiding-center path, so a particle that moves into a
    stronger field turns where B = B_start |u|^2/u_perp^2; the gyro-resolved
    Boris orbit turns at the same point (test_oracle_pins.py).  The state
    holds u_par half a step before the position, so the leapfrog starts from
    u_par(t = 0) = u_par - (dt/2) F with F the deceleration, and keeps the
    time-centred energy u_par^{n-1/2} u_par^{n+1/2} + 2 mu B(R^n)/m (exactly
    for a constant force and Gamma);
  * with u_par = 0 in a field of uniform direction, the guiding center moves
    at the relativistic grad-B drift c u_perp^2/(2 (q/m) Gamma B^2) b x grad|B|
    with Gamma = sqrt(1 + u_perp^2/c^2);
  * both terms carry mu: with mu = 0 the option changes nothing, bit for bit.
A dropped 1/Gamma, a factor 2, a wrong sign or a term missing from one of the
two places fails one of these.
"""
import numpy as np
import torch

import oracle as O

F64 = torch.float64


def T(*v):
    return torch.tensor(v, dtype=F64)


def params(**kw):
    base = dict(dt=1.0, c=0.45, f_rho=0.4, f_E=1.0, curvature=True, n_iter=4,
                Lx=1.0e6, Ly=1.0e6, dl=1.0, mirror=True)
    base.update(kw)
    return O.Params(**base)


def state(x, y, ux, uy, uz, qm):
    n = len(ux)
    x = torch.full((n,), x, dtype=F64)
    y = torch.full((n,), y, dtype=F64)
    return O.State(x, y, x.clone(), y.clone(), T(*ux), T(*uy), T(*uz), T(*qm),
                   torch.zeros(n, dtype=torch.uint8))


# B = B0 (1 + g x) x_hat from x = X0: b = x_hat, grad|B| = B0 g x_hat is along b
GRAD, X0 = 0.2, 5.0
UPAR = np.array([0.03, 0.2, 0.3, 0.9])
UPERP = np.array([0.04, 0.3, 0.4, 1.2])


def _ramp():
    return O.LinearFields([0, 0, 0], np.zeros((3, 2)), [1.0, 0, 0],
                          [[GRAD, 0], [0, 0], [0, 0]])


def _turn_steps(upar, uperp, c=0.45):
    """Steps to the turn: u_par falls at the constant rate
    (mu/(m Gamma)) g = u_perp^2 g/(2 Gamma B(X0))."""
    gam = np.sqrt(1.0 + (upar ** 2 + uperp ** 2) / c ** 2)
    return 2.0 * upar * gam * (1.0 + GRAD * X0) / (uperp ** 2 * GRAD)


def _expected_turn(c=0.45):
    """Distance from X0 to the turn: B0 u_par(0)^2/(u_perp^2 g), with
    u_par(0) = u_par - (dt/2) u_perp^2 g/(2 Gamma B0) (dt = 1)."""
    B0 = 1.0 + GRAD * X0
    gam = np.sqrt(1.0 + (UPAR ** 2 + UPERP ** 2) / c ** 2)
    u0 = UPAR - 0.5 * UPERP ** 2 * GRAD / (2.0 * gam * B0)
    return B0 * u0 ** 2 / (UPERP ** 2 * GRAD)


def _bounce(p, lim, three_d=False, make=None):
    """Guiding-center paths in the ramp, each followed for lim[i] steps (the
    particle is back at X0 after about twice its turn time); returns (largest
    distance from X0 along the ramp, u_par at the end of each path, largest
    relative change of the time-centred energy)."""
    n = len(UPAR)
    st = make() if make else state(X0, 2.0, list(UPAR), [0.0] * n, list(UPERP), [-20.0] * n)
    if three_d:
        step, prov, pos, prev, upar = O.step3, _ramp3(), "z", "zp", "uz"
    else:
        step, prov, pos, prev, upar = O.step, _ramp(), "x", "xp", "ux"
    mu = UPERP ** 2 / (2.0 * (1.0 + GRAD * X0))
    xmax, dev, upar_end = np.zeros(n), np.zeros(n), np.zeros(n)
    u_old, I0 = getattr(st, upar).numpy(), None
    for k in range(int(np.max(lim))):
        st, S, _ = step(prov, st, p)
        assert not bool(S.any())            # guiding center throughout
        live = k < lim
        u_new = getattr(st, upar).numpy()
        I = u_old * u_new + 2.0 * mu * (1.0 + GRAD * getattr(st, prev).numpy())
        I0 = I if I0 is None else I0
        u_old = u_new
        xmax = np.where(live, np.maximum(xmax, getattr(st, pos).numpy() - X0), xmax)
        dev = np.where(live, np.maximum(dev, np.abs(I / I0 - 1.0)), dev)
        upar_end = np.where(live, u_new, upar_end)
    return xmax, upar_end, dev


def test_mirror_force_turns_at_the_mirror_point():
    """The four particles (Gamma from 1.006 to 3.5, all with the guiding-center
    step, 43 to 380 steps to the turn) turn where the mirror force has taken
    all of u_par(0)^2, within 5e-4 of the distance travelled (3e-7 to 8e-5
    measured), keep the time-centred energy within 1e-4 (3e-9 to 2e-5), and
    come back.  Without the staggering correction the error would be up to
    2 % (the O(dt) offset of the start)."""
    x_m = _expected_turn()
    xmax, upar_end, dev = _bounce(params(), 1.6 * _turn_steps(UPAR, UPERP))
    err = np.abs(xmax - x_m) / x_m
    assert np.all(err < 5e-4), (xmax, x_m, err)
    assert np.all(dev < 1e-4), dev
    # turned: moving back towards the weaker field
    assert np.all(upar_end < 0.0), upar_end


def test_without_the_option_the_particle_passes_the_mirror_point():
    """The paper's reduced equations (no mirror force): u_par stays constant
    in this field and the particle runs through the mirror point (slowing
    down, as Gamma grows with u_perp^2 = 2 mu B/m)."""
    B0 = 1.0 + GRAD * X0
    u2 = UPAR ** 2 + UPERP ** 2
    x_m = (B0 * u2 / UPERP ** 2 - 1.0) / GRAD - X0
    gam = np.sqrt(1.0 + u2 / 0.45 ** 2)
    xmax, upar_end, _ = _bounce(params(mirror=False), np.ceil(2.0 * x_m * gam / UPAR))
    assert np.all(xmax > 1.3 * x_m), (xmax, x_m)
    assert np.allclose(upar_end, UPAR, rtol=1e-15, atol=0)


def test_gradB_drift_matches_the_relativistic_formula():
    """B = B0 (1 + g x) z_hat, u = u_perp x_hat (u_par = 0): the guiding center
    moves along y at c u_perp^2 B0 g/(2 (q/m) Gamma B^2) per unit time, with
    the sign of q, for non-relativistic to Gamma = 4.6 particles; x and
    u_par stay fixed."""
    B0, g, c = 1.0, 0.05, 0.45
    prov = O.LinearFields([0, 0, 0], np.zeros((3, 2)), [0, 0, B0],
                          [[0, 0], [0, 0], [B0 * g, 0]])
    uperp = [0.05, 0.3, 1.0, 2.0, 0.3]
    qm = [-1.0, -1.0, -1.0, -2.0, 1.0]
    x0, y0, steps = 20.0, 2.0, 50
    st = state(x0, y0, uperp, [0.0] * 5, [0.0] * 5, qm)
    p = params(c=c)
    for _ in range(steps):
        st, S, _ = O.step(prov, st, p)
        assert not bool(S.any())
    up = np.array(uperp)
    Bm = B0 * (1.0 + g * x0)
    gam = np.sqrt(1.0 + up ** 2 / c ** 2)
    v = c * up ** 2 * B0 * g / (2.0 * np.array(qm) * gam * Bm ** 2)
    got = (st.y.numpy() - y0) / steps
    assert np.allclose(got, v, rtol=1e-10, atol=0), (got, v)
    assert np.all(st.x.numpy() == x0)
    assert np.all(st.uz.numpy() == 0.0)
    # without the option: no drift at all (the paper's reduced equations)
    st = state(x0, y0, uperp, [0.0] * 5, [0.0] * 5, qm)
    for _ in range(5):
        st, _, _ = O.step(prov, st, params(c=c, mirror=False))
    assert np.all(st.y.numpy() == y0)


def _general_fields():
    """Uniform-gradient fields with E != 0 and every component varying."""
    rng = np.random.default_rng(5)
    return O.LinearFields([0.02, -0.01, 0.015], 0.002 * rng.standard_normal((3, 2)),
                          [0.3, 0.5, 1.0], 0.01 * rng.standard_normal((3, 2)))


def _random_state(n=64, seed=3):
    rng = np.random.default_rng(seed)
    x = 10.0 + rng.random(n)
    y = 10.0 + rng.random(n)
    u = 0.2 * rng.standard_normal((3, n))
    return O.State(T(*x), T(*y), T(*x), T(*y), T(*u[0]), T(*u[1]), T(*u[2]),
                   torch.full((n,), -30.0, dtype=F64), torch.zeros(n, dtype=torch.uint8))


def test_mirror_terms_vanish_with_mu():
    """mu = 0 (GYR_ZERO): the option changes no bit; with mu conserved it
    changes the paths (the test is not vacuous)."""
    prov = _general_fields()
    a, b = _random_state(), _random_state()
    for _ in range(8):
        a, Sa, _ = O.step(prov, a, params(mirror=True, gyration=O.GYR_ZERO))
        b, Sb, _ = O.step(prov, b, params(mirror=False, gyration=O.GYR_ZERO))
        assert torch.equal(Sa, Sb)
        assert not bool(Sa.all())
    for k in ("x", "y", "xp", "yp", "ux", "uy", "uz", "status"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    a, b = _random_state(), _random_state()
    for _ in range(8):
        a, _, _ = O.step(prov, a, params(mirror=True))
        b, _, _ = O.step(prov, b, params(mirror=False))
    assert not torch.equal(a.x, b.x) and not torch.equal(a.ux, b.ux)


def test_three_dimensions():
    """The 3D step: the grad-B drift with the gradient along z (B = B0 (1 + g z)
    x_hat, b x grad|B| = -B0 g y_hat) and the mirror turn along z
    (B = (1 + g z) z_hat)."""
    c, g = 0.45, 0.05
    base = dict(dt=1.0, c=c, f_rho=0.4, f_E=1.0, curvature=True, n_iter=4,
                Lx=1.0e6, Ly=1.0e6, Lz=1.0e6, dl=1.0, mirror=True)
    p = O.Params3(**base)

    def st3(z, ux, uy, uz, qm):
        n = len(ux)
        x = torch.full((n,), 3.0, dtype=F64)
        y = torch.full((n,), 4.0, dtype=F64)
        zz = torch.full((n,), z, dtype=F64)
        return O.State3(x, y, zz, x.clone(), y.clone(), zz.clone(), T(*ux), T(*uy), T(*uz),
                        T(*qm), torch.zeros(n, dtype=torch.uint8))

    prov = O.LinearFields3([0, 0, 0], np.zeros((3, 3)), [1.0, 0, 0],
                           [[0, 0, g], [0, 0, 0], [0, 0, 0]])
    uperp, qm, z0, steps = [0.3, 1.0], [-1.0, 1.0], 20.0, 40
    st = st3(z0, [0.0, 0.0], [0.0, 0.0], uperp, qm)
    for _ in range(steps):
        st, S, _ = O.step3(prov, st, p)
        assert not bool(S.any())
    up = np.array(uperp)
    Bm = 1.0 + g * z0
    gam = np.sqrt(1.0 + up ** 2 / c ** 2)
    v = -c * up ** 2 * g / (2.0 * np.array(qm) * gam * Bm ** 2)
    assert np.allclose((st.y.numpy() - 4.0) / steps, v, rtol=1e-10, atol=0)
    assert np.all(st.z.numpy() == z0) and np.all(st.x.numpy() == 3.0)

    # the mirror turn along z, u_perp along y
    n = len(UPAR)
    make = lambda: st3(X0, [0.0] * n, list(UPERP), list(UPAR), [-20.0] * n)
    z_m = _expected_turn()
    zmax, upar_end, dev = _bounce(p, 1.6 * _turn_steps(UPAR, UPERP), True, make)
    assert np.all(np.abs(zmax - z_m) / z_m < 5e-4), (zmax, z_m)
    assert np.all(dev < 1e-4), dev
    assert np.all(upar_end < 0.0)


def _ramp3():
    return O.LinearFields3([0, 0, 0], np.zeros((3, 3)), [0, 0, 1.0],
                           [[0, 0, 0], [0, 0, 0], [0, 0, GRAD]])


def test_mirror_check_flags_fast_gyration():
    """The check of the neglect (Params.mirror_tol, ST_MIRROR): in a uniform
    B = z_hat (no drifts, so u_perp_g is the in-plane part of u exactly) a
    guiding-center particle is flagged iff u_perp^2/(Gamma^2 c^2) > tol, with
    Gamma of the full u; the flag is sticky; tol = 0 turns the check off and
    full-orbit particles are never checked.  The cases sit at least 10 %
    from the threshold."""
    c, tol = 0.45, 0.04                     # v_perp_g > 0.2 c
    prov = O.LinearFields([0, 0, 0], np.zeros((3, 2)), [0, 0, 1.0], np.zeros((3, 2)))
    uperp = np.array([0.05, 0.08, 0.12, 0.3, 1.0, 0.3, 2.0])
    upar = np.array([0.0, 0.02, 0.0, 0.5, 3.0, 2.5, 0.0])
    ratio = uperp ** 2 / ((1.0 + (uperp ** 2 + upar ** 2) / c ** 2) * c ** 2)
    want = ratio > tol
    assert np.all(np.abs(ratio / tol - 1.0) > 0.1) and want.any() and not want.all()
    n = len(uperp)
    st = state(3.0, 4.0, list(uperp), [0.0] * n, list(upar), [-20.0] * n)
    for k in range(3):
        st, S, _ = O.step(prov, st, params(mirror=False, mirror_tol=tol, f_rho=1e9))
        assert not bool(S.any())
        got = (st.status.numpy() & O.ST_MIRROR) != 0
        assert np.array_equal(got, want), (k, got, want, ratio)
    st = state(3.0, 4.0, list(uperp), [0.0] * n, list(upar), [-20.0] * n)
    st, _, _ = O.step(prov, st, params(mirror_tol=0.0, f_rho=1e9))
    assert not np.any(st.status.numpy() & O.ST_MIRROR)
    st = state(3.0, 4.0, list(uperp), [0.0] * n, list(upar), [-20.0] * n)
    st, S, _ = O.step(prov, st, params(mirror_tol=tol, f_rho=0.0))
    assert bool(S.all()) and not np.any(st.status.numpy() & O.ST_MIRROR)
    # 3D: the same decision
    p3 = O.Params3(dt=1.0, c=c, f_rho=1e9, f_E=1.0, curvature=True, n_iter=4, Lx=1.0e6,
                   Ly=1.0e6, Lz=1.0e6, dl=1.0, mirror_tol=tol)
    prov3 = O.LinearFields3([0, 0, 0], np.zeros((3, 3)), [0, 0, 1.0], np.zeros((3, 3)))
    x = torch.full((n,), 3.0, dtype=F64)
    s3 = O.State3(x, x + 1, x + 2, x.clone(), x + 1, x + 2, T(*uperp), torch.zeros(n, dtype=F64),
                  T(*upar), torch.full((n,), -20.0, dtype=F64), torch.zeros(n, dtype=torch.uint8))
    s3, S, _ = O.step3(prov3, s3, p3)
    assert np.array_equal((s3.status.numpy() & O.ST_MIRROR) != 0, want)


def test_check_does_not_change_the_orbit():
    """The check only sets a status bit: with and without mirror_tol the
    states agree bit for bit (flat space with E != 0, and curved spacetime on
    the small magnetosphere), and a particle flagged at a threshold is flagged
    at every smaller one."""
    prov = _general_fields()
    runs = {}
    for tol in (0.0, 1e-3, 1e-2):
        st = _random_state(n=200, seed=7)
        for _ in range(6):
            st, _, _ = O.step(prov, st, params(mirror_tol=tol))
        runs[tol] = st
    for k in ("x", "y", "xp", "yp", "ux", "uy", "uz"):
        assert torch.equal(getattr(runs[0.0], k), getattr(runs[1e-2], k)), k
    f3, f2 = ((runs[t].status.numpy() & O.ST_MIRROR) != 0 for t in (1e-3, 1e-2))
    assert not np.any(f2 & ~f3) and f3.any() and not (runs[0.0].status.numpy() & O.ST_MIRROR).any()

    from oracle import gr
    from workloads.gr import make_gr_config
    cfg = make_gr_config("grbh64")
    F = cfg.fields()
    e = cfg.particles(n=400, seed_offset=3)
    out = {}
    for tol in (0.0, 0.01, 0.1):
        p = gr.GRParams(dt=cfg.dt, f_rho=cfg.f_rho, f_E=cfg.f_E, n_iter=cfg.n_iter, mirror_tol=tol)
        out[tol], _, _ = gr.push(gr.KerrSchild(cfg.a), gr.GRGrid(F, cfg.r_min, cfg.r_max),
                                 gr.GRState.from_numpy(e), p, 5)
    for k in ("r", "th", "ph", "ur", "uth", "uph"):
        assert torch.equal(getattr(out[0.0], k), getattr(out[0.1], k)), k
    g1, g2 = ((out[t].status.numpy() & gr.ST_MIRROR) != 0 for t in (0.01, 0.1))
    assert not np.any(g2 & ~g1) and g1.any()
    assert not (out[0.0].status.numpy() & gr.ST_MIRROR).any()
