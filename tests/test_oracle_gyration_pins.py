"""Pins of the oracle's gyration options of the guiding-center step (Sec. 2.2)
against what the paper states of them: the magnetic moment is an adiabatic
invariant under eq. dmudt; holding u_perp_g fixed instead conserves the
energy exactly when E = 0 and the curvature terms vanish; mu = 0 discards
the gyration.  No GPU.

The field: B = (1 + g x) x_hat, E = 0.  Its direction is uniform, so b = x_hat
exactly, the curvature terms and v_E vanish and u_par cannot change, while
|B| grows along the guiding-center path: the three options then separate in
closed form.  (b_x = B_x (1/|B|) may differ from 1 by an ulp, hence the
tolerances of order 1e-15 on u_par.)"""
import numpy as np
import pytest
import torch

import oracle as O

F64 = torch.float64
GRAD = 0.05


def T(*v):
    return torch.tensor(v, dtype=F64)


def params(**kw):
    base = dict(dt=1.0, c=0.45, f_rho=0.4, f_E=1.0, curvature=True, n_iter=4,
                Lx=1.0e6, Ly=1.0e6, dl=1.0)
    base.update(kw)
    return O.Params(**base)


def state(ux, uy, uz, qm=-20.0, x=20.0, y=2.0):
    n = len(ux)
    x = torch.full((n,), x, dtype=F64)
    y = torch.full((n,), y, dtype=F64)
    return O.State(x, y, x.clone(), y.clone(), T(*ux), T(*uy), T(*uz),
                   torch.full((n,), qm, dtype=F64), torch.zeros(n, dtype=torch.uint8))


def ramp():
    return O.LinearFields([0, 0, 0], np.zeros((3, 2)), [1.0, 0, 0], [[GRAD, 0], [0, 0], [0, 0]])


def run(prov, st, p, n):
    traj = [st]
    for _ in range(n):
        st, S, _ = O.step(prov, st, p)
        assert not bool(S.any()), "the pins need guiding-center steps throughout"
        traj.append(st)
    return traj


def _perp2(st):
    return (st.uy * st.uy + st.uz * st.uz).numpy()


U0 = ([0.3, -0.2, 0.1], [0.2, 0.05, -0.3], [0.1, 0.3, 0.0])   # u_x (= u_par), u_y, u_z


@pytest.mark.parametrize("curv", [True, False])
def test_mu_is_conserved_and_u_perp_follows_B(curv):
    """Eq. dmudt: u_perp_g^2 = 2 mu B/m at every reconstruction point
    R^{n+1/2} = (x^n + x^{n+1})/2, with mu fixed by the first decomposition;
    u_par is untouched (E = 0, no curvature terms in this field), so the
    energy grows with |B| (the paper's remark on dropping the mirror force)."""
    p = params(curvature=curv, gyration=O.GYR_MU)
    traj = run(ramp(), state(*U0), p, 60)
    mu = None
    for a, b in zip(traj[:-1], traj[1:]):
        assert np.allclose(b.ux.numpy(), traj[0].ux.numpy(), rtol=1e-15, atol=0)
        Bm = 1.0 + GRAD * (0.5 * (a.x + b.x)).numpy()
        m = _perp2(b) / (2.0 * Bm)
        mu = m if mu is None else mu
        assert np.allclose(m, mu, rtol=1e-13, atol=0)
    # and the first mu is the one of the initial perpendicular four-velocity
    # at the first decomposition point x^0
    B0 = 1.0 + GRAD * traj[0].x.numpy()
    assert np.allclose(mu, _perp2(traj[0]) / (2.0 * B0), rtol=1e-14)
    # the energy follows |B| at the last reconstruction point (not conserved)
    g0 = np.sqrt(1 + (traj[0].ux ** 2 + traj[0].uy ** 2 + traj[0].uz ** 2).numpy() / p.c2)
    g1 = np.sqrt(1 + (traj[-1].ux ** 2 + traj[-1].uy ** 2 + traj[-1].uz ** 2).numpy() / p.c2)
    Bl = 1.0 + GRAD * (0.5 * (traj[-2].x + traj[-1].x)).numpy()
    want = np.sqrt(1 + ((traj[0].ux ** 2).numpy() + 2.0 * mu * Bl) / p.c2)
    assert np.allclose(g1, want, rtol=1e-13)
    assert np.all(np.abs(g1 - g0) > 1e-3 * g0)


@pytest.mark.parametrize("curv", [True, False])
def test_fixed_u_perp_conserves_energy_exactly(curv):
    """The alternative to eq. dmudt: u_perp_g held at its decomposed value
    keeps |u|, hence Gamma, constant up to rounding, and the guiding center
    then moves at the constant speed u_par/Gamma along b."""
    p = params(curvature=curv, gyration=O.GYR_UPERP)
    traj = run(ramp(), state(*U0), p, 60)
    st0 = traj[0]
    p2 = _perp2(st0)
    gam = np.sqrt(1 + ((st0.ux ** 2).numpy() + p2) / p.c2)
    for k, st in enumerate(traj[1:], start=1):
        assert np.allclose(st.ux.numpy(), st0.ux.numpy(), rtol=1e-15, atol=0)
        assert np.allclose(_perp2(st), p2, rtol=1e-13, atol=0)
        want = st0.x.numpy() + k * p.dt * st0.ux.numpy() / gam
        assert np.allclose(st.x.numpy(), want, rtol=1e-13, atol=0)
        assert torch.equal(st.y, st0.y)


def test_zero_mu_discards_the_gyration():
    """mu = 0: after one guiding-center step u = u_par b exactly (E = 0)."""
    p = params(gyration=O.GYR_ZERO)
    traj = run(ramp(), state(*U0), p, 5)
    for st in traj[1:]:
        assert np.allclose(st.ux.numpy(), traj[0].ux.numpy(), rtol=1e-15, atol=0)
        assert torch.all(st.uy == 0.0) and torch.all(st.uz == 0.0)


def test_options_coincide_without_gyration():
    """A particle with u = u_par b has u_perp_g = 0 (up to the rounding of
    u - (u.b) b) under every option: in a curved field without E and
    curvature terms the three agree to rounding over many steps."""
    prov = O.CircularFields(1.0, 500.0, 500.0, Bz=0.3)
    # u along b at the start point (503, 500): B = (0, 1, 0.3) there
    b = np.array([0.0, 1.0, 0.3]) / np.hypot(1.0, 0.3)
    u = 0.25 * b
    outs = []
    for g in (O.GYR_MU, O.GYR_UPERP, O.GYR_ZERO):
        st = state([u[0]], [u[1]], [u[2]], x=503.0, y=500.0)
        outs.append(run(prov, st, params(gyration=g, curvature=False), 30)[-1])
    for o in outs[1:]:
        for k in ("x", "y", "ux", "uy", "uz"):
            assert np.allclose(getattr(o, k).numpy(), getattr(outs[0], k).numpy(),
                               rtol=1e-13, atol=1e-15), k


def test_uniform_field_options_agree():
    """Uniform |B| (and E): conserved mu and held u_perp_g are the same
    physics; they differ by rounding only."""
    prov = O.UniformFields([0.01, -0.02, 0.0], [0.3, -0.2, 0.9])
    res = []
    for g in (O.GYR_MU, O.GYR_UPERP):
        st = state([0.1], [-0.2], [0.15])
        res.append(run(prov, st, params(gyration=g), 40)[-1])
    for k in ("x", "y", "ux", "uy", "uz"):
        assert np.allclose(getattr(res[0], k).numpy(), getattr(res[1], k).numpy(),
                           rtol=1e-13, atol=1e-15), k


def test_options_in_three_dimensions():
    """The 3D step uses the same options: in B = (1 + g z) z_hat, held
    u_perp_g keeps |u| (and u_z = u_par) and mu = 0 leaves u = u_par b."""
    prov = O.LinearFields3([0, 0, 0], np.zeros((3, 3)), [0, 0, 1.0],
                           [[0, 0, 0], [0, 0, 0], [0, 0, GRAD]])

    def st3(ux, uy, uz):
        x = T(1.0, 1.0, 1.0)
        return O.State3(x, x + 1, x + 19, x.clone(), x + 1, x + 19, T(*ux), T(*uy), T(*uz),
                        torch.full((3,), -20.0, dtype=F64), torch.zeros(3, dtype=torch.uint8))

    base = dict(dt=1.0, c=0.45, f_rho=0.4, f_E=1.0, curvature=True, n_iter=4,
                Lx=1.0e6, Ly=1.0e6, Lz=1.0e6, dl=1.0)
    ux, uy, uz = U0[1], U0[2], U0[0]     # u_par along z
    s0 = st3(ux, uy, uz)
    p = O.Params3(**base, gyration=O.GYR_UPERP)
    st = s0
    for _ in range(30):
        st, S, _ = O.step3(prov, st, p)
        assert not bool(S.any())
        assert np.allclose(st.uz.numpy(), s0.uz.numpy(), rtol=1e-15, atol=0)
        assert np.allclose((st.ux ** 2 + st.uy ** 2).numpy(), (s0.ux ** 2 + s0.uy ** 2).numpy(),
                           rtol=1e-13, atol=0)
    p = O.Params3(**base, gyration=O.GYR_ZERO)
    st, S, _ = O.step3(prov, s0, p)
    assert torch.all(st.ux == 0.0) and torch.all(st.uy == 0.0)
    assert np.allclose(st.uz.numpy(), s0.uz.numpy(), rtol=1e-15, atol=0)
    p = O.Params3(**base, gyration=O.GYR_MU)
    st = s0
    for _ in range(30):
        stn, S, _ = O.step3(prov, st, p)
        Bm = 1.0 + GRAD * (0.5 * (st.z + stn.z)).numpy()
        mu = (stn.ux ** 2 + stn.uy ** 2).numpy() / (2.0 * Bm)
        B0 = 1.0 + GRAD * s0.z.numpy()
        assert np.allclose(mu, (s0.ux ** 2 + s0.uy ** 2).numpy() / (2.0 * B0), rtol=1e-13)
        st = stn
