"""Pin of the oracle gradient (reverse-mode autograd of the oracle push)
against central finite differences of the oracle forward push.  No GPU.

The loss is the mean final kinetic energy.  A finite-difference pair whose
switch trace differs from the base run crosses a switch boundary, where the
loss is not differentiable; such samples are skipped (the switch is held
fixed along the forward path).
"""
import numpy as np
import pytest
import torch

import oracle as O
from workloads import make_config, make_config3

F64 = torch.float64


def _setup(n=24, steps=6, seed_offset=3, curvature=True):
    cfg = make_config("harris64")
    F = cfg.fields()
    ens = cfg.particles(n=n, seed_offset=seed_offset)
    st0 = O.State.from_numpy(ens)
    p = O.Params(dt=cfg.dt, c=cfg.c, f_rho=cfg.f_rho, f_E=cfg.f_E,
                 curvature=curvature, n_iter=cfg.n_iter, Lx=cfg.Lx, Ly=cfg.Ly,
                 dl=1.0)
    return cfg, F, st0, p, steps


def _loss(cfg, F, st0, p, steps):
    prov = O.GridFields(torch.as_tensor(F), cfg.dx, cfg.dy, cfg.stagger)
    out, tr, _ = O.push(prov, st0.clone(), p, steps, trace=True)
    return float(O.kinetic_energy(out.ux, out.uy, out.uz, p.c)), tr


@pytest.mark.parametrize("curvature", [True, False])
def test_oracle_gradient_matches_central_differences(curvature):
    cfg, F, st0, p, steps = _setup(curvature=curvature)
    g = O.push_gradients(F, cfg.dx, cfg.dy, cfg.stagger, st0, p, steps)
    tr0 = g["trace"]
    # both regimes are exercised
    assert 0 < int(tr0.sum()) < tr0.numel()
    rng = np.random.default_rng(11)
    checked = 0

    def fd(perturb, h):
        s_plus, s_minus = perturb(+h), perturb(-h)
        lp, tp = _loss(cfg, *s_plus, p, steps)
        lm, tm = _loss(cfg, *s_minus, p, steps)
        if not (torch.equal(tp, tr0) and torch.equal(tm, tr0)):
            return None
        return (lp - lm) / (2 * h)

    # initial four-velocities and positions
    for name in ("ux", "uy", "uz", "x", "y"):
        for i in rng.choice(st0.x.shape[0], 4, replace=False):
            base = float(getattr(st0, name)[i])
            h = 1e-6 * max(1.0, abs(base))

            def perturb(d, name=name, i=i):
                s = st0.clone()
                getattr(s, name)[i] += d
                return F, s
            v = fd(perturb, h)
            if v is None:
                continue
            a = float(g["d" + name][i])
            assert abs(a - v) <= 1e-6 * max(abs(v), 1e-4 * abs(g["loss"])) + 1e-10, (name, i, a, v)
            checked += 1
    # grid nodes with a non-negligible gradient
    dF = g["dF"].abs().flatten()
    cand = torch.nonzero(dF > 1e-3 * dF.max()).flatten().numpy()
    for flat in rng.choice(cand, 16, replace=False):
        k, j, i = np.unravel_index(flat, F.shape)
        h = 1e-6

        def perturb(d, k=k, j=j, i=i):
            Fp = F.copy()
            Fp[k, j, i] += d
            return Fp, st0.clone()
        v = fd(perturb, h)
        if v is None:
            continue
        a = float(g["dF"][k, j, i])
        assert abs(a - v) <= 1e-6 * abs(v) + 1e-10, (k, j, i, a, v)
        checked += 1
    assert checked >= 20


def test_oracle_gradient3_matches_central_differences():
    """The 3D push (harris3d32, curvature on): autograd of the oracle against
    central differences of its forward on initial positions, four-velocities
    and grid nodes of all six components, both regimes present."""
    cfg = make_config3("harris3d32")
    F = cfg.fields()
    ens = cfg.particles(n=24, seed_offset=5)
    st0 = O.State3.from_numpy(ens)
    p = O.Params3(dt=cfg.dt, c=cfg.c, f_rho=cfg.f_rho, f_E=cfg.f_E, curvature=True,
                  n_iter=cfg.n_iter, Lx=cfg.Lx, Ly=cfg.Ly, Lz=cfg.Lz, dl=cfg.dl)
    steps = 5
    g = O.push_gradients3(F, cfg.dx, cfg.dy, cfg.dz, cfg.stagger, st0, p, steps)
    tr0 = g["trace"]
    assert 0 < int(tr0.sum()) < tr0.numel()

    def loss(Fp, s):
        prov = O.GridFields3(torch.as_tensor(Fp), cfg.dx, cfg.dy, cfg.dz, cfg.stagger)
        out, tr, _ = O.push3(prov, s, p, steps, trace=True)
        return float(O.kinetic_energy(out.ux, out.uy, out.uz, p.c)), tr

    def fd(perturb, h):
        (lp, tp), (lm, tm) = loss(*perturb(+h)), loss(*perturb(-h))
        if not (torch.equal(tp, tr0) and torch.equal(tm, tr0)):
            return None
        return (lp - lm) / (2 * h)

    rng = np.random.default_rng(13)
    checked = 0
    for name in ("ux", "uy", "uz", "x", "y", "z"):
        for i in rng.choice(st0.x.shape[0], 3, replace=False):
            base = float(getattr(st0, name)[i])

            def perturb(d, name=name, i=i):
                s = st0.clone()
                getattr(s, name)[i] += d
                return F, s
            v = fd(perturb, 1e-6 * max(1.0, abs(base)))
            if v is None:
                continue
            a = float(g["d" + name][i])
            assert abs(a - v) <= 1e-6 * max(abs(v), 1e-4 * abs(g["loss"])) + 1e-10, (name, i, a, v)
            checked += 1
    dF = g["dF"].abs().flatten()
    for comp in range(6):
        sub = g["dF"][comp].abs().flatten()
        cand = torch.nonzero(sub > 1e-3 * dF.max()).flatten().numpy()
        for flat in rng.choice(cand, min(2, len(cand)), replace=False):
            l, j, i = np.unravel_index(flat, F.shape[1:])

            def perturb(d, comp=comp, l=l, j=j, i=i):
                Fp = F.copy()
                Fp[comp, l, j, i] += d
                return Fp, st0.clone()
            v = fd(perturb, 1e-6)
            if v is None:
                continue
            a = float(g["dF"][comp, l, j, i])
            assert abs(a - v) <= 1e-6 * abs(v) + 1e-10, (comp, l, j, i, a, v)
            checked += 1
    assert checked >= 20


def test_kinetic_energy_closed_form():
    c = 0.5
    ux = torch.tensor([0.0, 0.5 * np.sqrt(3.0)], dtype=F64)   # Gamma = 1, 2
    z = torch.zeros(2, dtype=F64)
    assert abs(float(O.kinetic_energy(ux, z, z, c)) - 0.5 * (0.0 + 1.0) * c * c) < 1e-16
