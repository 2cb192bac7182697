"""Hand-written adjoint (gcb_push_backward, GcbPush autograd) against the
oracle gradient and against central finite differences of the GPU forward.

Tolerances (from the arithmetic):
  * state cotangents are binary64 recurrences evaluated in a different order
    than the oracle's autograd: relative agreement 1e-8 (max norm per array)
    after tens of steps;
  * field cotangents are accumulated in binary32 (atomic adds of binary64
    contributions rounded to binary32): agreement 2e-5 of the largest entry;
  * finite differences (full-size differentiation workload): central
    differences of the binary64 forward with the switch decisions replayed
    from the base run, h = 1e-6 (1e-9 for grid nodes) relative, formed from
    the per-particle kinetic-energy differences KE_p(+h) - KE_p(-h) summed
    over particles (the mean over 1e6 particles would bury a single particle's
    change in the rounding of the total); samples whose difference quotient
    changes by more than 1e-3 when h is divided by 10 (outside the linear
    regime of a chaotic orbit) are discarded; the rest must agree with the
    adjoint to 1e-3.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import log, oracle_params
from workloads import make_config

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NAMES = ("x", "y", "xp", "yp", "ux", "uy", "uz")


def _tensors(ens):
    return {k: torch.as_tensor(np.ascontiguousarray(getattr(ens, k)), dtype=torch.float64,
                               device=DEV) for k in NAMES}


def _fields(F):
    t = torch.as_tensor(F, dtype=torch.float64, device=DEV)
    return t[:3].contiguous(), t[3:].contiguous()


def _grad_gpu(cfg, F, ens, steps, checkpoint, curvature=1):
    from paper_2007_14401_amd import autograd as A, gcb
    pctx = A.PushContext(0)
    try:
        E, B = _fields(F)
        E.requires_grad_(True)
        B.requires_grad_(True)
        st = _tensors(ens)
        for k in NAMES:
            st[k].requires_grad_(True)
        qm = torch.as_tensor(ens.qm, dtype=torch.float64, device=DEV)
        prm = gcb.params(dt=cfg.dt, c=cfg.c, qm=cfg.qm, f_rho=cfg.f_rho, f_E=cfg.f_E,
                         curvature=curvature, n_iter=cfg.n_iter)
        out = A.push(E, B, *[st[k] for k in NAMES], qm, pctx, prm, steps, checkpoint)
        L = A.kinetic_energy(out[4], out[5], out[6], pctx, prm)
        L.backward()
        torch.cuda.synchronize()
        g = {k: st[k].grad.cpu().numpy() for k in NAMES}
        gF = torch.cat([E.grad, B.grad]).cpu().numpy()
        return float(L), g, gF
    finally:
        pctx.close()


@pytest.mark.parametrize("curvature", [1, 0])
def test_adjoint_matches_oracle_gradient(curvature):
    cfg = make_config("harris64", curvature=curvature)
    F = cfg.fields()
    ens = cfg.particles(n=400, seed_offset=21)
    steps = 24
    Lg, g, gF = _grad_gpu(cfg, F, ens, steps, 8, curvature)
    st0 = O.State.from_numpy(ens)
    ref = O.push_gradients(F, cfg.dx, cfg.dy, cfg.stagger, st0, oracle_params(cfg), steps)
    assert abs(Lg - ref["loss"]) <= 1e-12 * abs(ref["loss"])
    tr = ref["trace"]
    assert 0 < int(tr.sum()) < tr.numel()
    for k in NAMES:
        a, b = g[k], ref["d" + k].numpy()
        err = np.max(np.abs(a - b)) / np.max(np.abs(b))
        log(f"curv={curvature} d{k}: max-norm rel err {err:.2e}")
        assert err <= 1e-8, (k, err)
    b = ref["dF"].numpy()
    err = np.max(np.abs(gF - b)) / np.max(np.abs(b))
    log(f"curv={curvature} dF: max-norm rel err {err:.2e}")
    assert err <= 2e-5


def test_adjoint_on_a_narrow_grid_matches_oracle():
    """On a 32 x 64 grid the backward's tile order of the particles (32-cell
    tiles) has a single column of tiles; the gradients, mapped back to the
    caller's particle order, still match the oracle's."""
    cfg = make_config("harris64", nx=32)
    F = cfg.fields()
    ens = cfg.particles(n=300, seed_offset=22)
    steps = 16
    Lg, g, gF = _grad_gpu(cfg, F, ens, steps, 8)
    st0 = O.State.from_numpy(ens)
    ref = O.push_gradients(F, cfg.dx, cfg.dy, cfg.stagger, st0, oracle_params(cfg), steps)
    assert abs(Lg - ref["loss"]) <= 1e-12 * abs(ref["loss"])
    for k in NAMES:
        a, b = g[k], ref["d" + k].numpy()
        err = np.max(np.abs(a - b)) / np.max(np.abs(b))
        log(f"32x64 d{k}: max-norm rel err {err:.2e}")
        assert err <= 1e-8, (k, err)
    b = ref["dF"].numpy()
    err = np.max(np.abs(gF - b)) / np.max(np.abs(b))
    log(f"32x64 dF: max-norm rel err {err:.2e}")
    assert err <= 2e-5


def _oracle_jvp(cfg, F, ens, steps, vF, vs):
    """J v of the oracle's multi-step push (final state over the initial state
    and the field grid) along the direction (vF, vs), by torch autograd's
    forward-over-reverse product (the switch decisions carry no derivative,
    as in the adjoint)."""
    p = oracle_params(cfg)
    qm = torch.as_tensor(ens.qm, dtype=torch.float64)

    def f(Ft, *s0):
        st = O.State(*s0, qm=qm, status=torch.zeros(ens.n, dtype=torch.uint8))
        prov = O.GridFields(Ft, cfg.dx, cfg.dy, cfg.stagger)
        out, _, _ = O.push(prov, st, p, steps)
        return tuple(getattr(out, k) for k in NAMES)

    inputs = (torch.as_tensor(F, dtype=torch.float64),) + tuple(
        torch.as_tensor(np.ascontiguousarray(getattr(ens, k)), dtype=torch.float64)
        for k in NAMES)
    v = (torch.as_tensor(vF),) + tuple(torch.as_tensor(vs[k]) for k in NAMES)
    _, Jv = torch.autograd.functional.jvp(f, inputs, v)
    return {k: j.numpy() for k, j in zip(NAMES, Jv)}


def test_adjoint_dot_product():
    """<J v, w> = <v, J^T w> for random dense directions: J v from the
    oracle's forward-mode product, J^T w from the GPU adjoint (the cotangent w
    of every final state component seeded through the autograd function).
    The state part agrees to the binary64 rounding of the two recurrences
    (measured 2.5e-17 of sum |v_i (J^T w)_i|), the field part to the binary32
    accumulation of the field cotangents (measured 6.2e-10)."""
    from paper_2007_14401_amd import autograd as A, gcb
    cfg = make_config("harris64")
    F = cfg.fields()
    ens = cfg.particles(n=240, seed_offset=31)
    steps = 10
    rng = np.random.default_rng(5)
    w = {k: rng.normal(size=ens.n) for k in NAMES}
    # the GPU adjoint: J^T w for the initial state and the fields
    pctx = A.PushContext(0)
    try:
        E, B = _fields(F)
        E.requires_grad_(True)
        B.requires_grad_(True)
        st = {k: v.requires_grad_(True) for k, v in _tensors(ens).items()}
        qm = torch.as_tensor(ens.qm, dtype=torch.float64, device=DEV)
        prm = gcb.params(dt=cfg.dt, c=cfg.c, qm=cfg.qm, f_rho=cfg.f_rho, f_E=cfg.f_E,
                         curvature=cfg.curvature, n_iter=cfg.n_iter)
        out = A.push(E, B, *[st[k] for k in NAMES], qm, pctx, prm, steps, 4)
        s = sum(torch.sum(o * torch.as_tensor(w[k], device=DEV)) for k, o in zip(NAMES, out))
        s.backward()
        torch.cuda.synchronize()
        gs = {k: st[k].grad.cpu().numpy() for k in NAMES}
        gF = torch.cat([E.grad, B.grad]).cpu().numpy()
    finally:
        pctx.close()
    for part in ("state", "fields"):
        vs = {k: (rng.normal(size=ens.n) if part == "state" else np.zeros(ens.n))
              for k in NAMES}
        vF = rng.normal(size=F.shape) if part == "fields" else np.zeros(F.shape)
        Jv = _oracle_jvp(cfg, F, ens, steps, vF, vs)
        lhs = sum(float(np.dot(Jv[k], w[k])) for k in NAMES)
        terms = [vs[k] * gs[k] for k in NAMES] + [(vF * gF).ravel()]
        rhs = float(sum(np.sum(t) for t in terms))
        scale = float(sum(np.sum(np.abs(t)) for t in terms))
        rel = abs(lhs - rhs) / scale
        log(f"dot product ({part}): <Jv, w> = {lhs:.15e}, <v, J^T w> = {rhs:.15e}, "
            f"difference / sum|v J^T w| = {rel:.2e}")
        assert rel <= (1e-14 if part == "state" else 1e-8), (part, lhs, rhs, rel)


def test_checkpoint_segments_do_not_change_gradients():
    cfg = make_config("harris64")
    F = cfg.fields()
    ens = cfg.particles(n=300, seed_offset=4)
    _, g1, f1 = _grad_gpu(cfg, F, ens, 20, 20)
    _, g2, f2 = _grad_gpu(cfg, F, ens, 20, 3)
    for k in NAMES:
        assert np.array_equal(g1[k], g2[k]), k
    assert np.max(np.abs(f1 - f2)) <= 1e-6 * np.max(np.abs(f1))


def test_backward_after_second_forward_on_shared_context():
    """Two forwards on one PushContext (the second with perturbed fields, as
    in a finite-difference pair), then the backward of the first: its
    gradients equal those of a run on a context of its own, bit for bit."""
    from paper_2007_14401_amd import autograd as A, gcb
    cfg = make_config("harris64")
    F = cfg.fields()
    ens = cfg.particles(n=300, seed_offset=6)
    steps = 10
    _, g_ref, f_ref = _grad_gpu(cfg, F, ens, steps, 4)
    pctx = A.PushContext(0)
    try:
        prm = gcb.params(dt=cfg.dt, c=cfg.c, qm=cfg.qm, f_rho=cfg.f_rho, f_E=cfg.f_E,
                         curvature=cfg.curvature, n_iter=cfg.n_iter)
        qm = torch.as_tensor(ens.qm, dtype=torch.float64, device=DEV)

        def forward(scale):
            E, B = _fields(F)
            E = (E * scale).requires_grad_(True)
            B = (B * scale).requires_grad_(True)
            st = {k: v.requires_grad_(True) for k, v in _tensors(ens).items()}
            out = A.push(E, B, *[st[k] for k in NAMES], qm, pctx, prm, steps, 4)
            return E, B, st, A.kinetic_energy(out[4], out[5], out[6], pctx, prm)

        E1, B1, st1, L1 = forward(1.0)
        forward(1.001)          # replaces the fields held by the context
        L1.backward()
        torch.cuda.synchronize()
        for k in NAMES:
            assert np.array_equal(st1[k].grad.cpu().numpy(), g_ref[k]), k
        gF = torch.cat([E1.grad, B1.grad]).cpu().numpy()
        assert np.max(np.abs(gF - f_ref)) <= 1e-6 * np.max(np.abs(f_ref))
    finally:
        pctx.close()


def _c4_fd(steps, n_nodes, n_u, node_h, min_nodes, min_u):
    """Central differences of the push with replayed switch decisions against
    the adjoint on the differentiation workload (1024^2 grid, 1e6 particles)."""
    from paper_2007_14401_amd import gcb
    cfg = make_config("harris1024")
    log(f"c4 ({steps} steps): inputs")
    F = cfg.fields()
    ens = cfg.particles()
    n = ens.n
    log(f"c4 ({steps} steps): adjoint")
    L0, g, gF = _grad_gpu(cfg, F, ens, steps, 32)

    ctx = gcb.gcb_create(0)
    desc = gcb.grid_desc(cfg.nx, cfg.ny, cfg.dx, cfg.dy, cfg.stagger, gcb.GCB_F64)
    kw = dict(dt=cfg.dt, c=cfg.c, qm=cfg.qm, f_rho=cfg.f_rho, f_E=cfg.f_E,
              curvature=cfg.curvature, n_iter=cfg.n_iter)
    prm = gcb.params(**kw)
    prm_replay = gcb.params(replay=1, **kw)
    qm = torch.as_tensor(ens.qm, dtype=torch.float64, device=DEV)
    base = _tensors(ens)
    trace = torch.empty((steps, n), dtype=torch.uint8, device=DEV)
    out = torch.zeros(1, dtype=torch.float64, device=DEV)
    inv_c2 = 1.0 / (cfg.c * cfg.c)

    def ke_vec(st):
        u2 = (st["ux"] * st["ux"] + st["uy"] * st["uy"]) + st["uz"] * st["uz"]
        return (torch.sqrt(1.0 + u2 * inv_c2) - 1.0) * (cfg.c * cfg.c)

    def loss(Fp, pert=None, replay=True):
        gcb.gcb_load_fields(ctx, desc, [Fp[0], Fp[1], Fp[2]], [Fp[3], Fp[4], Fp[5]])
        st = {k: v.clone() for k, v in base.items()}
        if pert is not None:
            k, i, d = pert
            st[k][i] += d
        st["status"] = torch.zeros(n, dtype=torch.uint8, device=DEV)
        st["qm"] = qm
        st["id"] = None
        parts = gcb.particles(st)
        gcb.gcb_push(ctx, parts, prm_replay if replay else prm, steps, s_trace=trace)
        gcb.gcb_kinetic_energy(ctx, parts, prm, out)
        torch.cuda.synchronize()
        return float(out), ke_vec(st)

    try:
        Lb, _ = loss(F, replay=False)       # records the decisions in `trace`
        Lr, _ = loss(F)
        assert Lr == Lb                        # replaying them reproduces the run
        assert abs(Lb - L0) <= 1e-13 * abs(L0)
        rng = np.random.default_rng(99)
        checked = {"node": 0, "u": 0}
        skipped = {"node": 0, "u": 0}

        def fd(mk, h):
            (_, kp), (_, km) = mk(+h), mk(-h)
            return float(torch.sum(kp - km)) / n / (2 * h)

        def judge(kind, adj, mk, h):
            v = fd(mk, h)
            if abs(v - adj) <= 1e-3 * abs(adj):
                checked[kind] += 1
                return
            v2 = fd(mk, h / 10)
            if abs(v2 - v) > 1e-3 * abs(v):
                skipped[kind] += 1     # outside the linear regime
                return
            raise AssertionError((kind, adj, v, v2))

        flat = np.abs(gF).reshape(-1)
        cand = np.nonzero(flat > 1e-4 * flat.max())[0]
        for fl in rng.choice(cand, n_nodes, replace=False):
            k, j, i = np.unravel_index(fl, F.shape)

            def mk(d, k=k, j=j, i=i):
                Fp = F.copy()
                Fp[k, j, i] += d
                return loss(Fp)
            judge("node", float(gF[k, j, i]), mk, node_h * max(1.0, abs(F[k, j, i])))
        gcb.gcb_load_fields(ctx, desc, [F[0], F[1], F[2]], [F[3], F[4], F[5]])
        for p in rng.choice(n, n_u, replace=False):
            comp = ("ux", "uy", "uz")[int(rng.integers(3))]
            u = float(getattr(ens, comp)[p])

            def mk(d, comp=comp, p=p):
                return loss(F, (comp, int(p), d))
            judge("u", float(g[comp][p]), mk, 1e-6 * max(cfg.c, abs(u)))
        log(f"c4 ({steps} steps) finite differences: checked {checked}, "
            f"outside the linear regime {skipped}")
        assert checked["node"] >= min_nodes and checked["u"] >= min_u
    finally:
        gcb.gcb_destroy(ctx)


def test_c4_finite_differences_full_horizon():
    """512 steps (checkpoint every 32): 64 initial four-velocity components
    (at least 48 inside the linear regime of their orbits)."""
    _c4_fd(512, 0, 64, 1e-6, 0, 48)


def test_c4_finite_differences_grid_nodes():
    """Grid-node cotangents at full size over one checkpoint segment (32
    steps): over 512 steps a node perturbation reaches hundreds of particle-
    steps on chaotic orbits, and the guiding-center map is discontinuous in
    position (the bilinear gradient of B jumps across cell lines), so almost
    every difference quotient leaves the linear regime."""
    _c4_fd(32, 64, 0, 1e-7, 48, 0)


def test_recomputation_kernels_agree():
    """gcb_push_backward recomputes a segment with the in-place tiled push
    (sort_every > 0) or the global kernel (sort_every = 0); both run the
    parity arithmetic, so the state cotangents are equal bit for bit and the
    binary32 field cotangents to their accumulation order."""
    from paper_2007_14401_amd import gcb
    cfg = make_config("harris64")
    F = cfg.fields()
    ens = cfg.particles(n=1000 + 13, seed_offset=41)
    steps = 12
    ctx = gcb.gcb_create(0)
    try:
        desc = gcb.grid_desc(cfg.nx, cfg.ny, cfg.dx, cfg.dy, cfg.stagger, gcb.GCB_F64)
        gcb.gcb_load_fields(ctx, desc, [F[0], F[1], F[2]], [F[3], F[4], F[5]])
        st = _tensors(ens)
        st["status"] = torch.zeros(ens.n, dtype=torch.uint8, device=DEV)
        st["qm"] = torch.as_tensor(ens.qm, dtype=torch.float64, device=DEV)
        st["id"] = None
        rng = np.random.default_rng(3)
        lam_end = [torch.as_tensor(rng.normal(size=ens.n), device=DEV) for _ in range(7)]
        out = {}
        for se, tile in ((0, 0), (4, 16), (3, 8)):
            lam = [torch.empty(ens.n, dtype=torch.float64, device=DEV) for _ in range(7)]
            dE = torch.zeros((3, cfg.ny, cfg.nx), dtype=torch.float32, device=DEV)
            dB = torch.zeros((3, cfg.ny, cfg.nx), dtype=torch.float32, device=DEV)
            prm = gcb.params(dt=cfg.dt, c=cfg.c, qm=cfg.qm, f_rho=cfg.f_rho, f_E=cfg.f_E,
                             curvature=cfg.curvature, n_iter=cfg.n_iter, sort_every=se,
                             tile=tile)
            gcb.gcb_push_backward(ctx, gcb.particles(st), prm, steps, lam_end, lam,
                                  [dE[0], dE[1], dE[2]], [dB[0], dB[1], dB[2]])
            torch.cuda.synchronize()
            out[se] = ([v.cpu().numpy() for v in lam], torch.cat([dE, dB]).cpu().numpy())
        base_l, base_f = out[0]
        for se in (4, 3):
            l, f = out[se]
            for a, b in zip(l, base_l):
                assert np.array_equal(a, b), se
            assert np.max(np.abs(f - base_f)) <= 1e-5 * np.max(np.abs(base_f)), se
    finally:
        gcb.gcb_destroy(ctx)
