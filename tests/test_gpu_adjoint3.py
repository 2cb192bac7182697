"""Hand-written 3D adjoint (gcb_push_backward_3d, GcbPush3 autograd) against
the oracle gradient of the 3D push (needs an MI355X).

Tolerances as for 2D: state cotangents are binary64 recurrences in another
order than the oracle's autograd (1e-8 of the largest entry per array); field
cotangents are accumulated in binary32 with atomics (2e-5 of the largest
entry)."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import log
from workloads import make_config3

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NAMES3 = ("x", "y", "z", "xp", "yp", "zp", "ux", "uy", "uz")


def _grad_gpu3(cfg, F, ens, steps, checkpoint, curvature=1):
    from paper_2007_14401_amd import autograd as A, gcb
    pctx = A.PushContext3(0, (cfg.dx, cfg.dy, cfg.dz), cfg.stagger)
    try:
        Ft = torch.as_tensor(F, dtype=torch.float64, device=DEV)
        E = Ft[:3].contiguous().requires_grad_(True)
        B = Ft[3:].contiguous().requires_grad_(True)
        st = {k: torch.as_tensor(np.ascontiguousarray(getattr(ens, k)), dtype=torch.float64,
                                 device=DEV).requires_grad_(True) for k in NAMES3}
        qm = torch.as_tensor(ens.qm, dtype=torch.float64, device=DEV)
        prm = gcb.params(dt=cfg.dt, c=cfg.c, qm=cfg.qm, f_rho=cfg.f_rho, f_E=cfg.f_E,
                         curvature=curvature, n_iter=cfg.n_iter)
        out = A.push3(E, B, *[st[k] for k in NAMES3], qm, pctx, prm, steps, checkpoint)
        L = A.kinetic_energy(out[6], out[7], out[8], pctx, prm)
        L.backward()
        torch.cuda.synchronize()
        g = {k: st[k].grad.cpu().numpy() for k in NAMES3}
        gF = torch.cat([E.grad, B.grad]).cpu().numpy()
        return float(L), g, gF
    finally:
        pctx.close()


@pytest.mark.parametrize("curvature", [1, 0])
def test_adjoint3_matches_oracle_gradient(curvature):
    cfg = make_config3("harris3d32", curvature=curvature)
    F = cfg.fields()
    ens = cfg.particles(n=300, seed_offset=31)
    steps = 12
    log(f"3d adjoint curvature={curvature}: gpu")
    Lg, g, gF = _grad_gpu3(cfg, F, ens, steps, 5, curvature)
    log("3d adjoint: oracle")
    st0 = O.State3.from_numpy(ens)
    p = O.Params3(dt=cfg.dt, c=cfg.c, f_rho=cfg.f_rho, f_E=cfg.f_E, curvature=bool(curvature),
                  n_iter=cfg.n_iter, Lx=cfg.Lx, Ly=cfg.Ly, Lz=cfg.Lz, dl=cfg.dl)
    ref = O.push_gradients3(F, cfg.dx, cfg.dy, cfg.dz, cfg.stagger, st0, p, steps)
    assert abs(Lg - ref["loss"]) <= 1e-12 * abs(ref["loss"])
    tr = ref["trace"]
    assert 0 < int(tr.sum()) < tr.numel()
    for k in NAMES3:
        a, b = g[k], ref["d" + k].numpy()
        err = np.max(np.abs(a - b)) / np.max(np.abs(b))
        log(f"3d curv={curvature} d{k}: max-norm rel err {err:.2e}")
        assert err <= 1e-8, (k, err)
    b = ref["dF"].numpy()
    err = np.max(np.abs(gF - b)) / np.max(np.abs(b))
    log(f"3d curv={curvature} dF: max-norm rel err {err:.2e}")
    assert err <= 2e-5


def test_adjoint3_recomputation_kernels_agree():
    """gcb_push_backward_3d recomputes a segment with the in-place tiled push
    (sort_every > 0 and a window that fits) or one launch of the global
    kernel per step (sort_every = 0); both run the parity arithmetic, so the
    state cotangents are equal bit for bit and the binary32 field cotangents
    to their accumulation order."""
    from paper_2007_14401_amd import gcb, state
    cfg = make_config3("harris3d32")
    F = cfg.fields()
    ens = cfg.particles(n=800 + 13, seed_offset=41)
    steps = 9
    ctx = gcb.gcb_create(0)
    try:
        desc = gcb.grid3_desc(cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, cfg.dz, cfg.stagger,
                              gcb.GCB_F64)
        gcb.gcb_load_fields_3d(ctx, desc, [F[0], F[1], F[2]], [F[3], F[4], F[5]])
        t = state.to_device(ens, DEV, with_id=False)
        rng = np.random.default_rng(3)
        lam_end = [torch.as_tensor(rng.normal(size=ens.n), device=DEV) for _ in range(9)]
        shape = (3, cfg.nz, cfg.ny, cfg.nx)
        out = {}
        for se, tile in ((0, 0), (4, 4), (3, 6)):
            log(f"3d backward recomputation sort_every={se} tile={tile}")
            lam = [torch.empty(ens.n, dtype=torch.float64, device=DEV) for _ in range(9)]
            dE = torch.zeros(shape, dtype=torch.float32, device=DEV)
            dB = torch.zeros(shape, dtype=torch.float32, device=DEV)
            prm = gcb.params(dt=cfg.dt, c=cfg.c, qm=cfg.qm, f_rho=cfg.f_rho, f_E=cfg.f_E,
                             curvature=cfg.curvature, n_iter=cfg.n_iter, sort_every=se,
                             tile=tile)
            gcb.gcb_push_backward_3d(ctx, gcb.particles3(t), prm, steps, lam_end, lam,
                                     [dE[0], dE[1], dE[2]], [dB[0], dB[1], dB[2]])
            torch.cuda.synchronize()
            out[se] = ([v.cpu().numpy() for v in lam], torch.cat([dE, dB]).cpu().numpy())
        base_l, base_f = out[0]
        for se in (4, 3):
            lam_s, f = out[se]
            for a, b in zip(lam_s, base_l):
                assert np.array_equal(a, b), se
            assert np.max(np.abs(f - base_f)) <= 1e-5 * np.max(np.abs(base_f)), se
    finally:
        gcb.gcb_destroy(ctx)


def test_adjoint3_checkpoint_segments_do_not_change_gradients():
    cfg = make_config3("harris3d32")
    F = cfg.fields()
    ens = cfg.particles(n=200, seed_offset=32)
    _, g1, f1 = _grad_gpu3(cfg, F, ens, 10, 10)
    _, g2, f2 = _grad_gpu3(cfg, F, ens, 10, 3)
    for k in NAMES3:
        assert np.array_equal(g1[k], g2[k]), k
    assert np.max(np.abs(f1 - f2)) <= 1e-6 * np.max(np.abs(f1))


def test_adjoint3_argument_checks():
    from paper_2007_14401_amd import gcb
    cfg = make_config3("harris3d32")
    F = cfg.fields()
    ctx = gcb.gcb_create(0)
    try:
        n = 16
        ens = cfg.particles(n=n)
        t = {k: torch.as_tensor(np.ascontiguousarray(getattr(ens, k)), dtype=torch.float64,
                                device=DEV) for k in NAMES3}
        t["status"] = torch.zeros(n, dtype=torch.uint8, device=DEV)
        lam = [torch.zeros(n, dtype=torch.float64, device=DEV) for _ in range(9)]
        out = [torch.zeros(n, dtype=torch.float64, device=DEV) for _ in range(9)]
        grid = [torch.zeros((cfg.nz, cfg.ny, cfg.nx), dtype=torch.float32, device=DEV)
                for _ in range(6)]
        with pytest.raises(gcb.GcbError) as e:
            gcb.gcb_push_backward_3d(ctx, gcb.particles3(t), gcb.params(), 1, lam, out,
                                     grid[:3], grid[3:])
        assert e.value.code == gcb.GCB_ENOFIELDS
        desc = gcb.grid3_desc(cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, cfg.dz, cfg.stagger,
                              gcb.GCB_F64)
        gcb.gcb_load_fields_3d(ctx, desc, [F[0], F[1], F[2]], [F[3], F[4], F[5]])
        for bad in (dict(gyration=1), dict(frame=1, curvature=0), dict(n_iter=9),
                    dict(mirror=1)):
            with pytest.raises(gcb.GcbError) as e:
                gcb.gcb_push_backward_3d(ctx, gcb.particles3(t), gcb.params(**bad), 1, lam,
                                         out, grid[:3], grid[3:])
            assert e.value.code == gcb.GCB_EUNSUPPORTED, bad
        # zero steps: lam_start = lam_end, grids untouched
        lam[6].fill_(0.25)
        gcb.gcb_push_backward_3d(ctx, gcb.particles3(t), gcb.params(), 0, lam, out, grid[:3],
                                 grid[3:])
        torch.cuda.synchronize()
        assert torch.equal(out[6], lam[6])
        assert all(float(gr.abs().max()) == 0.0 for gr in grid)
        # no particles: nothing to do, grids untouched
        t0 = {k: v[:0] for k, v in t.items()}
        gcb.gcb_push_backward_3d(ctx, gcb.particles3(t0), gcb.params(), 3,
                                 [v[:0] for v in lam], [v[:0] for v in out], grid[:3], grid[3:])
        torch.cuda.synchronize()
        assert all(float(gr.abs().max()) == 0.0 for gr in grid)
    finally:
        gcb.gcb_destroy(ctx)
