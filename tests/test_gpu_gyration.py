"""Parity of the gyration options of the guiding-center step (Sec. 2.2:
u_perp_g held over the step, or mu = 0, instead of a conserved mu; and the
gyration phase advanced over the step, the extra equation Sec. 3.1 allows)
with the oracle (needs an MI355X).  Bar: the binary64 path of the parity tests,
1e-12 relative with identical switch decisions and status bits (bit for bit
expected); the mixed form to the bounds of its one-step test."""
import numpy as np
import pytest
import torch

from gpu_util import GpuRun, log, rel_errors, run_oracle
from test_gpu_3d import GpuRun3, _check as _check3, _state as _state3, run_oracle3
from workloads import make_config, make_config3

pytestmark = pytest.mark.gpu

TOL = 1e-12
UPERP, ZERO, PHASE = 1, 2, 3


def _check(got, ref, cfg, what, tr_gpu, tr_ref):
    errs = rel_errors(got, ref, cfg)
    log(f"{what}: max rel err {max(errs.values()):.2e}")
    for k, v in errs.items():
        assert v <= TOL, (what, k, v)
    assert np.array_equal(got["status"] & ~np.uint8(32), ref.status.numpy()), what
    assert np.count_nonzero(tr_gpu.cpu().numpy() != tr_ref.numpy()) == 0, what


@pytest.fixture(scope="module")
def h64():
    cfg = make_config("harris64")
    F = cfg.fields()
    run = GpuRun(cfg, F)
    yield cfg, F, run
    run.close()


@pytest.mark.parametrize("gyr", [UPERP, ZERO, PHASE])
@pytest.mark.parametrize("kernel,sort_every,tile,steps", [(1, 0, 0, 1), (2, 1, 16, 1),
                                                          (1, 0, 0, 20), (2, 3, 24, 20)])
def test_gyration_parity(h64, gyr, kernel, sort_every, tile, steps):
    """Curvature scheme (Sec. 2.2.2) on the Harris sheet; tile 24 leaves a
    ragged last tile on the 64-cell grid."""
    from paper_2007_14401_amd import state
    cfg, F, run = h64
    ens = cfg.particles(n=4096 + 37, seed_offset=5)
    log(f"gyration={gyr} kernel={kernel} sort_every={sort_every} tile={tile} steps={steps}")
    t = state.to_device(ens, "cuda:0")
    tr, st = run.push(t, steps, trace=True, stats=True, kernel=kernel, sort_every=sort_every,
                      tile=tile, gyration=gyr)
    ref, rtr, rres = run_oracle(cfg, F, ens, steps, trace=True, gyration=gyr)
    _check(state.unsort(t), ref, cfg, f"gyration {gyr}", tr, rtr)
    assert st["gca_steps"] == int((rtr == 0).sum()) > 0
    assert st["max_fp_residual"] == float(rres.max())


def test_gyration_with_exact_frame(h64):
    """The held u_perp_g with the exact frame and the zero-curvature scheme."""
    from paper_2007_14401_amd import gcb, state
    cfg, F, run = h64
    ens = cfg.particles(n=3000, seed_offset=6)
    log("gyration=1 exact frame, tiled, 12 steps")
    t = state.to_device(ens, "cuda:0")
    tr, _ = run.push(t, 12, trace=True, kernel=2, sort_every=2, tile=16, curvature=0,
                     frame=gcb.GCB_FRAME_EXACT, gyration=UPERP)
    ref, rtr, _ = run_oracle(cfg, F, ens, 12, trace=True, curvature=False, exact_frame=True,
                             gyration=UPERP)
    _check(state.unsort(t), ref, cfg, "gyration 1 exact frame", tr, rtr)


def test_gyration_options_differ(h64):
    """Sanity of the option itself: on the Harris sheet the three options
    give different orbits (the oracle's pins decide which is which)."""
    from paper_2007_14401_amd import state
    cfg, F, run = h64
    ens = cfg.particles(n=2000, seed_offset=7)
    out = []
    for gyr in (0, UPERP, ZERO, PHASE):
        t = state.to_device(ens, "cuda:0")
        run.push(t, 10, kernel=1, gyration=gyr)
        out.append(state.unsort(t))
    for a, b in ((0, 1), (0, 2), (1, 2), (0, 3)):
        assert np.abs(out[a]["ux"] - out[b]["ux"]).max() > 1e-9, (a, b)


@pytest.mark.parametrize("gyr", [UPERP, ZERO, PHASE])
@pytest.mark.parametrize("kernel,sort_every,tile,steps", [(1, 0, 0, 1), (2, 2, 6, 12)])
def test_gyration_parity_3d(gyr, kernel, sort_every, tile, steps):
    cfg = make_config3("harris3d32")
    F = cfg.fields()
    run = GpuRun3(cfg, F)
    try:
        ens = cfg.particles(n=3000, seed_offset=8)
        log(f"3d gyration={gyr} kernel={kernel} steps={steps}")
        t = _state3(ens)
        tr, st = run.push(t, steps, trace=True, stats=True, kernel=kernel,
                          sort_every=sort_every, tile=tile, gyration=gyr)
        from paper_2007_14401_amd import state
        ref, rtr, _ = run_oracle3(cfg, F, ens, steps, trace=True, gyration=gyr)
        _check3(state.unsort(t), ref, cfg, f"3d gyration {gyr}", tr, rtr)
        assert st["gca_steps"] > 0
    finally:
        run.close()


@pytest.mark.parametrize("gyr", [UPERP, ZERO, PHASE])
def test_gyration_mixed_one_step(gyr):
    """Mixed form against the binary64 oracle with the same option, one
    step, both kernels: the bounds of the mixed form's one-step test."""
    from paper_2007_14401_amd import gcb, state
    cfg = make_config("harris64")
    F = cfg.fields()
    ens = cfg.particles(n=8192, seed_offset=9)
    run = GpuRun(cfg, F, dtype=gcb.GCB_F32)
    try:
        for kernel, se, tile in ((1, 0, 0), (2, 1, 16)):
            log(f"mixed gyration={gyr} kernel={kernel}")
            t = state.to_device(ens, "cuda:0", form=gcb.GCB_FORM_MIXED)
            tr, _ = run.push(t, 1, trace=True, form=gcb.GCB_FORM_MIXED, kernel=kernel,
                             sort_every=se, tile=tile, gyration=gyr)
            got = state.unsort(t)
            ref, rtr, _ = run_oracle(cfg, F, ens, 1, trace=True, gyration=gyr)
            u_g = np.stack([got[k].astype(np.float64) for k in ("ux", "uy", "uz")])
            u_r = np.stack([getattr(ref, k).numpy() for k in ("ux", "uy", "uz")])
            du = np.max(np.abs(u_g - u_r), axis=0) / np.maximum(np.max(np.abs(u_r), axis=0),
                                                                 cfg.c)
            dx = np.max(np.stack([np.minimum(np.abs(got[k] - getattr(ref, k).numpy()),
                                             L - np.abs(got[k] - getattr(ref, k).numpy()))
                                  for k, L in (("x", cfg.Lx), ("y", cfg.Ly))]), axis=0)
            mism = float((tr.cpu().numpy() != rtr.numpy()).mean())
            log(f"  u median {np.median(du):.2e} p99 {np.quantile(du, 0.99):.2e}; "
                f"x max {dx.max():.2e}; S mismatch {mism:.2e}")
            assert np.median(du) <= 1e-5
            assert np.quantile(du, 0.99) <= 1e-3
            assert dx.max() <= 1e-4
            assert mism <= 2e-3
    finally:
        run.close()


def test_gyration_argument_checks(h64):
    """Unknown values are invalid; the adjoint serves mu conserved only."""
    from paper_2007_14401_amd import gcb, state
    cfg, F, run = h64
    t = state.to_device(cfg.particles(n=64), "cuda:0")
    with pytest.raises(gcb.GcbError) as e:
        gcb.gcb_push(run.ctx, gcb.particles(t), gcb.params(gyration=4), 1)
    assert e.value.code == gcb.GCB_EINVAL
    # the phase option goes with the reduced frame and without the mirror terms
    for kw in (dict(curvature=0, frame=gcb.GCB_FRAME_EXACT), dict(mirror=1)):
        with pytest.raises(gcb.GcbError) as e:
            gcb.gcb_push(run.ctx, gcb.particles(t), gcb.params(gyration=PHASE, **kw), 1)
        assert e.value.code == gcb.GCB_EUNSUPPORTED, kw
    with pytest.raises(gcb.GcbError) as e:
        gcb.gcb_push(run.ctx, gcb.particles(t), gcb.params(gyration=-1), 1)
    assert e.value.code == gcb.GCB_EINVAL
    n = 64
    lam = [torch.zeros(n, dtype=torch.float64, device="cuda:0") for _ in range(7)]
    lam0 = [torch.zeros(n, dtype=torch.float64, device="cuda:0") for _ in range(7)]
    grid = [torch.zeros((cfg.ny, cfg.nx), dtype=torch.float32, device="cuda:0")
            for _ in range(6)]
    with pytest.raises(gcb.GcbError) as e:
        gcb.gcb_push_backward(run.ctx, gcb.particles(t), gcb.params(gyration=UPERP), 1, lam,
                              lam0, grid[:3], grid[3:])
    assert e.value.code == gcb.GCB_EUNSUPPORTED


@pytest.mark.parametrize("kernel,sort_every,tile", [(1, 0, 0), (2, 1, 16)])
def test_gyration_phase_production_one_step(h64, kernel, sort_every, tile):
    """The phase option in the production binary64 build (GCB_ARITH_FAST):
    one step within 1e-12 of the oracle, identical switch decisions."""
    from paper_2007_14401_amd import state
    cfg, F, run = h64
    ens = cfg.particles(n=4096 + 37, seed_offset=10)
    t = state.to_device(ens, "cuda:0")
    tr, _ = run.push(t, 1, trace=True, kernel=kernel, sort_every=sort_every, tile=tile,
                     gyration=PHASE, arith=1)
    ref, rtr, _ = run_oracle(cfg, F, ens, 1, trace=True, gyration=PHASE)
    _check(state.unsort(t), ref, cfg, "gyration phase, production build", tr, rtr)
