"""Parity of the mirror option (gcb_params.mirror: the mirror force and the
grad-B drift that Sec. 2.2 names and leaves out, added to the curvature
scheme of Sec. 2.2.2) with the oracle (needs an MI355X).  Bar: the binary64
path of the parity tests, 1e-12 relative with identical switch decisions
and status bits (bit for bit expected); the mixed form to the bounds of its
one-step test."""
import numpy as np
import pytest
import torch

from gpu_util import GpuRun, log, run_oracle
from test_gpu_3d import GpuRun3, _check as _check3, _state as _state3, run_oracle3
from test_gpu_gyration import _check
from workloads import make_config, make_config3

pytestmark = pytest.mark.gpu

UPERP = 1
TOL_CHECK = 1e-3   # (v_perp_g/c)^2 threshold of the check of the neglect
ST_MIRROR = 128


@pytest.fixture(scope="module")
def h64():
    cfg = make_config("harris64")
    F = cfg.fields()
    run = GpuRun(cfg, F)
    yield cfg, F, run
    run.close()


@pytest.mark.parametrize("kernel,sort_every,tile,steps", [(1, 0, 0, 1), (2, 1, 16, 1),
                                                          (1, 0, 0, 20), (2, 3, 24, 20)])
def test_mirror_parity(h64, kernel, sort_every, tile, steps):
    """Harris sheet, mu conserved; tile 24 leaves a ragged last tile on the
    64-cell grid.  The check of the neglect (mirror_tol) runs alongside: its
    status bit is part of the bitwise status comparison and of the
    histogram."""
    from paper_2007_14401_amd import gcb, state
    cfg, F, run = h64
    ens = cfg.particles(n=4096 + 37, seed_offset=15)
    log(f"mirror kernel={kernel} sort_every={sort_every} tile={tile} steps={steps}")
    t = state.to_device(ens, "cuda:0")
    tr, st = run.push(t, steps, trace=True, stats=True, kernel=kernel, sort_every=sort_every,
                      tile=tile, mirror=1, mirror_tol=TOL_CHECK)
    ref, rtr, rres = run_oracle(cfg, F, ens, steps, trace=True, mirror=True,
                                mirror_tol=TOL_CHECK)
    _check(state.unsort(t), ref, cfg, "mirror", tr, rtr)
    assert st["gca_steps"] == int((rtr == 0).sum()) > 0
    assert st["max_fp_residual"] == float(rres.max())
    flagged = int(((ref.status.numpy() & gcb.GCB_ST_MIRROR) != 0).sum())
    assert st["status_counts"][7] == flagged
    log(f"  mirror check: {flagged} of {ens.n} particles above (v_perp_g/c)^2 = {TOL_CHECK}")
    assert 0 < flagged < ens.n


@pytest.mark.parametrize("kernel,sort_every,tile", [(1, 0, 0), (2, 2, 24)])
def test_mirror_check_on_the_reduced_equations(h64, kernel, sort_every, tile):
    """The check of the neglect on the paper's own equations (mirror = 0),
    binary64, 10 steps: status bits bit for bit with the oracle."""
    from paper_2007_14401_amd import gcb, state
    cfg, F, run = h64
    ens = cfg.particles(n=4096 + 11, seed_offset=20)
    t = state.to_device(ens, "cuda:0")
    tr, st = run.push(t, 10, trace=True, stats=True, kernel=kernel, sort_every=sort_every,
                      tile=tile, mirror_tol=TOL_CHECK)
    ref, rtr, _ = run_oracle(cfg, F, ens, 10, trace=True, mirror_tol=TOL_CHECK)
    _check(state.unsort(t), ref, cfg, "mirror check", tr, rtr)
    flagged = int(((ref.status.numpy() & gcb.GCB_ST_MIRROR) != 0).sum())
    assert st["status_counts"][7] == flagged and 0 < flagged < ens.n


def test_mirror_with_held_uperp(h64):
    """The option with the other gyration handling (u_perp_g held)."""
    from paper_2007_14401_amd import state
    cfg, F, run = h64
    ens = cfg.particles(n=3000, seed_offset=16)
    log("mirror with gyration=1, tiled, 12 steps")
    t = state.to_device(ens, "cuda:0")
    tr, _ = run.push(t, 12, trace=True, kernel=2, sort_every=2, tile=16, mirror=1,
                     gyration=UPERP)
    ref, rtr, _ = run_oracle(cfg, F, ens, 12, trace=True, mirror=True, gyration=UPERP)
    _check(state.unsort(t), ref, cfg, "mirror gyration 1", tr, rtr)


def test_mirror_changes_the_orbits(h64):
    """The option is not a no-op on the Harris sheet."""
    from paper_2007_14401_amd import state
    cfg, F, run = h64
    ens = cfg.particles(n=2000, seed_offset=17)
    out = []
    for m in (0, 1):
        t = state.to_device(ens, "cuda:0")
        run.push(t, 10, kernel=1, mirror=m)
        out.append(state.unsort(t))
    assert np.abs(out[0]["ux"] - out[1]["ux"]).max() > 1e-9
    assert np.abs(out[0]["x"] - out[1]["x"]).max() > 1e-9


@pytest.mark.parametrize("kernel,sort_every,tile,steps", [(1, 0, 0, 1), (2, 2, 6, 12)])
def test_mirror_parity_3d(kernel, sort_every, tile, steps):
    from paper_2007_14401_amd import state
    cfg = make_config3("harris3d32")
    F = cfg.fields()
    run = GpuRun3(cfg, F)
    try:
        ens = cfg.particles(n=3000, seed_offset=18)
        log(f"3d mirror kernel={kernel} steps={steps}")
        t = _state3(ens)
        tr, st = run.push(t, steps, trace=True, stats=True, kernel=kernel,
                          sort_every=sort_every, tile=tile, mirror=1, mirror_tol=TOL_CHECK)
        ref, rtr, _ = run_oracle3(cfg, F, ens, steps, trace=True, mirror=True,
                                  mirror_tol=TOL_CHECK)
        _check3(state.unsort(t), ref, cfg, "3d mirror", tr, rtr)
        assert st["gca_steps"] > 0
    finally:
        run.close()


def _split_tol(run):
    """A mirror_tol that the oracle's one step flags for between 5 % and 95 %
    of the particles (run(tol) returns the oracle's state)."""
    for tol in (1e-4, 1e-3, 1e-2, 0.03, 0.1, 0.3):
        frac = float(((run(tol).status.numpy() & ST_MIRROR) != 0).mean())
        if 0.05 < frac < 0.95:
            log(f"mirror_tol {tol}: oracle flags {frac:.3f}")
            return tol
    raise AssertionError("no threshold splits the particles")


def _check_mirror_bits(got, ref, tol):
    """ST_MIRROR of the mixed form against the binary64 oracle: near the
    threshold the mixed form repeats the comparison in binary64, so the bits
    agree but for particles whose binary32 inputs moved them across it."""
    a = (got["status"] & ST_MIRROR) != 0
    b = (ref.status.numpy() & ST_MIRROR) != 0
    mism = float((a != b).mean())
    log(f"  ST_MIRROR at tol {tol}: {int(b.sum())} flagged by the oracle, mismatch {mism:.2e}")
    assert mism <= 1e-3


def test_mirror_mixed_one_step():
    """Mixed form against the binary64 oracle with the option, one step,
    both kernels: the bounds of the mixed form's one-step test."""
    from paper_2007_14401_amd import gcb, state
    cfg = make_config("harris64")
    F = cfg.fields()
    ens = cfg.particles(n=8192, seed_offset=19)
    run = GpuRun(cfg, F, dtype=gcb.GCB_F32)
    try:
        tol = _split_tol(lambda m: run_oracle(cfg, F, ens, 1, mirror=True, mirror_tol=m)[0])
        ref, rtr, _ = run_oracle(cfg, F, ens, 1, trace=True, mirror=True, mirror_tol=tol)
        for kernel, se, tile in ((1, 0, 0), (2, 1, 16)):
            log(f"mixed mirror kernel={kernel}")
            t = state.to_device(ens, "cuda:0", form=gcb.GCB_FORM_MIXED)
            tr, _ = run.push(t, 1, trace=True, form=gcb.GCB_FORM_MIXED, kernel=kernel,
                             sort_every=se, tile=tile, mirror=1, mirror_tol=tol)
            got = state.unsort(t)
            _check_mirror_bits(got, ref, tol)
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


def test_mirror_argument_checks(h64):
    """Values other than 0 and 1 are invalid; the option needs the curvature
    scheme; the adjoints and the curved-spacetime push refuse it."""
    from paper_2007_14401_amd import gcb, state
    cfg, F, run = h64
    t = state.to_device(cfg.particles(n=64), "cuda:0")
    for bad, code in ((dict(mirror=2), gcb.GCB_EINVAL), (dict(mirror=-1), gcb.GCB_EINVAL),
                      (dict(mirror_tol=-1e-3), gcb.GCB_EINVAL),
                      (dict(mirror_tol=float("nan")), gcb.GCB_EINVAL),
                      (dict(mirror=1, curvature=0), gcb.GCB_EUNSUPPORTED),
                      (dict(mirror=1, curvature=0, frame=gcb.GCB_FRAME_EXACT),
                       gcb.GCB_EUNSUPPORTED)):
        with pytest.raises(gcb.GcbError) as e:
            gcb.gcb_push(run.ctx, gcb.particles(t), gcb.params(**bad), 1)
        assert e.value.code == code, bad
    n = 64
    lam = [torch.zeros(n, dtype=torch.float64, device="cuda:0") for _ in range(7)]
    lam0 = [torch.zeros(n, dtype=torch.float64, device="cuda:0") for _ in range(7)]
    grid = [torch.zeros((cfg.ny, cfg.nx), dtype=torch.float32, device="cuda:0")
            for _ in range(6)]
    for opt in (dict(mirror=1), dict(mirror_tol=1e-3)):
        with pytest.raises(gcb.GcbError) as e:
            gcb.gcb_push_backward(run.ctx, gcb.particles(t), gcb.params(**opt), 1, lam, lam0,
                                  grid[:3], grid[3:])
        assert e.value.code == gcb.GCB_EUNSUPPORTED, opt
    z = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    g = {"r": z + 5.0, "th": z + 1.0, "ph": z.clone(), "ur": z.clone(), "uth": z.clone(),
         "uph": z.clone(), "status": torch.zeros(n, dtype=torch.uint8, device="cuda:0")}
    with pytest.raises(gcb.GcbError) as e:
        gcb.gcb_push_gr(run.ctx, gcb.gr_particles(g), gcb.params(mirror=1), 1)
    assert e.value.code == gcb.GCB_EUNSUPPORTED


@pytest.mark.parametrize("kernel,sort_every,tile", [(1, 0, 0), (2, 1, 6)])
def test_mirror_mixed_one_step_3d(kernel, sort_every, tile):
    """The 3D mixed form with the option against the binary64 oracle with it,
    one step: the bounds of the mixed form's one-step test."""
    from paper_2007_14401_amd import gcb, state
    cfg = make_config3("harris3d32")
    F = cfg.fields()
    ens = cfg.particles(n=8192, seed_offset=21)
    run = GpuRun3(cfg, F, dtype=gcb.GCB_F32)
    tol = _split_tol(lambda m: run_oracle3(cfg, F, ens, 1, mirror=True, mirror_tol=m)[0])
    try:
        t = state.to_device(ens, "cuda:0", form=gcb.GCB_FORM_MIXED)
        tr, _ = run.push(t, 1, trace=True, form=gcb.GCB_FORM_MIXED, kernel=kernel,
                         sort_every=sort_every, tile=tile, mirror=1, mirror_tol=tol)
    finally:
        run.close()
    got = state.unsort(t)
    ref, rtr, _ = run_oracle3(cfg, F, ens, 1, trace=True, mirror=True, mirror_tol=tol)
    _check_mirror_bits(got, ref, tol)
    u_g = np.stack([got[k].astype(np.float64) for k in ("ux", "uy", "uz")])
    u_r = np.stack([getattr(ref, k).numpy() for k in ("ux", "uy", "uz")])
    du = np.max(np.abs(u_g - u_r), axis=0) / np.maximum(np.max(np.abs(u_r), axis=0), cfg.c)
    dx = np.max(np.stack([np.minimum(np.abs(got[k] - getattr(ref, k).numpy()),
                                     L - np.abs(got[k] - getattr(ref, k).numpy()))
                          for k, L in (("x", cfg.Lx), ("y", cfg.Ly), ("z", cfg.Lz))]), axis=0)
    mism = float((tr.cpu().numpy() != rtr.numpy()).mean())
    log(f"3d mixed mirror kernel={kernel}: u median {np.median(du):.2e} "
        f"p99 {np.quantile(du, 0.99):.2e}; x max {dx.max():.2e}; S mismatch {mism:.2e}")
    assert np.median(du) <= 1e-5
    assert np.quantile(du, 0.99) <= 1e-3
    assert dx.max() <= 1e-4
    assert mism <= 2e-3
