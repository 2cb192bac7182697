"""Parity of the exact-frame option (Sec. 2.2: b*, exact v_E and kappa,
du_par/dt = (q/m) E'/kappa; zero-curvature scheme) with the oracle (needs an
MI355X).  Bar: the binary64 path of the parity tests, 1e-12 relative with
identical switch decisions and status bits (bit-for-bit expected)."""
import numpy as np
import pytest

from gpu_util import GpuRun, log, rel_errors, run_oracle
from workloads import make_config

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _check(got, ref, cfg, what, tr_gpu, tr_ref):
    errs = rel_errors(got, ref, cfg)
    log(f"{what}: max rel err {max(errs.values()):.2e}")
    for k, v in errs.items():
        assert v <= TOL, (what, k, v)
    assert np.array_equal(got["status"] & ~np.uint8(32), ref.status.numpy()), what
    assert np.count_nonzero(tr_gpu.cpu().numpy() != tr_ref.numpy()) == 0, what


@pytest.fixture(scope="module")
def strong():
    """harris64 with a stronger reconnection field and guide field: E.B up to
    about 0.15 B0^2 around the X points (E.B = E_z B_z there)."""
    cfg = make_config("harris64", E_rec=0.5, guide=0.3, curvature=0)
    F = cfg.fields()
    run = GpuRun(cfg, F)
    yield cfg, F, run
    run.close()


@pytest.mark.parametrize("kernel,sort_every,tile,steps", [(1, 0, 0, 1), (2, 1, 16, 1),
                                                          (1, 0, 0, 20), (2, 3, 16, 20)])
def test_exact_frame_parity(strong, kernel, sort_every, tile, steps):
    from paper_2007_14401_amd import gcb, state
    cfg, F, run = strong
    ens = cfg.particles(n=4096 + 37)
    log(f"exact frame kernel={kernel} sort_every={sort_every} steps={steps}")
    t = state.to_device(ens, "cuda:0")
    tr, st = run.push(t, steps, trace=True, stats=True, kernel=kernel, sort_every=sort_every,
                      tile=tile, frame=gcb.GCB_FRAME_EXACT, curvature=0)
    ref, rtr, rres = run_oracle(cfg, F, ens, steps, trace=True, exact_frame=True)
    _check(state.unsort(t), ref, cfg, "exact frame", tr, rtr)
    assert st["gca_steps"] == int((rtr == 0).sum()) > 0
    assert st["max_fp_residual"] == float(rres.max())


def test_exact_frame_differs_from_reduced_where_E_dot_B(strong):
    """Sanity of the option itself: with E.B != 0 somewhere the two frames
    give different orbits (the oracle decides which is right; its pins fix
    the exact frame against a resolved orbit)."""
    from paper_2007_14401_amd import gcb, state
    cfg, F, run = strong
    ens = cfg.particles(n=2000, seed_offset=3)
    out = []
    for frame in (gcb.GCB_FRAME_REDUCED, gcb.GCB_FRAME_EXACT):
        t = state.to_device(ens, "cuda:0")
        run.push(t, 10, kernel=1, frame=frame, curvature=0)
        out.append(state.unsort(t))
    d = np.abs(out[0]["ux"] - out[1]["ux"])
    assert d.max() > 1e-6


def test_exact_frame_argument_checks(strong):
    from paper_2007_14401_amd import gcb, state
    cfg, F, run = strong
    t = state.to_device(cfg.particles(n=64), "cuda:0")
    with pytest.raises(gcb.GcbError) as e:
        gcb.gcb_push(run.ctx, gcb.particles(t), gcb.params(frame=gcb.GCB_FRAME_EXACT,
                                                           curvature=1), 1)
    assert e.value.code == gcb.GCB_EUNSUPPORTED
    with pytest.raises(gcb.GcbError) as e:
        gcb.gcb_push(run.ctx, gcb.particles(t), gcb.params(frame=7), 1)
    assert e.value.code == gcb.GCB_EINVAL
    tm = state.to_device(cfg.particles(n=64), "cuda:0", form=gcb.GCB_FORM_MIXED)
    with pytest.raises(gcb.GcbError) as e:
        gcb.gcb_push(run.ctx, gcb.particles(tm), gcb.params(frame=gcb.GCB_FRAME_EXACT,
                                                            curvature=0,
                                                            form=gcb.GCB_FORM_MIXED), 1)
    assert e.value.code == gcb.GCB_EUNSUPPORTED
