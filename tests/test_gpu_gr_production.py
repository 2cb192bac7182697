"""The production arithmetic of the curved-spacetime binary64 push
(GCB_ARITH_FAST: contracted multiply-adds, shared reciprocals in the metric,
reciprocal square roots for square roots that serve as divisors) against the
binary64 oracle (needs an MI355X), by the chaos-aware protocol:

  * one step from identical states: 1e-12 relative (floors: 1 for the
    angles, c = 1 for u; phi compared modulo 2 pi), identical switch
    decisions and status bits for every particle;
  * many steps: a production step differs from the exact one by a few units
    in the last place, and an orbit amplifies such differences by its own
    sensitivity.  That sensitivity is measured on the oracle itself: the
    oracle run again with every particle's position and four-velocity moved
    by up to four units in the last place after every step (a random whole
    number in [-4, 4] per value, three independent runs).  Per particle the
    GPU error must stay within max(1e-12, 10 x the largest oracle deviation),
    and every particle whose oracle deviation stays within 1e-12 must also
    keep every switch decision of the oracle.
"""
import math

import numpy as np
import pytest
import torch

from gpu_util import log
from oracle import gr
from test_gpu_gr import DEV, NAMES, GrRun, run_oracle, to_device
from workloads import make_gr_config

pytestmark = pytest.mark.gpu

TOL = 1e-12
FAST = 1
ULPS = 4
FLOOR = {"r": 1.0, "th": 1.0, "ph": 1.0, "ur": 1.0, "uth": 1.0, "uph": 1.0}


def particle_errors(got, ref):
    """Per-particle max relative error over r, theta, phi (modulo 2 pi) and u."""
    err = None
    for k in NAMES:
        a = np.asarray(got[k], dtype=np.float64)
        b = np.asarray(getattr(ref, k).numpy() if hasattr(ref, k) else ref[k], dtype=np.float64)
        d = np.abs(a - b)
        if k == "ph":
            d = np.minimum(d, np.abs(2.0 * math.pi - d))
        with np.errstate(invalid="ignore"):
            r = d / np.maximum(np.abs(b), FLOOR[k])
        r = np.where((a == b) | (np.isnan(a) & np.isnan(b)), 0.0, r)
        r = np.where(np.isnan(r), np.inf, r)
        err = r if err is None else np.maximum(err, r)
    return err


def _nudge(t: torch.Tensor, rng) -> torch.Tensor:
    """Every element moved by a random whole number of units in the last
    place in [-ULPS, ULPS]."""
    a = t.numpy().copy()
    k = rng.integers(-ULPS, ULPS + 1, a.shape)
    for j in range(ULPS):
        a = np.where(k > j, np.nextafter(a, np.inf), a)
        a = np.where(k < -j, np.nextafter(a, -np.inf), a)
    return torch.as_tensor(a)


def oracle_runs(cfg, F, e, steps, seeds=(1, 2, 3)):
    """The oracle from the given start, and the same with the position and
    u nudged by up to ULPS units in the last place after every step."""
    ref, S, _ = run_oracle(cfg, F, e, steps)
    metric = gr.KerrSchild(cfg.a)
    grid = gr.GRGrid(F, cfg.r_min, cfg.r_max)
    dl = gr.cell_lengths(metric, grid)
    p = gr.GRParams(dt=cfg.dt, f_rho=cfg.f_rho, f_E=cfg.f_E, n_iter=cfg.n_iter)
    noisy = []
    for sd in seeds:
        rng = np.random.default_rng(sd)
        st = gr.GRState.from_numpy(e)
        for _ in range(steps):
            st, _, _ = gr.step(metric, grid, dl, st, p)
            for k in NAMES:
                setattr(st, k, _nudge(getattr(st, k), rng))
        noisy.append(st)
    return ref, S, noisy


def chaos_aware_check(got, tr_gpu, ref, S_ref, noisy, what):
    err = particle_errors(got, ref)
    sens = np.max(np.stack([particle_errors({k: getattr(s, k).numpy() for k in NAMES}, ref)
                            for s in noisy]), axis=0)
    bound = np.maximum(TOL, 10.0 * sens)
    sensitive = sens > TOL
    bad = err > bound
    log(f"{what}: {int(sensitive.sum())} of {err.size} particles sensitive beyond 1e-12 "
        f"(oracle deviation median {np.median(sens):.1e}, max {sens.max():.1e}); GPU error "
        f"median {np.median(err):.1e}, max {err.max():.1e}; over the bound: {int(bad.sum())}")
    assert not bad.any(), (what, np.flatnonzero(bad)[:10], err[bad][:10], sens[bad][:10])
    calm = ~sensitive
    mism = np.count_nonzero(tr_gpu[:, calm] != S_ref.numpy()[:, calm])
    assert mism == 0, (what, "switch decisions of insensitive particles differ", mism)
    return err, sens


@pytest.fixture(scope="module")
def g64():
    cfg = make_gr_config("grbh64")
    F = cfg.fields()
    run = GrRun(cfg, F)
    yield cfg, F, run
    run.close()


@pytest.mark.parametrize("sort_every", [0, 1])
def test_gr_fast_one_step(g64, sort_every):
    cfg, F, run = g64
    e = cfg.particles(n=4096 + 37)
    t = to_device(e, with_id=sort_every > 0)
    tr, st = run.push(t, 1, stats=True, arith=FAST, sort_every=sort_every)
    ref, S, _ = run_oracle(cfg, F, e, 1)
    if sort_every:
        order = np.argsort(t["id"].cpu().numpy())
        got = {k: t[k].cpu().numpy()[order] for k in NAMES + ("status",)}
    else:
        got = {k: t[k].cpu().numpy() for k in NAMES + ("status",)}
    err = particle_errors(got, ref)
    log(f"gr fast one step (sort_every={sort_every}): rel err median {np.median(err):.2e}, "
        f"p99 {np.quantile(err, 0.99):.2e}, max {err.max():.2e}; bit-identical "
        f"{np.mean(err == 0):.3f}")
    assert err.max() <= TOL
    assert np.array_equal(tr.cpu().numpy(), S.numpy())
    assert np.array_equal(got["status"], ref.status.numpy())
    s = S.numpy()
    assert st["gca_steps"] == int((s == 0).sum()) and st["boris_steps"] == int((s == 1).sum())
    # the production arithmetic is in effect: some results differ from the
    # exact ones
    t2 = to_device(e, with_id=sort_every > 0)
    run.push(t2, 1, sort_every=sort_every)
    assert any(not torch.equal(t2[k], t[k]) for k in NAMES)


def test_gr_fast_multistep_chaos_aware(g64):
    cfg, F, run = g64
    e = cfg.particles(n=1500, seed_offset=3)
    t = to_device(e)
    tr, _ = run.push(t, cfg.steps, arith=FAST)
    ref, S, noisy = oracle_runs(cfg, F, e, cfg.steps)
    got = {k: t[k].cpu().numpy() for k in NAMES}
    chaos_aware_check(got, tr.cpu().numpy(), ref, S, noisy, f"grbh64 {cfg.steps} steps")


def test_gr_fast_full_size_sampled():
    """grbh512 at full size (512^2 grid, 1e7 particles) for 40 steps in the
    benchmark's launch configuration (the (r, theta) tile sort every 16
    steps); 1500 sampled particles checked by the chaos-aware rule."""
    cfg = make_gr_config("grbh512")
    F = cfg.fields()
    log("gr fast full size: generating 1e7 particles")
    e = cfg.particles()
    run = GrRun(cfg, F)
    steps = 40
    try:
        t = to_device(e, per_particle_qm=False, with_id=True)
        tr, st = run.push(t, steps, stats=True, arith=FAST, sort_every=16)
        rng = np.random.default_rng(41)
        idx = np.sort(rng.choice(e.n, 1500, replace=False))
        pos = np.empty(e.n, dtype=np.int64)
        pos[t["id"].cpu().numpy()] = np.arange(e.n)
        sel = torch.as_tensor(pos[idx], device=DEV)
        got = {k: t[k][sel].cpu().numpy() for k in NAMES}
        trs = tr[:, torch.as_tensor(idx, device=DEV)].cpu().numpy()
        del t, tr
        torch.cuda.empty_cache()
    finally:
        run.close()
    log("gr fast full size: oracle runs on the sample")
    ref, S, noisy = oracle_runs(cfg, F, e.subset(idx), steps)
    chaos_aware_check(got, trs, ref, S, noisy, "grbh512 40 steps sampled")
    frac = st["gca_steps"] / max(1, st["gca_steps"] + st["boris_steps"])
    assert 0.3 < frac < 0.95


def test_gr_fast_refused(g64):
    cfg, F, run = g64
    gcb = run.gcb
    t = to_device(cfg.particles(n=16, seed_offset=5))
    with pytest.raises(gcb.GcbError) as ex:
        gcb.gcb_push_gr(run.ctx, gcb.gr_particles(t), run.params(arith=2), 1)
    assert ex.value.code == gcb.GCB_EINVAL
    with pytest.raises(gcb.GcbError) as ex:
        gcb.gcb_push_gr(run.ctx, gcb.gr_particles(t),
                        run.params(arith=FAST, form=gcb.GCB_FORM_MIXED), 1)
    assert ex.value.code == gcb.GCB_EUNSUPPORTED
