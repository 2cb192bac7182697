"""Curved-spacetime push on the GPU (gcb_push_gr) against the binary64 CPU
oracle (oracle/gr.py) on the same seeded inputs.

The kernel evaluates the oracle's operations in the same order with IEEE
binary64 arithmetic (no fused multiply-add, IEEE quotients and square roots,
the same sin/cos polynomial), so positions, four-velocities, status bits and
switch decisions are compared bit for bit; the stated tolerance 1e-12 (relative)
is the fallback bound should a compiler ever reorder an operation.
"""
import math

import numpy as np
import pytest
import torch

from gpu_util import log
from oracle import gr
from workloads import make_gr_config

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NAMES = ("r", "th", "ph", "ur", "uth", "uph")


class GrRun:
    def __init__(self, cfg, F):
        from paper_2007_14401_amd import gcb
        self.gcb = gcb
        self.cfg = cfg
        self.ctx = gcb.gcb_create(0)
        desc = gcb.gr_desc(cfg.nr, cfg.nth, cfg.r_min, cfg.r_max, cfg.a)
        gcb.gcb_load_fields_gr(self.ctx, desc, [np.ascontiguousarray(F[k]) for k in range(3)],
                               [np.ascontiguousarray(F[k]) for k in range(3, 6)])

    def params(self, **kw):
        cfg = self.cfg
        d = dict(dt=cfg.dt, c=1.0, qm=cfg.qm, f_rho=cfg.f_rho, f_E=cfg.f_E, n_iter=cfg.n_iter)
        d.update(kw)
        return self.gcb.params(**d)

    def push(self, t, steps, trace=True, stats=False, **kw):
        n = t["r"].shape[0]
        tr = torch.zeros((steps, n), dtype=torch.uint8, device=DEV) if trace else None
        st = self.gcb.gcb_push_gr(self.ctx, self.gcb.gr_particles(t), self.params(**kw), steps,
                                  s_trace=tr, want_stats=stats)
        torch.cuda.synchronize()
        return tr, st

    def close(self):
        self.gcb.gcb_destroy(self.ctx)


def to_device(e, per_particle_qm=True):
    t = {k: torch.as_tensor(np.ascontiguousarray(getattr(e, k)), dtype=torch.float64,
                            device=DEV) for k in NAMES}
    t["status"] = torch.zeros(e.n, dtype=torch.uint8, device=DEV)
    t["qm"] = (torch.as_tensor(e.qm, dtype=torch.float64, device=DEV)
               if per_particle_qm else None)
    return t


def run_oracle(cfg, F, e, steps, **kw):
    grid = gr.GRGrid(F, cfg.r_min, cfg.r_max)
    d = dict(dt=cfg.dt, f_rho=cfg.f_rho, f_E=cfg.f_E, n_iter=cfg.n_iter)
    d.update(kw)
    st, S, res = gr.push(gr.KerrSchild(cfg.a), grid, gr.GRState.from_numpy(e), gr.GRParams(**d),
                         steps, trace=True)
    return st, S, res


def compare(t, ref, tr=None, S=None, idx=None, what=""):
    worst = 0.0
    for k in NAMES:
        a = t[k].cpu().numpy()
        if idx is not None:
            a = a[idx]
        b = getattr(ref, k).numpy()
        same = a.view(np.uint64) == b.view(np.uint64)
        fin = np.isfinite(b)
        rel = np.abs(a - b) / np.maximum(np.abs(b), 1e-300)
        w = float(np.max(np.where(fin & ~same, rel, 0.0))) if (~same).any() else 0.0
        worst = max(worst, w)
        assert w <= 1e-12, (what, k, w)
        # non-finite entries must agree in kind
        assert np.array_equal(np.isnan(a), np.isnan(b)), (what, k)
    st = t["status"].cpu().numpy()
    if idx is not None:
        st = st[idx]
    assert np.array_equal(st, ref.status.numpy()), (what, "status")
    if tr is not None:
        trc = tr.cpu().numpy()
        if idx is not None:
            trc = trc[:, idx]
        assert np.array_equal(trc, S.numpy()), (what, "switch decisions")
    log(f"{what}: max rel err {worst:.1e}")
    return worst


@pytest.fixture(scope="module")
def g64():
    cfg = make_gr_config("grbh64")
    F = cfg.fields()
    run = GrRun(cfg, F)
    yield cfg, F, run
    run.close()


def test_gr_one_step(g64):
    cfg, F, run = g64
    e = cfg.particles(n=4096 + 37)          # ragged tail of the last workgroup
    t = to_device(e)
    tr, st = run.push(t, 1, stats=True)
    ref, S, res = run_oracle(cfg, F, e, 1)
    compare(t, ref, tr, S, what="gr one step")
    s = S.numpy()
    assert st["gca_steps"] == int((s == 0).sum()) and st["boris_steps"] == int((s == 1).sum())
    assert (s == 0).any() and (s == 1).any()


def test_gr_multistep(g64):
    cfg, F, run = g64
    e = cfg.particles(n=3000, seed_offset=1)
    t = to_device(e)
    tr, st = run.push(t, cfg.steps, stats=True)
    ref, S, res = run_oracle(cfg, F, e, cfg.steps)
    compare(t, ref, tr, S, what=f"gr {cfg.steps} steps")
    assert abs(st["max_fp_residual"] - float(res.max())) <= 1e-12 * max(1.0, float(res.max()))
    flagged = int(((ref.status.numpy() & ~np.uint8(32)) != 0).sum())
    assert st["flagged"] == flagged


@pytest.mark.parametrize("kw", [{"n_iter": 1}, {"n_iter": 3}, {"f_rho": 0.0},
                                {"f_rho": math.inf, "f_E": math.inf}, {"f_E": 0.5}])
def test_gr_variants(g64, kw):
    cfg, F, run = g64
    e = cfg.particles(n=1500, seed_offset=2)
    t = to_device(e)
    tr, _ = run.push(t, 10, **kw)
    ref, S, _ = run_oracle(cfg, F, e, 10, **kw)
    compare(t, ref, tr, S, what=f"gr variant {kw}")


def test_gr_scalar_qm(g64):
    cfg, F, run = g64
    e = cfg.particles(n=1000, seed_offset=3)
    t = to_device(e, per_particle_qm=False)
    tr, _ = run.push(t, 8)
    ref, S, _ = run_oracle(cfg, F, e, 8)
    compare(t, ref, tr, S, what="gr scalar q/m")


def test_gr_edge_cases(g64):
    """Empty input; one particle; particles outside the domain (below r_min,
    beyond r_max, past a pole) are flagged and left unchanged; a particle
    falling through r_min stops there."""
    cfg, F, run = g64
    e0 = cfg.particles(n=0)
    t0 = to_device(e0)
    run.push(t0, 3)
    e1 = cfg.particles(n=1, seed_offset=4)
    t1 = to_device(e1)
    tr1, _ = run.push(t1, 5)
    ref1, S1, _ = run_oracle(cfg, F, e1, 5)
    compare(t1, ref1, tr1, S1, what="gr one particle")
    e = cfg.particles(n=6, seed_offset=5)
    e.r[0] = cfg.r_min - 0.1
    e.r[1] = cfg.r_max + 1.0
    e.th[2] = -0.01
    e.th[3] = math.pi + 0.01
    e.r[4] = cfg.r_min + 1e-3                 # inward bound: leaves within a few steps
    e.ur[4] = -50.0
    t = to_device(e)
    tr, _ = run.push(t, 6)
    ref, S, _ = run_oracle(cfg, F, e, 6)
    compare(t, ref, tr, S, what="gr out of domain")
    st = t["status"].cpu().numpy()
    assert all(st[k] & 64 for k in range(5))
    for k in range(4):
        assert t["r"][k].item() == e.r[k] and t["th"][k].item() == e.th[k]


def test_gr_full_size_sampled():
    """grbh512 at its full size (512^2 grid, 1e7 particles) for 20 steps in
    the launch configuration the benchmark times; 2000 sampled particles are
    pushed by the oracle and compared bit for bit."""
    cfg = make_gr_config("grbh512")
    F = cfg.fields()
    log("gr full size: generating 1e7 particles")
    e = cfg.particles()
    run = GrRun(cfg, F)
    try:
        t = to_device(e, per_particle_qm=False)
        steps = 20
        tr, st = run.push(t, steps, stats=True)
        log(f"gr full size: stats {st}")
        rng = np.random.default_rng(99)
        idx = np.sort(rng.choice(e.n, 2000, replace=False))
        got = {k: t[k][torch.as_tensor(idx, device=DEV)].cpu() for k in NAMES + ("status",)}
        trs = tr[:, torch.as_tensor(idx, device=DEV)].cpu()
        del t, tr
        torch.cuda.empty_cache()
        ref, S, _ = run_oracle(cfg, F, e.subset(idx), steps)
        compare(got, ref, trs, S, what="gr full size sample")
        frac = st["gca_steps"] / max(1, st["gca_steps"] + st["boris_steps"])
        log(f"gr full size: guiding-center fraction {frac:.3f}")
        assert 0.3 < frac < 0.95
    finally:
        run.close()


def test_gr_argument_validation(g64):
    cfg, F, run = g64
    gcb = run.gcb
    e = cfg.particles(n=10, seed_offset=6)
    t = to_device(e)
    with pytest.raises(gcb.GcbError) as ex:
        gcb.gcb_push_gr(run.ctx, gcb.gr_particles(t), run.params(form=gcb.GCB_FORM_MIXED), 1)
    assert ex.value.code == gcb.GCB_EUNSUPPORTED
    with pytest.raises(gcb.GcbError) as ex:
        gcb.gcb_push_gr(run.ctx, gcb.gr_particles(t), run.params(n_iter=0), 1)
    assert ex.value.code == gcb.GCB_EINVAL
    with pytest.raises(gcb.GcbError) as ex:
        gcb.gcb_push_gr(run.ctx, gcb.gr_particles(t), run.params(dt=-1.0), 1)
    assert ex.value.code == gcb.GCB_EINVAL
    p = gcb.gr_particles(t)
    p.ur = None
    with pytest.raises(gcb.GcbError):
        gcb.gcb_push_gr(run.ctx, p, run.params(), 1)
    bad = gcb.gr_desc(cfg.nr, cfg.nth, 2.0, 1.0, cfg.a)
    with pytest.raises(gcb.GcbError):
        gcb.gcb_load_fields_gr(run.ctx, bad, [F[0], F[1], F[2]], [F[3], F[4], F[5]])
    bad = gcb.gr_desc(cfg.nr, cfg.nth, cfg.r_min, cfg.r_max, 1.0)
    with pytest.raises(gcb.GcbError):
        gcb.gcb_load_fields_gr(run.ctx, bad, [F[0], F[1], F[2]], [F[3], F[4], F[5]])
    ctx = gcb.gcb_create(0)
    try:
        with pytest.raises(gcb.GcbError) as ex:
            gcb.gcb_push_gr(ctx, gcb.gr_particles(t), run.params(), 1)
        assert ex.value.code == gcb.GCB_ENOFIELDS
    finally:
        gcb.gcb_destroy(ctx)
