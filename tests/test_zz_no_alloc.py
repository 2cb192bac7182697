"""gcb_push_noalloc (the push for callers that cannot allocate device memory)
against gcb_push, through the C ABI (needs an MI355X).

Both run the same kernels on the same inputs, so the results must agree bit
for bit (state, ids, status bits, switch trace and statistics).  Two calls in
a row exercise the reuse of the fixed scratch: the second with fewer
particles, so stale contents of the first would show.
"""
import numpy as np
import pytest
import torch

from gpu_util import GpuRun, log
from workloads import make_config

pytestmark = pytest.mark.gpu


def _state(ens, **kw):
    from paper_2007_14401_amd import state
    return state.to_device(ens, "cuda:0", **kw)


def _same(a, b, what):
    for k in ("x", "y", "xp", "yp", "ux", "uy", "uz", "status", "id", "qm"):
        if a.get(k) is None:
            continue
        assert torch.equal(a[k], b[k]), (what, k)


@pytest.mark.parametrize("kernel,sort_every,tile", [(2, 4, 16), (1, 0, 0), (0, 3, 8)])
def test_noalloc_matches_push_twice(kernel, sort_every, tile):
    from paper_2007_14401_amd import gcb
    cfg = make_config("harris64")
    F = cfg.fields()
    run = GpuRun(cfg, F)
    try:
        for call, (n, steps, seed) in enumerate(((20000 + 37, 9, 31), (3001, 6, 32))):
            log(f"noalloc call {call}: n={n} kernel={kernel} sort_every={sort_every}")
            ens = cfg.particles(n=n, seed_offset=seed)
            prm = gcb.params(dt=cfg.dt, c=cfg.c, qm=cfg.qm, f_rho=cfg.f_rho, f_E=cfg.f_E,
                             curvature=cfg.curvature, n_iter=cfg.n_iter, kernel=kernel,
                             sort_every=sort_every, tile=tile)
            a = _state(ens)
            tra = torch.zeros((steps, n), dtype=torch.uint8, device="cuda:0")
            sta = gcb.gcb_push(run.ctx, gcb.particles(a), prm, steps, s_trace=tra,
                               want_stats=True)
            b = _state(ens)
            trb = torch.full((steps, n), 7, dtype=torch.uint8, device="cuda:0")
            stb = gcb.gcb_push_noalloc(run.ctx, gcb.particles(b), prm, steps, s_trace=trb,
                                       want_stats=True)
            torch.cuda.synchronize()
            _same(a, b, f"call {call}")
            assert torch.equal(tra, trb)
            assert sta == stb, (sta, stb)
            assert 0 < sta["gca_steps"] and 0 < sta["boris_steps"]
    finally:
        run.close()


def test_noalloc_mixed_form_and_no_stats():
    from paper_2007_14401_amd import gcb
    cfg = make_config("harris64")
    F = cfg.fields()
    run = GpuRun(cfg, F, dtype=gcb.GCB_F32)
    try:
        for n in (5000, 700):
            ens = cfg.particles(n=n, seed_offset=33)
            prm = gcb.params(dt=cfg.dt, c=cfg.c, qm=cfg.qm, f_rho=cfg.f_rho, f_E=cfg.f_E,
                             curvature=cfg.curvature, n_iter=cfg.n_iter,
                             form=gcb.GCB_FORM_MIXED, sort_every=2, tile=16)
            a = _state(ens, form=gcb.GCB_FORM_MIXED)
            gcb.gcb_push(run.ctx, gcb.particles(a), prm, 5)
            b = _state(ens, form=gcb.GCB_FORM_MIXED)
            gcb.gcb_push_noalloc(run.ctx, gcb.particles(b), prm, 5)
            torch.cuda.synchronize()
            _same(a, b, f"mixed n={n}")
    finally:
        run.close()


def test_noalloc_rejects_what_does_not_fit():
    """A sorted push of more particles than the fixed scratch holds fails with
    GCB_EINVAL and leaves the state untouched; without sorting the same
    particles need only the statistics slots and run."""
    from paper_2007_14401_amd import gcb
    cfg = make_config("harris64")
    F = cfg.fields()
    run = GpuRun(cfg, F)
    try:
        n = 1_000_000
        ens = cfg.particles(n=n, seed_offset=34)
        t = _state(ens)
        before = {k: v.clone() for k, v in t.items() if v is not None}
        prm = gcb.params(dt=cfg.dt, c=cfg.c, qm=cfg.qm, curvature=cfg.curvature,
                         n_iter=cfg.n_iter, sort_every=4, tile=16)
        with pytest.raises(gcb.GcbError) as e:
            gcb.gcb_push_noalloc(run.ctx, gcb.particles(t), prm, 2, want_stats=True)
        assert e.value.code == gcb.GCB_EINVAL
        assert "scratch" in str(e.value)
        torch.cuda.synchronize()
        _same(before, t, "rejected call")
        prm.sort_every = 0
        prm.kernel = gcb.GCB_KERNEL_GLOBAL
        st = gcb.gcb_push_noalloc(run.ctx, gcb.particles(t), prm, 1, want_stats=True)
        assert st["gca_steps"] + st["boris_steps"] == n
    finally:
        run.close()
