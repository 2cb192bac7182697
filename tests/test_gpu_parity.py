"""Parity of the HIP binary64 path with the CPU oracle (needs an MI355X).

Bar (from the arithmetic): the binary64 kernels evaluate the same operations
in the same order as the oracle with correctly rounded +, -, *, /, sqrt and no
contraction, so results are expected to agree to the last bit; the asserted
tolerance is 1e-12 relative (floors: one cell for positions, c for u) with
identical switch decisions at every step and identical status bits (the
informational LDS-window bit excluded).
"""
import math

import numpy as np
import pytest
import torch

from gpu_util import GpuRun, log, rel_errors, run_oracle
from workloads import make_config

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _state(ens, **kw):
    from paper_2007_14401_amd import state
    return state.to_device(ens, "cuda:0", **kw)


def _check(got, ref, cfg, what, tr_gpu=None, tr_ref=None):
    errs = rel_errors(got, ref, cfg)
    log(f"{what}: max rel err {errs}")
    for k, v in errs.items():
        assert v <= TOL, (what, k, v)
    st_ref = ref.status.numpy()
    st_gpu = got["status"] & ~np.uint8(32)
    assert np.array_equal(st_gpu, st_ref), (what, "status bits differ",
                                            np.count_nonzero(st_gpu != st_ref))
    if tr_gpu is not None:
        a = tr_gpu.cpu().numpy()
        b = tr_ref.numpy()
        assert a.shape == b.shape
        mism = np.count_nonzero(a != b)
        assert mism == 0, (what, "switch decisions differ", mism)


@pytest.fixture(scope="module")
def h64():
    cfg = make_config("harris64")
    F = cfg.fields()
    run = GpuRun(cfg, F)
    yield cfg, F, run
    run.close()


@pytest.mark.parametrize("kernel,sort_every,tile", [(1, 0, 0), (2, 1, 16), (2, 4, 16), (0, 3, 8)])
def test_one_step(h64, kernel, sort_every, tile):
    from paper_2007_14401_amd import state
    cfg, F, run = h64
    ens = cfg.particles(n=4096 + 37)      # ragged tail
    log(f"one step kernel={kernel} sort_every={sort_every} tile={tile}")
    t = _state(ens)
    tr, _ = run.push(t, 1, trace=True, kernel=kernel, sort_every=sort_every, tile=tile)
    ref, rtr, _ = run_oracle(cfg, F, ens, 1, trace=True)
    _check(state.unsort(t), ref, cfg, "one step", tr, rtr)
    assert 0 < int(rtr.sum()) < rtr.numel()


@pytest.mark.parametrize("kernel,sort_every,tile", [(1, 0, 0), (2, 4, 16), (2, 1, 32)])
def test_multistep(h64, kernel, sort_every, tile):
    from paper_2007_14401_amd import state
    cfg, F, run = h64
    ens = cfg.particles(n=3000)
    steps = 50
    log(f"multistep kernel={kernel} sort_every={sort_every} tile={tile}")
    t = _state(ens)
    tr, st = run.push(t, steps, trace=True, stats=True, kernel=kernel,
                      sort_every=sort_every, tile=tile)
    ref, rtr, rres = run_oracle(cfg, F, ens, steps, trace=True)
    _check(state.unsort(t), ref, cfg, "multistep", tr, rtr)
    assert st["gca_steps"] == int((rtr == 0).sum())
    assert st["boris_steps"] == int((rtr == 1).sum())
    assert st["max_fp_residual"] == float(rres.max())
    # status histogram: particles per status bit (the halo bit is the GPU's own)
    bits = ref.status.numpy()
    for k in range(8):
        if k == 5:
            continue
        assert st["status_counts"][k] == int(((bits >> k) & 1).sum()), k
    assert st["flagged"] == int(((bits & ~np.uint8(32)) != 0).sum())


VARIANTS = [
    dict(curvature=0),
    dict(n_iter=1),
    dict(n_iter=3),
    dict(f_rho=0.0),                          # every particle Boris
    dict(f_rho=math.inf, f_E=math.inf),       # every particle guiding center (E > B too)
    dict(f_rho=1.0, f_E=0.5),
]


@pytest.mark.parametrize("var", VARIANTS, ids=[str(v) for v in VARIANTS])
@pytest.mark.parametrize("kernel", [1, 2])
def test_variants(h64, var, kernel):
    from paper_2007_14401_amd import state
    cfg, F, run = h64
    cfg2 = cfg.with_(**{k: v for k, v in var.items() if k in ("curvature", "n_iter", "f_rho", "f_E")})
    ens = cfg.particles(n=1500, seed_offset=5)
    steps = 12
    log(f"variant {var} kernel={kernel}")
    t = _state(ens)
    tr, _ = run.push(t, steps, trace=True, kernel=kernel, sort_every=2 if kernel == 2 else 0,
                     tile=16, **var)
    ref, rtr, _ = run_oracle(cfg2, F, ens, steps, trace=True)
    _check(state.unsort(t), ref, cfg2, f"variant {var}", tr, rtr)


def test_scalar_qm_and_no_ids(h64):
    """params.qm instead of a per-particle array; no id array, no sort."""
    from paper_2007_14401_amd import state
    cfg, F, run = h64
    ens = cfg.particles(n=777)
    t = _state(ens, per_particle_qm=False, with_id=False)
    run.push(t, 10, kernel=1, sort_every=0)
    ref, _, _ = run_oracle(cfg, F, ens, 10)
    _check(state.to_host(t), ref, cfg, "scalar qm")


@pytest.mark.parametrize("geom", ["collocated", "dx_half"])
def test_grid_geometry(geom):
    """Non-Yee lattice (runtime offsets) and a non-unit cell size."""
    from paper_2007_14401_amd import state
    from workloads.harris import COLLOCATED
    base = make_config("harris64")
    if geom == "collocated":
        cfg = base.with_(stagger=tuple(map(tuple, COLLOCATED)))
    else:
        cfg = base.with_(dx=0.5, dy=0.5, delta=2.0, c=0.225)
    F = cfg.fields()
    run = GpuRun(cfg, F)
    try:
        ens = cfg.particles(n=2000, seed_offset=9)
        for kernel in (1, 2):
            log(f"geometry {geom} kernel={kernel}")
            t = _state(ens)
            tr, _ = run.push(t, 10, trace=True, kernel=kernel,
                             sort_every=2 if kernel == 2 else 0, tile=16)
            ref, rtr, _ = run_oracle(cfg, F, ens, 10, trace=True)
            _check(state.unsort(t), ref, cfg, f"geometry {geom}", tr, rtr)
    finally:
        run.close()


def test_edge_sizes(h64):
    """n = 0 and n = 1 through both kernels."""
    from paper_2007_14401_amd import state
    cfg, F, run = h64
    for n in (0, 1):
        ens = cfg.particles(n=max(n, 1))
        if n == 0:
            ens = ens.subset(slice(0, 0))
        for kernel, se in ((1, 0), (2, 1)):
            t = _state(ens)
            run.push(t, 3, kernel=kernel, sort_every=se, tile=16)
            if n:
                ref, _, _ = run_oracle(cfg, F, ens, 3)
                _check(state.unsort(t), ref, cfg, f"n={n}")


def test_deterministic(h64):
    """Two runs give bitwise identical states (no atomics on the forward path)."""
    cfg, F, run = h64
    ens = cfg.particles(n=5000, seed_offset=2)
    outs = []
    for _ in range(2):
        t = _state(ens)
        run.push(t, 20, kernel=2, sort_every=4, tile=16)
        outs.append({k: v.cpu().numpy().copy() for k, v in t.items() if v is not None})
    for k in outs[0]:
        assert np.array_equal(outs[0][k].view(np.uint8), outs[1][k].view(np.uint8)), k


def test_c1_full_run():
    """harris256: 1e4 electrons, 1000 steps, Omega_c0 dt in [0.1, 1e3]; every
    switch decision and the final state against the oracle."""
    from paper_2007_14401_amd import state
    cfg = make_config("harris256")
    F = cfg.fields()
    ens = cfg.particles()
    run = GpuRun(cfg, F)
    try:
        log("c1 full run: gpu")
        t = _state(ens)
        tr, st = run.push(t, cfg.steps, trace=True, stats=True, kernel=2, sort_every=4, tile=32)
        log(f"c1 stats {st}")
        log("c1 full run: oracle")
        ref, rtr, _ = run_oracle(cfg, F, ens, cfg.steps, trace=True)
        _check(state.unsort(t), ref, cfg, "c1 full", tr, rtr)
        frac = 1.0 - float(rtr.double().mean())
        log(f"c1 guiding-center fraction {frac:.3f}")
        assert 0.3 < frac < 0.95
    finally:
        run.close()


def test_c2_full_size_sampled():
    """harris4096 at full size (1e7 particles, 100 steps) in the benchmark's
    launch configuration; 3000 sampled particles recomputed by the oracle."""
    from paper_2007_14401_amd import state
    cfg = make_config("harris4096")
    log("c2: generating inputs")
    F = cfg.fields()
    ens = cfg.particles()
    run = GpuRun(cfg, F)
    try:
        log("c2: gpu push")
        t = _state(ens)
        steps = cfg.steps
        _, st = run.push(t, steps, stats=True, kernel=2, sort_every=10, tile=20)
        log(f"c2 stats {st}")
        frac = st["gca_steps"] / (st["gca_steps"] + st["boris_steps"])
        log(f"c2 guiding-center fraction over the run {frac:.3f}")
        ids = t["id"].cpu().numpy()
        rng = np.random.default_rng(77)
        sample = np.sort(rng.choice(ens.n, 3000, replace=False))
        pos = np.empty(ens.n, dtype=np.int64)
        pos[ids] = np.arange(ens.n)
        h = {k: (v.cpu().numpy()[pos[sample]] if v is not None else None) for k, v in t.items()}
        del t
        log("c2: oracle on the sample")
        ref, _, _ = run_oracle(cfg, F, ens.subset(sample), steps)
        _check(h, ref, cfg, "c2 sampled")
    finally:
        run.close()


def test_kinetic_energy(h64):
    from paper_2007_14401_amd import gcb
    import oracle as O
    cfg, F, run = h64
    ens = cfg.particles(n=10001)
    t = _state(ens)
    out = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    lam = [torch.zeros_like(t["ux"]) for _ in range(3)]
    gcb.gcb_kinetic_energy(run.ctx, gcb.particles(t), gcb.params(c=cfg.c), out, lam)
    torch.cuda.synchronize()
    ux, uy, uz = (torch.as_tensor(getattr(ens, k)) for k in ("ux", "uy", "uz"))
    ref = float(O.kinetic_energy(ux, uy, uz, cfg.c))
    assert abs(float(out) - ref) <= 1e-13 * abs(ref)
    g = torch.sqrt(1 + (ux**2 + uy**2 + uz**2) / cfg.c**2)
    assert torch.allclose(lam[0].cpu(), ux / (ens.n * g), rtol=1e-14, atol=0)


def test_argument_validation(h64):
    from paper_2007_14401_amd import gcb
    cfg, F, run = h64
    ens = cfg.particles(n=64)
    t = _state(ens)
    bad = [dict(dt=0.0), dict(c=-1.0), dict(n_iter=0), dict(form=7), dict(kernel=9),
           dict(sort_every=-1), dict(curvature=2)]
    for b in bad:
        with pytest.raises(gcb.GcbError) as e:
            gcb.gcb_push(run.ctx, gcb.particles(t), gcb.params(**b), 1)
        assert e.value.code == gcb.GCB_EINVAL, b
    p = gcb.particles(t)
    p.x = None
    with pytest.raises(gcb.GcbError):
        gcb.gcb_push(run.ctx, p, gcb.params(), 1)
    # mixed form needs float fields
    with pytest.raises(gcb.GcbError):
        gcb.gcb_push(run.ctx, gcb.particles(t), gcb.params(form=gcb.GCB_FORM_MIXED), 1)
    # tiled kernel without sorting
    with pytest.raises(gcb.GcbError) as e:
        gcb.gcb_push(run.ctx, gcb.particles(t), gcb.params(kernel=2, sort_every=0), 1)
    assert e.value.code == gcb.GCB_EUNSUPPORTED
    # fresh context without fields
    ctx = gcb.gcb_create(0)
    try:
        with pytest.raises(gcb.GcbError) as e:
            gcb.gcb_push(ctx, gcb.particles(t), gcb.params(), 1)
        assert e.value.code == gcb.GCB_ENOFIELDS
    finally:
        gcb.gcb_destroy(ctx)


@pytest.mark.parametrize("tile", [16, 24])
def test_cell_sort_order(h64, tile):
    """The cell sort is a stable sort by tile (row-major tiles): after one
    step with sort_every = 1 the particles sit in that order of their start
    positions (bit-exact index work; the 64-cell grid leaves a ragged last
    tile for tile = 24)."""
    cfg, F, run = h64
    ens = cfg.particles(n=4096 + 37, seed_offset=11)
    t = _state(ens)
    run.push(t, 1, kernel=2, sort_every=1, tile=tile)
    cx = np.floor(ens.x / cfg.dx).astype(np.int64)
    cy = np.floor(ens.y / cfg.dy).astype(np.int64)
    ntx = -(-cfg.nx // tile)
    key = (cy // tile) * ntx + cx // tile
    want = np.argsort(key, kind="stable")
    got = t["id"].cpu().numpy()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("kernel,sort_every", [(1, 0), (2, 3)])
def test_replayed_switch_decisions_reproduce_the_run(h64, kernel, sort_every):
    """A push with params.replay = 1 reads S from the trace of an earlier push
    and reproduces it bit for bit."""
    cfg, F, run = h64
    ens = cfg.particles(n=2500, seed_offset=8)
    t1 = _state(ens)
    tr, _ = run.push(t1, 15, trace=True, kernel=kernel, sort_every=sort_every, tile=16)
    t2 = _state(ens)
    from paper_2007_14401_amd import gcb
    prm = gcb.params(dt=cfg.dt, c=cfg.c, qm=cfg.qm, f_rho=cfg.f_rho, f_E=cfg.f_E,
                     curvature=cfg.curvature, n_iter=cfg.n_iter, kernel=kernel,
                     sort_every=sort_every, tile=16, replay=1)
    tr_copy = tr.clone()
    gcb.gcb_push(run.ctx, gcb.particles(t2), prm, 15, s_trace=tr)
    torch.cuda.synchronize()
    assert torch.equal(tr, tr_copy)            # replay reads, does not write
    for k in ("x", "y", "xp", "yp", "ux", "uy", "uz", "status", "id"):
        assert torch.equal(t1[k], t2[k]), k


@pytest.mark.parametrize("kernel", [1, 2])
def test_split_calls_equal_one_call(h64, kernel):
    """13 steps as 7 + 6 steps in two calls equal 13 steps in one call, bit for
    bit: with a sort every 3 steps the first call ends after an odd number of
    sorts (its state comes back from the library's buffer) and the second
    call sorts on a different schedule; every particle is independent of the
    others, so the results do not depend on the order."""
    from paper_2007_14401_amd import state
    cfg, F, run = h64
    ens = cfg.particles(n=3001, seed_offset=12)
    a = _state(ens)
    run.push(a, 13, kernel=kernel, sort_every=3, tile=16)
    b = _state(ens)
    run.push(b, 7, kernel=kernel, sort_every=3, tile=16)
    run.push(b, 6, kernel=kernel, sort_every=3, tile=16)
    ha, hb = state.unsort(a), state.unsort(b)
    for k in ("x", "y", "xp", "yp", "ux", "uy", "uz", "status", "qm"):
        assert np.array_equal(ha[k], hb[k]), k


def test_non_default_stream(h64):
    """Work enqueued on a caller's stream gives the null stream's result."""
    from paper_2007_14401_amd import gcb, state
    cfg, F, run = h64
    ens = cfg.particles(n=2048, seed_offset=13)
    a = _state(ens)
    run.push(a, 8, kernel=2, sort_every=2, tile=16)
    b = _state(ens)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    prm = gcb.params(dt=cfg.dt, c=cfg.c, qm=cfg.qm, f_rho=cfg.f_rho, f_E=cfg.f_E,
                     curvature=cfg.curvature, n_iter=cfg.n_iter, kernel=2, sort_every=2,
                     tile=16)
    gcb.gcb_push(run.ctx, gcb.particles(b), prm, 8, stream=s)
    s.synchronize()
    for k in ("x", "y", "ux", "uy", "uz", "status", "id"):
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("kernel,sort_every,tile,steps", [(2, 4, 16, 12), (2, 3, 8, 7),
                                                          (1, 4, 0, 6), (0, 1, 16, 3)])
def test_keep_order(h64, kernel, sort_every, tile, steps):
    """keep_order: the particles are cell-sorted and pushed tile by tile, but
    every one is written back to its own slot, so the arrays keep their order
    and the switch trace is in slot order without ids.  The state and the
    trace equal the oracle's in input order, bit for bit."""
    cfg, F, run = h64
    ens = cfg.particles(n=4096 + 37, seed_offset=11)
    log(f"keep_order kernel={kernel} sort_every={sort_every} tile={tile} steps={steps}")
    t = _state(ens, with_id=False)
    tr, st = run.push(t, steps, trace=True, stats=True, kernel=kernel, sort_every=sort_every,
                      tile=tile, keep_order=1)
    ref, rtr, rres = run_oracle(cfg, F, ens, steps, trace=True)
    got = {k: v.cpu().numpy() for k, v in t.items() if v is not None}
    _check(got, ref, cfg, "keep_order", tr, rtr)
    assert st["gca_steps"] == int((rtr == 0).sum())
    assert st["max_fp_residual"] == float(rres.max())
