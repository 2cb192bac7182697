"""Parity of the HIP path with the oracle on the method's edge cases (needs an
MI355X), on the crafted field and particle set of workloads/edge.py:

  * B = 0 at a conversion point (GCB_ST_BZERO) and at x^n (the switch takes
    the full orbit), E > B at a conversion point (drift speed above c:
    GCB_ST_KAPPA) and at x^n;
  * NaN and infinite components of u (GCB_ST_NONFINITE);
  * particles exactly at f_rho and at f_E and a few ulp either side
    (the switch's strict "<", Sec. 4.1);
  * every particle on the guiding-center branch (f_rho = f_E = inf): the
    quadratic of the parallel update without an admissible root
    (GCB_ST_QUAD, with and without the mirror terms), fixed-point iterations
    that do not settle (GCB_ST_FPRES);
  * conversion points 11.75 cells from x^n, outside the LDS window of the
    tiled kernel (GCB_ST_HALO: the gather falls back to global memory with
    the same values);
  * time steps other than 1 (0.37 and 2).

Bar: the binary64 parity bar (bit for bit expected, 1e-12 asserted, NaN equal
to NaN), identical switch decisions at every step, identical status bits
(the LDS-window bit excluded from the comparison, asserted separately).
The precision form is checked on the threshold groups: there the field
samples are exact in binary32, so its binary64 re-check near a threshold must
take the oracle's decision.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import log, rel_errors
from test_gpu_3d import rel_errors3
from workloads.edge import (C_LIGHT, F_E, F_RHO, NX, NY, NZ, edge_fields, edge_fields3,
                            edge_particles, edge_particles3)
from workloads.harris import YEE_STAGGER

pytestmark = pytest.mark.gpu

TOL = 1e-12
INF = math.inf
STEPS = 6
HALO = 32
ST = dict(nonfinite=1, kappa=2, quad=4, bzero=8, fpres=16, mirror=128)

# parameter sets: the paper's switch with the edge thresholds (and the check
# of the neglect of the mirror terms), and every particle guiding center
RUNS = {
    "switch": (dict(f_rho=F_RHO, f_E=F_E, mirror_tol=1e-3),
               ("nonfinite", "kappa", "bzero", "fpres", "mirror")),
    "all_gca": (dict(f_rho=INF, f_E=INF), ("nonfinite", "kappa", "quad", "bzero", "fpres")),
    "all_gca_mirror": (dict(f_rho=INF, f_E=INF, mirror=1),
                       ("nonfinite", "kappa", "quad", "bzero", "fpres")),
}
KERNELS = [(1, 0, 0), (2, 1, 16), (2, 3, 8)]


class Cfg:
    """The edge workload's geometry in the attribute names of the helpers."""
    nx, ny, nz = NX, NY, NZ
    dx = dy = dz = 1.0
    Lx, Ly, Lz = float(NX), float(NY), float(NZ)
    c = C_LIGHT


_oracle_cache = {}


def _oracle(dim, dt, name, F, ens):
    key = (dim, dt, name)
    if key not in _oracle_cache:
        kw = dict(RUNS[name][0])
        p = dict(dt=dt, c=C_LIGHT, curvature=True, n_iter=4, Lx=float(NX), Ly=float(NY),
                 dl=1.0, f_rho=kw["f_rho"], f_E=kw["f_E"], mirror=bool(kw.get("mirror", 0)),
                 mirror_tol=kw.get("mirror_tol", 0.0))
        if dim == 2:
            prov = O.GridFields(F, 1.0, 1.0, YEE_STAGGER)
            out = O.push(prov, O.State.from_numpy(ens), O.Params(**p), STEPS, trace=True)
        else:
            prov = O.GridFields3(F, 1.0, 1.0, 1.0, O.YEE3)
            out = O.push3(prov, O.State3.from_numpy(ens), O.Params3(Lz=float(NZ), **p), STEPS,
                          trace=True)
        _oracle_cache[key] = out
    return _oracle_cache[key]


def _gpu(dim, F, ens, dt, name, kernel, sort_every, tile, form=0):
    from paper_2007_14401_amd import gcb, state
    ctx = gcb.gcb_create(0)
    try:
        fdt = gcb.GCB_F64 if form == gcb.GCB_FORM_F64 else gcb.GCB_F32
        if dim == 2:
            desc = gcb.grid_desc(NX, NY, 1.0, 1.0, gcb.YEE_STAGGER, fdt)
            gcb.gcb_load_fields(ctx, desc, [F[0], F[1], F[2]], [F[3], F[4], F[5]])
        else:
            desc = gcb.grid3_desc(NX, NY, NZ, 1.0, 1.0, 1.0, gcb.YEE3_STAGGER, fdt)
            gcb.gcb_load_fields_3d(ctx, desc, [F[0], F[1], F[2]], [F[3], F[4], F[5]])
        t = state.to_device(ens, "cuda:0", form=form)
        kw = dict(RUNS[name][0])
        prm = gcb.params(dt=dt, c=C_LIGHT, qm=-1.0, curvature=1, n_iter=4, form=form,
                         kernel=kernel, sort_every=sort_every, tile=tile, **kw)
        tr = torch.zeros((STEPS, ens.n), dtype=torch.uint8, device="cuda:0")
        push = gcb.gcb_push if dim == 2 else gcb.gcb_push_3d
        parts = gcb.particles(t) if dim == 2 else gcb.particles3(t)
        st = push(ctx, parts, prm, STEPS, s_trace=tr, want_stats=True)
        torch.cuda.synchronize()
        return state.unsort(t), tr.cpu().numpy(), st
    finally:
        gcb.gcb_destroy(ctx)


def _compare(dim, got, tr, st, ref, rtr, what, kernel, sort_every, required):
    errs = (rel_errors if dim == 2 else rel_errors3)(got, ref, Cfg)
    log(f"{what}: max rel err {max(errs.values()):.2e}, stats {st}")
    for k, v in errs.items():
        assert v <= TOL, (what, k, v)
    s_ref = ref.status.numpy()
    s_gpu = got["status"]
    assert np.array_equal(s_gpu & ~np.uint8(HALO), s_ref), (
        what, "status bits differ", np.count_nonzero((s_gpu & ~np.uint8(HALO)) != s_ref))
    assert np.array_equal(tr, rtr.numpy()), (what, "switch decisions differ")
    for b in required:
        assert int(((s_ref & ST[b]) != 0).sum()) > 0, (what, f"no particle with {b}")
    halo = (s_gpu & HALO) != 0
    if kernel == 1:
        assert st["halo_misses"] == 0 and not halo.any()
    elif sort_every == 1:
        # the far_prev group's conversion points lie outside every window
        assert st["halo_misses"] > 0 and halo.any(), what
    assert st["status_counts"][5] == int(halo.sum())
    assert st["gca_steps"] == int((rtr == 0).sum())
    assert st["boris_steps"] == int((rtr == 1).sum())


@pytest.fixture(scope="module")
def fields2():
    return edge_fields()


@pytest.fixture(scope="module")
def fields3():
    return edge_fields3()


@pytest.mark.parametrize("kernel,sort_every,tile", KERNELS)
@pytest.mark.parametrize("dt", [1.0, 0.37, 2.0])
@pytest.mark.parametrize("name", list(RUNS))
def test_edge_2d(fields2, name, dt, kernel, sort_every, tile):
    es = edge_particles(dt=dt)
    log(f"edge 2d {name} dt={dt} kernel={kernel} sort_every={sort_every} tile={tile}")
    got, tr, st = _gpu(2, fields2, es.ens, dt, name, kernel, sort_every, tile)
    ref, rtr, _ = _oracle(2, dt, name, fields2, es.ens)
    _compare(2, got, tr, st, ref, rtr, f"edge 2d {name} dt={dt} k={kernel}", kernel,
             sort_every, RUNS[name][1])


@pytest.mark.parametrize("kernel,sort_every,tile", [(1, 0, 0), (2, 1, 6)])
@pytest.mark.parametrize("dt", [1.0, 0.37])
@pytest.mark.parametrize("name", list(RUNS))
def test_edge_3d(fields3, name, dt, kernel, sort_every, tile):
    es = edge_particles3(dt=dt)
    log(f"edge 3d {name} dt={dt} kernel={kernel} sort_every={sort_every} tile={tile}")
    got, tr, st = _gpu(3, fields3, es.ens, dt, name, kernel, sort_every, tile)
    ref, rtr, _ = _oracle(3, dt, name, fields3, es.ens)
    _compare(3, got, tr, st, ref, rtr, f"edge 3d {name} dt={dt} k={kernel}", kernel,
             sort_every, RUNS[name][1])


def test_threshold_decisions_closed_form(fields2):
    """The switch at exact equality (strict '<' of Sec. 4.1: equality takes
    the full orbit), independent of the oracle: rho~/dl = f_rho for
    q/m = -1/2 with u = 0, B = 1 (j = 0), larger for j < 0; E/B = f_E at
    w = 1/2 (k = 32), larger for k < 32."""
    es = edge_particles(dt=1.0)
    _, tr, _ = _gpu(2, fields2, es.ens, 1.0, "switch", 1, 0, 0)
    want = np.array([1] * 9 + [0] * 8, dtype=np.uint8)
    assert np.array_equal(tr[0][es.groups["rho_edge"]], want)
    assert np.array_equal(tr[0][es.groups["e_edge"]], want)
    # B = 0 and E > B at x^n: the full orbit
    assert (tr[0][es.groups["in_zero"]] == 1).all()
    assert (tr[0][es.groups["in_e_gt_b"]] == 1).all()


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("kernel,sort_every", [(1, 0), (2, 1)])
def test_edge_mixed_threshold_groups(fields2, fields3, dim, kernel, sort_every):
    """The precision form on the threshold groups: binary32 switch ratios lie
    within 1e-4 of f_rho / f_E, the binary64 re-check decides, and with
    binary32-exact samples it must decide as the binary64 oracle."""
    from paper_2007_14401_amd import gcb
    es = edge_particles(dt=1.0) if dim == 2 else edge_particles3(dt=1.0)
    F = fields2 if dim == 2 else fields3
    tile = 16 if dim == 2 else 6
    got, tr, _ = _gpu(dim, F, es.ens, 1.0, "switch", kernel, sort_every, tile,
                      form=gcb.GCB_FORM_MIXED)
    _, rtr, _ = _oracle(dim, 1.0, "switch", F, es.ens)
    for g in ("rho_edge", "e_edge"):
        sl = es.groups[g]
        assert np.array_equal(tr[0][sl], rtr.numpy()[0][sl]), g
    # the rho group does not move (u = 0 in a uniform B without E): every
    # step repeats the first decision
    sl = es.groups["rho_edge"]
    assert np.array_equal(tr[:, sl], rtr.numpy()[:, sl])
