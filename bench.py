"""Benchmark: particle-steps/s of the coupled guiding-center/Boris push on one
MI355X, with the HBM roofline fraction of the push kernel and the CPU oracle
timed beside it.

Workload (default): a 4096 x 4096 periodic double Harris sheet with guide
field, tearing perturbation, inflow E and reconnection E_z at the X points
(fields in binary64, 805 MB); 1e7 electrons (half Maxwell-Juttner theta = 1,
half a Gamma^-2 power law to 1e4), about 70 % in the guiding-center regime;
binary64 plain path, curvature terms on, K = 4 fixed-point iterations,
cell-sorted every 4 steps, LDS-tiled kernel.  A step is one time step of the
whole population: cell sort (every 4th step), switch, per-regime queues,
Boris and guiding-center updates.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/sec at 1e7 particles (fwd, fwd+adjoint) + % HBM peak"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, AMD published
FP64_VECTOR_PEAK_TF = 78.6      # MI355X FP64 vector, AMD published
# Floating-point operations of one oracle step per particle and branch (K = 4,
# curvature terms on), counted by `python -m oracle.opcount`: every elementwise
# add, sub, mul, div, sqrt, floor, comparison and select of the definition.
FLOPS_BORIS = 287.0
FLOPS_GCA = 2216.0
# The same count for one step of the curved-spacetime scheme (K = 4), the
# switch part included.
FLOPS_GR_ORBIT = 1611.0
FLOPS_GR_GCA = 2218.0
# The same count for one step of the 3D scheme (trilinear gather, K = 4).
FLOPS_BORIS_3D = 528.0
FLOPS_GCA_3D = 4025.0

# Hardware-counter record of the binary64 push kernel (rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs, calibrated against a plain device copy); it is used only
# while the kernel sources still hash to the value it was taken with.
COUNTER_RECORD = os.path.join(ROOT, "profiles", "k_push_tiled_harris4096.md")
KERNEL_SOURCES = tuple(os.path.join("paper_2007_14401_amd", "csrc", f) for f in (
    "gcb_common.hpp", "gcb_access.hpp", "gcb_math.hpp", "gcb_queues.hpp",
    "gcb_push_kernels.hpp", "gcb_push_f64.hip", "gcb_push_f64_fast.hip", "gcb_push_mixed.hip",
    "gcb_sort.hip", "gcb_host.hip", "gcb_internal.h")) + (
    os.path.join("paper_2007_14401_amd", "build.py"),)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def push_bytes_per_step(n: int, nx: int, ny: int, form: int) -> int:
    """Algorithmic HBM bytes of one push launch: the state read and written once
    (x, y, xp, yp as binary64; u as binary64 or binary32; the status byte) plus
    the field grid read once (6 components per node)."""
    ub = 8 if form == 0 else 4
    fb = 8 if form == 0 else 4
    state = n * 2 * (4 * 8 + 3 * ub + 1)
    fields = nx * ny * 6 * fb
    return state + fields


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        h.update(rel.encode())
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_record(path: str = COUNTER_RECORD):
    """The `<!-- counters: {...} -->` line of a committed profile summary."""
    import re
    try:
        text = open(path).read()
    except OSError:
        return None
    m = re.search(r"<!-- counters: (\{.*?\}) -->", text)
    return json.loads(m.group(1)) if m else None


def measured_traffic(workload: str, n: int, sort_every: int, tile: int):
    """HBM bytes per launch of the binary64 push (a launch runs the steps
    between two sorts) from the counter record, or None when there is none for
    this launch or the kernel changed since."""
    rec = counter_record()
    if not rec:
        return None
    if (rec.get("sources_sha256") != kernel_sources_sha256() or rec.get("workload") != workload
            or rec.get("n") != n or rec.get("sort_every") != sort_every
            or rec.get("tile") != tile):
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def counter_limiter(workload: str, n: int, sort_every: int, tile: int):
    """What the committed counter record of the binary64 push says limits it
    (VALU busy share, waves per SIMD, traffic over algorithmic bytes), or
    None when the record is for another launch or the kernel changed."""
    rec = counter_record()
    if not rec or "limiter" not in rec:
        return None
    if (rec.get("sources_sha256") != kernel_sources_sha256() or rec.get("workload") != workload
            or rec.get("n") != n or rec.get("sort_every") != sort_every
            or rec.get("tile") != tile):
        return None
    return rec["limiter"]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(cfg, F, ens, budget_s: float = 20.0):
    """The CPU oracle (torch float64) on a bounded sample of the same workload:
    a random subset of the particles, pushed for up to the workload's step
    count or about `budget_s` seconds with all host threads, then a smaller
    subset on one thread."""
    import numpy as np
    import torch

    import oracle as O
    p = O.Params(dt=cfg.dt, c=cfg.c, f_rho=cfg.f_rho, f_E=cfg.f_E, curvature=True,
                 n_iter=cfg.n_iter, Lx=cfg.Lx, Ly=cfg.Ly, dl=math.sqrt(cfg.dx * cfg.dy))
    prov = O.GridFields(F, cfg.dx, cfg.dy, cfg.stagger)
    rng = np.random.default_rng(5)

    def run(n, budget):
        sub = ens.subset(np.sort(rng.choice(ens.n, n, replace=False)))
        st = O.State.from_numpy(sub)
        steps = 0
        t0 = time.perf_counter()
        while True:
            st, _, _ = O.step(prov, st, p)
            steps += 1
            el = time.perf_counter() - t0
            if el >= budget or steps >= cfg.steps:
                break
        return n * steps / el, steps, el

    threads = int(torch.get_num_threads())
    n = 60000
    v, steps, el = run(n, budget_s)
    torch.set_num_threads(1)
    try:
        n1 = 4000
        v1, steps1, el1 = run(n1, 0.25 * budget_s)
    finally:
        torch.set_num_threads(threads)
    return {"value": v, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_logical_cpus": os.cpu_count(),
            "sample": f"{n} random particles of the workload x {steps} steps "
                      f"({el:.1f} s, torch CPU float64, {threads} threads)",
            "single_thread": {"value": v1, "sample": f"{n1} particles x {steps1} steps "
                                                     f"({el1:.1f} s, 1 thread)"}}


def copy_bandwidth(dev, gib: float = 1.0, reps: int = 5) -> float:
    """Measured device-to-device copy rate (read + write bytes per second) of a
    gib-GiB buffer: the practical HBM ceiling beside the published peak."""
    import torch
    n = int(gib * (1 << 30)) // 8
    x = torch.empty(n, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    del x, y
    torch.cuda.empty_cache()
    return 2 * n * 8 / el / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--config", default="harris4096")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--kernel", type=int, default=0)
    ap.add_argument("--sort-every", type=int, default=10)
    ap.add_argument("--tile", type=int, default=20)
    ap.add_argument("--arith", choices=("fast", "exact"), default="fast",
                    help="binary64 arithmetic of the headline push: contracted "
                         "multiply-adds (fast, the production build) or the parity build")
    ap.add_argument("--mixed-tile", type=int, default=28)
    ap.add_argument("--mixed-sort-every", type=int, default=10,
                    help="cell-sort period of the mixed form (default: --sort-every)")
    ap.add_argument("--mixed-1e8-steps", type=int, default=20,
                    help="steps of the precision form at 1e8 particles (0: skip)")
    ap.add_argument("--f-rho", type=float, default=None)
    ap.add_argument("--f-E", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the Boris-only (f_rho = 0) and guiding-center-only "
                         "(f_rho = f_E = inf) runs of the headline push")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=100)
    ap.add_argument("--adjoint-sort-every", type=int, default=10,
                    help="in-place cell-sort period of the differentiable push")
    ap.add_argument("--adjoint-c4-steps", type=int, default=512)
    ap.add_argument("--adjoint3-steps", type=int, default=32)
    ap.add_argument("--no-gr", action="store_true")
    ap.add_argument("--gr-steps", type=int, default=40)
    ap.add_argument("--gr-warmup", type=int, default=4)
    ap.add_argument("--gr-sort-every", type=int, default=16)
    ap.add_argument("--no-frame", action="store_true")
    ap.add_argument("--no-mirror", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--d3-steps", type=int, default=40)
    ap.add_argument("--d3-warmup", type=int, default=4)
    ap.add_argument("--d3-sort-every", type=int, default=4)
    ap.add_argument("--d3-tile", type=int, default=4)
    ap.add_argument("--d3-kernel", type=int, default=0)
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    a = ap.parse_args()

    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}): the library pushes "
              "particles on a single GPU", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2007_14401_amd import gcb, state
    from workloads import make_config

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    over = {}
    if a.f_rho is not None:
        over["f_rho"] = a.f_rho
    if a.f_E is not None:
        over["f_E"] = a.f_E
    cfg = make_config(a.config, **over)
    n = cfg.n if a.n is None else a.n
    log(f"[bench] generating {cfg.name}: {cfg.nx}x{cfg.ny}, n={n}")
    F = cfg.fields()
    ens = cfg.particles(n=n)

    dev = torch.device("cuda:0")

    def time_form(form: int, fields_dtype: int, steps: int, warmup: int, ens_=None, **extra):
        """Time `steps` pushes of the whole population (ens_, else the
        workload's) in one form (extra: overrides of the push parameters)."""
        ctx = gcb.gcb_create(0)
        try:
            desc = gcb.grid_desc(cfg.nx, cfg.ny, cfg.dx, cfg.dy, cfg.stagger, fields_dtype)
            gcb.gcb_load_fields(ctx, desc, [F[0], F[1], F[2]], [F[3], F[4], F[5]])
            t = state.to_device(ens if ens_ is None else ens_, dev, form=form,
                                per_particle_qm=False)
            parts = gcb.particles(t)
            kw = dict(dt=cfg.dt, c=cfg.c, qm=cfg.qm, f_rho=cfg.f_rho, f_E=cfg.f_E,
                      n_iter=cfg.n_iter, form=form, sort_every=a.sort_every, kernel=a.kernel,
                      curvature=cfg.curvature, tile=a.tile)
            if form == gcb.GCB_FORM_F64:
                kw["arith"] = ARITH
            kw.update(extra)
            prm = gcb.params(**kw)
            log(f"[bench] form {form} {extra}: warmup {warmup} steps")
            st = gcb.gcb_push(ctx, parts, prm, warmup, want_stats=True)
            log(f"[bench] warmup stats {st}")
            gcb.gcb_set_timing(ctx, True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gcb.gcb_push(ctx, parts, prm, steps)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ms, cnt = gcb.gcb_get_timing(ctx)
            gcb.gcb_set_timing(ctx, False)
            log(f"[bench] form {form}: {steps} steps in {t1 - t0:.3f} s; kernel ms {ms} "
                f"launches {cnt}")
            st = gcb.gcb_push(ctx, parts, prm, 1, want_stats=True)
            torch.cuda.synchronize()
            del t
            # push time per step (a tiled launch runs the steps between two sorts)
            return {"wall": t1 - t0, "launches": cnt[gcb.GCB_TIMER_PUSH],
                    "push_ms": ms[gcb.GCB_TIMER_PUSH] / steps,
                    "sort_ms": ms[gcb.GCB_TIMER_SORT] / max(1, cnt[gcb.GCB_TIMER_SORT]),
                    "gca_frac": st["gca_steps"] / max(1, st["gca_steps"] + st["boris_steps"])}
        finally:
            gcb.gcb_destroy(ctx)
            torch.cuda.empty_cache()

    def time_fwd_adjoint(steps: int, checkpoint: int, wcfg=None, F=F, ens=ens):
        """Forward + reverse pass of the differentiable push (loss: mean final
        kinetic energy; gradients to the E/B grids and the initial state), on
        the benchmark workload or on `wcfg` with its fields F and particles ens."""
        from paper_2007_14401_amd import autograd as A
        cfg_ = cfg if wcfg is None else wcfg
        n_ = ens.n
        pctx = A.PushContext(0)
        try:
            Ft = torch.as_tensor(F, dtype=torch.float64, device=dev)
            E = Ft[:3].contiguous().requires_grad_(True)
            B = Ft[3:].contiguous().requires_grad_(True)
            del Ft
            names = ("x", "y", "xp", "yp", "ux", "uy", "uz")
            # initial positions cell-sorted (row-major cells), as the workload states;
            # the differentiable push sorts in place (keep_order), so the arrays
            # keep this order
            cell = (np.floor(ens.y / cfg_.dy).astype(np.int64) * cfg_.nx
                    + np.floor(ens.x / cfg_.dx).astype(np.int64))
            order = np.argsort(cell, kind="stable")
            st = {k: torch.as_tensor(getattr(ens, k)[order], dtype=torch.float64, device=dev)
                  .requires_grad_(True) for k in names}
            prm = gcb.params(dt=cfg_.dt, c=cfg_.c, qm=cfg_.qm, f_rho=cfg_.f_rho, f_E=cfg_.f_E,
                             curvature=cfg_.curvature, n_iter=cfg_.n_iter,
                             sort_every=a.adjoint_sort_every, tile=a.tile)
            # warm-up: two steps forward and backward
            out = A.push(E, B, *[st[k] for k in names], None, pctx, prm, 2, checkpoint)
            A.kinetic_energy(out[4], out[5], out[6], pctx, prm).backward()
            for v in list(st.values()) + [E, B]:
                v.grad = None
            gcb.gcb_set_timing(pctx.ctx, True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = A.push(E, B, *[st[k] for k in names], None, pctx, prm, steps, checkpoint)
            L = A.kinetic_energy(out[4], out[5], out[6], pctx, prm)
            L.backward()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ms, cnt = gcb.gcb_get_timing(pctx.ctx)
            gcb.gcb_set_timing(pctx.ctx, False)
            log(f"[bench] fwd+adjoint: {steps} steps in {t1 - t0:.3f} s; kernel ms {ms}")
            return {"value": n_ * steps / (t1 - t0), "unit": "particle-steps/s",
                    "workload": f"{cfg_.name}: {cfg_.nx}x{cfg_.ny}, {n_} particles",
                    "steps": steps, "checkpoint": checkpoint, "seconds": t1 - t0,
                    "forward_push_ms_per_step": ms[gcb.GCB_TIMER_PUSH] / max(1, steps),
                    "sort_ms_per_step": ms[gcb.GCB_TIMER_SORT] / max(1, steps),
                    "backward_ms_per_step": ms[gcb.GCB_TIMER_BACKWARD] / max(1, steps),
                    "sort_every": a.adjoint_sort_every, "tile": a.tile,
                    "kernel": "k_push_tiled in place (keep_order, parity binary64) + "
                              "k_adjoint_step + k_scatter_batch",
                    "loss": float(L.detach())}
        finally:
            pctx.close()
            torch.cuda.empty_cache()

    def time_fwd_adjoint3(steps: int, checkpoint: int):
        """Forward + reverse pass of the differentiable 3D push on the 3D
        workload (harris3d128, 1e7 particles; loss: mean final kinetic
        energy), initial positions cell-sorted (row-major cells)."""
        from paper_2007_14401_amd import autograd as A
        from workloads import make_config3
        c3 = make_config3("harris3d128")
        log(f"[bench] 3d fwd+adjoint: generating {c3.name}, n={c3.n}")
        F3 = c3.fields()
        e3 = c3.particles()
        pctx = A.PushContext3(0, (c3.dx, c3.dy, c3.dz), c3.stagger)
        try:
            Ft = torch.as_tensor(F3, dtype=torch.float64, device=dev)
            del F3
            E = Ft[:3].contiguous().requires_grad_(True)
            B = Ft[3:].contiguous().requires_grad_(True)
            del Ft
            names = ("x", "y", "z", "xp", "yp", "zp", "ux", "uy", "uz")
            cell = ((np.floor(e3.z / c3.dz).astype(np.int64) * c3.ny
                     + np.floor(e3.y / c3.dy).astype(np.int64)) * c3.nx
                    + np.floor(e3.x / c3.dx).astype(np.int64))
            order = np.argsort(cell, kind="stable")
            st = {k: torch.as_tensor(getattr(e3, k)[order], dtype=torch.float64, device=dev)
                  .requires_grad_(True) for k in names}
            prm = gcb.params(dt=c3.dt, c=c3.c, qm=c3.qm, f_rho=c3.f_rho, f_E=c3.f_E,
                             curvature=c3.curvature, n_iter=c3.n_iter,
                             sort_every=a.d3_sort_every, tile=a.d3_tile)
            out = A.push3(E, B, *[st[k] for k in names], None, pctx, prm, 2, checkpoint)
            A.kinetic_energy(out[6], out[7], out[8], pctx, prm).backward()
            for v in list(st.values()) + [E, B]:
                v.grad = None
            gcb.gcb_set_timing(pctx.ctx, True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = A.push3(E, B, *[st[k] for k in names], None, pctx, prm, steps, checkpoint)
            L = A.kinetic_energy(out[6], out[7], out[8], pctx, prm)
            L.backward()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ms, cnt = gcb.gcb_get_timing(pctx.ctx)
            gcb.gcb_set_timing(pctx.ctx, False)
            log(f"[bench] 3d fwd+adjoint: {steps} steps in {t1 - t0:.3f} s; kernel ms {ms}")
            return {"value": e3.n * steps / (t1 - t0), "unit": "particle-steps/s",
                    "workload": f"{c3.name}: {c3.nx}x{c3.ny}x{c3.nz}, {e3.n} particles",
                    "steps": steps, "checkpoint": checkpoint, "seconds": t1 - t0,
                    "forward_push_ms_per_step": ms[gcb.GCB_TIMER_PUSH] / max(1, steps),
                    "backward_ms_per_step": ms[gcb.GCB_TIMER_BACKWARD] / max(1, steps),
                    "sort_every": a.d3_sort_every, "tile": a.d3_tile,
                    "kernel": "k_push3_tiled in place (keep_order, parity binary64) + "
                              "k_adjoint3_step + k_scatter3_batch",
                    "loss": float(L)}
        finally:
            pctx.close()
            torch.cuda.empty_cache()

    def time_gr(steps: int, warmup: int, mixed: bool = False, arith=None):
        """Curved-spacetime push: Kerr a = 0.9, 512 x 512 (r, theta) grid,
        1e7 particles (the workload's own size), binary64 (the headline's
        arithmetic unless `arith` says otherwise) or the precision form."""
        if arith is None:
            arith = gcb.GCB_ARITH_EXACT if mixed else ARITH
        from workloads import make_gr_config
        gcfg = make_gr_config("grbh512")
        log(f"[bench] curved spacetime: generating {gcfg.name}, n={gcfg.n}")
        GF = gcfg.fields()
        ge = gcfg.particles()
        ctx = gcb.gcb_create(0)
        try:
            desc = gcb.gr_desc(gcfg.nr, gcfg.nth, gcfg.r_min, gcfg.r_max, gcfg.a,
                               gcb.GCB_F32 if mixed else gcb.GCB_F64)
            gcb.gcb_load_fields_gr(ctx, desc, [GF[0], GF[1], GF[2]], [GF[3], GF[4], GF[5]])
            t = {k: torch.as_tensor(getattr(ge, k), device=dev,
                                    dtype=torch.float32 if (mixed and k[0] == "u")
                                    else torch.float64)
                 for k in ("r", "th", "ph", "ur", "uth", "uph")}
            t["status"] = torch.zeros(ge.n, dtype=torch.uint8, device=dev)
            t["id"] = torch.arange(ge.n, dtype=torch.int32, device=dev)
            parts = gcb.gr_particles(t)
            prm = gcb.params(dt=gcfg.dt, c=1.0, qm=gcfg.qm, f_rho=gcfg.f_rho, f_E=gcfg.f_E,
                             n_iter=gcfg.n_iter, sort_every=a.gr_sort_every,
                             form=gcb.GCB_FORM_MIXED if mixed else gcb.GCB_FORM_F64,
                             arith=arith)
            st = gcb.gcb_push_gr(ctx, parts, prm, warmup, want_stats=True)
            frac = st["gca_steps"] / max(1, st["gca_steps"] + st["boris_steps"])
            gcb.gcb_set_timing(ctx, True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gcb.gcb_push_gr(ctx, parts, prm, steps)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ms, cnt = gcb.gcb_get_timing(ctx)
            gcb.gcb_set_timing(ctx, False)
            kms = ms[gcb.GCB_TIMER_PUSH] / steps
            sort_ms = ms[gcb.GCB_TIMER_SORT] / max(1, cnt[gcb.GCB_TIMER_SORT])
            fl = FLOPS_GR_GCA * frac + FLOPS_GR_ORBIT * (1.0 - frac)
            tf = fl * ge.n / (kms * 1e-3) / 1e12
            log(f"[bench] curved spacetime: {steps} steps in {t1 - t0:.3f} s")
            return {"value": ge.n * steps / (t1 - t0), "unit": "particle-steps/s",
                    "workload": f"{gcfg.name}: Kerr a={gcfg.a} Kerr-Schild, "
                                f"{gcfg.nr}x{gcfg.nth} (r, theta) grid r in "
                                f"[{gcfg.r_min}, {gcfg.r_max}], split monopole with an "
                                f"equatorial current sheet, {ge.n} particles, "
                                + ("binary32 bulk, binary64 positions" if mixed else
                                   "binary64, " + ("production" if arith == gcb.GCB_ARITH_FAST
                                                   else "exact") + " arithmetic"),
                    "steps": steps, "ms_per_step": (t1 - t0) * 1e3 / steps,
                    "kernel_ms_per_step": kms, "gca_fraction": frac,
                    "sort_every": a.gr_sort_every, "sort_ms_per_sort": sort_ms,
                    "algorithmic_flops_per_particle_step": fl,
                    "alu_achieved_TFLOPs": tf, "alu_frac": tf / FP64_VECTOR_PEAK_TF,
                    "kernel": "k_gr_push (regime queues per workgroup, one lane per "
                              "particle for the 8 steps of a launch, blocks in XCD order), "
                              "(r, theta) tile sort every sort_every steps"}
        finally:
            gcb.gcb_destroy(ctx)
            torch.cuda.empty_cache()

    def time_3d(steps: int, warmup: int, mixed: bool = False, arith=None):
        """3D push: 128^3 periodic double Harris sheet with oblique tearing,
        1e7 particles (the workload's own size), binary64 (production
        arithmetic unless `arith` says otherwise) or the mixed form."""
        from workloads import make_config3
        c3 = make_config3("harris3d128")
        log(f"[bench] 3d: generating {c3.name}, n={c3.n}")
        F3 = c3.fields()
        e3 = c3.particles()
        form = gcb.GCB_FORM_MIXED if mixed else gcb.GCB_FORM_F64
        ctx = gcb.gcb_create(0)
        try:
            desc = gcb.grid3_desc(c3.nx, c3.ny, c3.nz, c3.dx, c3.dy, c3.dz, c3.stagger,
                                  gcb.GCB_F32 if mixed else gcb.GCB_F64)
            gcb.gcb_load_fields_3d(ctx, desc, [F3[0], F3[1], F3[2]], [F3[3], F3[4], F3[5]])
            del F3
            t = state.to_device(e3, dev, form=form, per_particle_qm=False)
            parts = gcb.particles3(t)
            prm = gcb.params(dt=c3.dt, c=c3.c, qm=c3.qm, f_rho=c3.f_rho, f_E=c3.f_E,
                             curvature=c3.curvature, n_iter=c3.n_iter, form=form,
                             sort_every=a.d3_sort_every, kernel=a.d3_kernel, tile=a.d3_tile,
                             arith=(gcb.GCB_ARITH_EXACT if mixed else
                                    (ARITH if arith is None else arith)))
            st = gcb.gcb_push_3d(ctx, parts, prm, warmup, want_stats=True)
            frac = st["gca_steps"] / max(1, st["gca_steps"] + st["boris_steps"])
            halo = st["halo_misses"] / max(1, st["gca_steps"] + st["boris_steps"])
            gcb.gcb_set_timing(ctx, True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gcb.gcb_push_3d(ctx, parts, prm, steps)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ms, cnt = gcb.gcb_get_timing(ctx)
            gcb.gcb_set_timing(ctx, False)
            kms = ms[gcb.GCB_TIMER_PUSH] / steps
            sort_ms = ms[gcb.GCB_TIMER_SORT] / max(1, cnt[gcb.GCB_TIMER_SORT])
            fl = FLOPS_GCA_3D * frac + FLOPS_BORIS_3D * (1.0 - frac)
            tf = fl * e3.n / (kms * 1e-3) / 1e12
            log(f"[bench] 3d: {steps} steps in {t1 - t0:.3f} s; kernel ms {ms}")
            del t
            return {"value": e3.n * steps / (t1 - t0), "unit": "particle-steps/s",
                    "workload": f"{c3.name}: {c3.nx}x{c3.ny}x{c3.nz} periodic double Harris "
                                f"sheet (guide 0.1 B0, oblique tearing, inflow E, reconnection "
                                f"Ez along the X lines), 3D Yee lattice, trilinear gather, "
                                f"{e3.n} electrons MJ theta=1 + Gamma^-2 power law to 1e4, "
                                + ("binary32 bulk, binary64 positions" if mixed
                                   else "binary64"),
                    "steps": steps, "ms_per_step": (t1 - t0) * 1e3 / steps,
                    "kernel_ms_per_step": kms, "gca_fraction": frac,
                    "halo_miss_fraction": halo,
                    "sort_every": a.d3_sort_every, "tile": a.d3_tile,
                    "sort_ms_per_sort": sort_ms,
                    "algorithmic_flops_per_particle_step": fl,
                    "alu_achieved_TFLOPs": tf, "alu_frac": tf / FP64_VECTOR_PEAK_TF,
                    "kernel": ["auto", "k_push3_global", "k_push3_tiled"][a.d3_kernel]}
        finally:
            gcb.gcb_destroy(ctx)
            torch.cuda.empty_cache()

    ARITH = gcb.GCB_ARITH_FAST if a.arith == "fast" else gcb.GCB_ARITH_EXACT
    r64 = time_form(gcb.GCB_FORM_F64, gcb.GCB_F64, a.steps, a.warmup)
    wall, push_ms, sort_ms, gca_frac = r64["wall"], r64["push_ms"], r64["sort_ms"], r64["gca_frac"]
    # a launch runs the steps between two sorts: the roofline is taken per
    # launch (algorithmic bytes and flops of its particle-steps over its
    # average HIP-event duration), which is the same ratio as per step
    steps_per_launch = a.steps / max(1, r64["launches"])
    launch_ms = push_ms * steps_per_launch
    bytes_step = push_bytes_per_step(n, cfg.nx, cfg.ny, 0)
    bytes_launch = bytes_step * steps_per_launch
    achieved = bytes_step / (push_ms * 1e-3) / 1e9
    value = n * a.steps / wall
    flops = FLOPS_GCA * gca_frac + FLOPS_BORIS * (1.0 - gca_frac)
    alu_tf = flops * n / (push_ms * 1e-3) / 1e12
    traffic = measured_traffic(cfg.name, n, a.sort_every, a.tile)

    def roof(flops_pp: float, kms: float, nbytes: float) -> dict:
        """Both roofs of a push: algorithmic flops and bytes per step over its
        HIP-event time per step, and which roof the arithmetic intensity
        puts it under (the ridge of the binary64 vector peak and the HBM
        peak: 78.6 TFLOP/s / 8 TB/s = 9.8 flop/B)."""
        tf = flops_pp * n / (kms * 1e-3) / 1e12
        gbs = nbytes / (kms * 1e-3) / 1e9
        ai = flops_pp * n / nbytes
        ridge = FP64_VECTOR_PEAK_TF * 1e12 / (HBM_PEAK_GBS * 1e9)
        return {"kernel_ms": kms, "algorithmic_flops_per_particle_step": flops_pp,
                "algorithmic_bytes_per_step": nbytes,
                "arithmetic_intensity_flop_per_byte": ai,
                "bound_by_intensity": "hbm" if ai < ridge else "alu",
                "alu_achieved_TFLOPs": tf, "alu_frac": tf / FP64_VECTOR_PEAK_TF,
                "hbm_achieved_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}

    hroof = roof(flops, push_ms, bytes_step)
    hbm_bound = hroof["bound_by_intensity"] == "hbm"
    forms = {}
    if a.arith == "fast":
        # the same push in the parity build (no contraction), for comparison
        rx = time_form(gcb.GCB_FORM_F64, gcb.GCB_F64, a.steps, a.warmup,
                       arith=gcb.GCB_ARITH_EXACT)
        forms["f64_exact_arith"] = {
            "workload": f"{cfg.name}, binary64 without contraction (bit for bit with the "
                        f"oracle)", "value": n * a.steps / rx["wall"],
            "unit": "particle-steps/s", "kernel_ms": rx["push_ms"],
            "headline_over_this": value / (n * a.steps / rx["wall"])}
    if not a.no_legs:
        # the two branches of the coupled step on their own (the same
        # particles and kernel): every particle Boris, every particle guiding
        # center
        for leg, kw in (("boris_only", dict(f_rho=0.0)),
                        ("gca_only", dict(f_rho=math.inf, f_E=math.inf))):
            r = time_form(gcb.GCB_FORM_F64, gcb.GCB_F64, a.steps, a.warmup, **kw)
            fl = FLOPS_GCA * r["gca_frac"] + FLOPS_BORIS * (1.0 - r["gca_frac"])
            forms[leg] = {"workload": f"{cfg.name}, binary64, " + ", ".join(
                              f"{k}={v}" for k, v in kw.items()),
                          "value": n * a.steps / r["wall"], "unit": "particle-steps/s",
                          "gca_fraction": r["gca_frac"],
                          **roof(fl, r["push_ms"], bytes_step)}
    if not a.no_mixed:
        # the binary32 window is half the size: the mixed form's best tile is larger
        mse = a.mixed_sort_every if a.mixed_sort_every else a.sort_every
        rm = time_form(gcb.GCB_FORM_MIXED, gcb.GCB_F32, a.steps, a.warmup, tile=a.mixed_tile,
                       sort_every=mse)
        bm = push_bytes_per_step(n, cfg.nx, cfg.ny, 1)
        forms["mixed"] = {
            "value": n * a.steps / rm["wall"], "unit": "particle-steps/s",
            "ms_per_step": rm["wall"] * 1e3 / a.steps, "kernel_ms": rm["push_ms"],
            "sort_ms_per_sort": rm["sort_ms"],
            "hbm_achieved_GBs": bm / (rm["push_ms"] * 1e-3) / 1e9,
            "hbm_frac": bm / (rm["push_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "algorithmic_bytes_per_step": bm,
            "speedup_vs_f64": (n * a.steps / rm["wall"]) / value,
            "tile": a.mixed_tile, "sort_every": mse,
            "dtype": "f32 bulk, f64 positions"}
        if a.mixed_1e8_steps > 0 and a.config == "harris4096" and a.n is None:
            # the precision form's second size: 1e8 particles on the same fields
            n8 = 100_000_000
            log(f"[bench] mixed form at {n8} particles: generating")
            ens8 = cfg.particles(n=n8)
            r8 = time_form(gcb.GCB_FORM_MIXED, gcb.GCB_F32, a.mixed_1e8_steps, 2, ens_=ens8,
                           tile=a.mixed_tile, sort_every=mse)
            del ens8
            b8 = push_bytes_per_step(n8, cfg.nx, cfg.ny, 1)
            forms["mixed_1e8"] = {
                "workload": "harris4096 fields, 100000000 particles of the same mix",
                "value": n8 * a.mixed_1e8_steps / r8["wall"], "unit": "particle-steps/s",
                "steps": a.mixed_1e8_steps,
                "ms_per_step": r8["wall"] * 1e3 / a.mixed_1e8_steps, "kernel_ms": r8["push_ms"],
                "hbm_achieved_GBs": b8 / (r8["push_ms"] * 1e-3) / 1e9,
                "hbm_frac": b8 / (r8["push_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "algorithmic_bytes_per_step": b8,
                "tile": a.mixed_tile, "sort_every": mse,
                "dtype": "f32 bulk, f64 positions"}

    if not a.no_gr:
        forms["gr"] = time_gr(a.gr_steps, a.gr_warmup)
        if a.arith == "fast":
            forms["gr_exact_arith"] = time_gr(a.gr_steps, a.gr_warmup,
                                              arith=gcb.GCB_ARITH_EXACT)
        if not a.no_mixed:
            forms["gr_mixed"] = time_gr(a.gr_steps, a.gr_warmup, mixed=True)
            forms["gr_mixed"]["speedup_vs_gr_f64"] = (forms["gr_mixed"]["value"]
                                                      / forms["gr"]["value"])

    if not a.no_frame:
        # the exact guiding-center frame against the reduced one, both with the
        # zero-curvature scheme
        fr = {}
        for name, frame in (("reduced", gcb.GCB_FRAME_REDUCED), ("exact", gcb.GCB_FRAME_EXACT)):
            r = time_form(gcb.GCB_FORM_F64, gcb.GCB_F64, a.steps, a.warmup, curvature=0,
                          frame=frame)
            fr[name] = {"value": n * a.steps / r["wall"], "kernel_ms": r["push_ms"],
                        "gca_fraction": r["gca_frac"]}
        forms["frame_no_curvature"] = {
            "workload": f"{cfg.name}, binary64, curvature terms off (Sec. 2.2.1)",
            "unit": "particle-steps/s", "reduced": fr["reduced"], "exact": fr["exact"],
            "exact_over_reduced": fr["exact"]["value"] / fr["reduced"]["value"]}
        # the exact frame with the curvature scheme (gradient of b* through E
        # and B) against the headline, the reduced frame with curvature
        r = time_form(gcb.GCB_FORM_F64, gcb.GCB_F64, a.steps, a.warmup, curvature=1,
                      frame=gcb.GCB_FRAME_EXACT)
        forms["frame_exact_curvature"] = {
            "workload": f"{cfg.name}, binary64, exact frame with the curvature scheme",
            "unit": "particle-steps/s", "value": n * a.steps / r["wall"],
            "kernel_ms": r["push_ms"], "gca_fraction": r["gca_frac"],
            "over_headline": n * a.steps / r["wall"] / value}

    if not a.no_mirror:
        # the mirror force and grad-B drift (their own kernel instance) on the
        # benchmark workload, binary64, curvature scheme
        r = time_form(gcb.GCB_FORM_F64, gcb.GCB_F64, a.steps, a.warmup, mirror=1)
        forms["mirror"] = {
            "workload": f"{cfg.name}, binary64, curvature scheme with the mirror terms",
            "unit": "particle-steps/s", "value": n * a.steps / r["wall"],
            "kernel_ms": r["push_ms"], "gca_fraction": r["gca_frac"],
            "over_headline": n * a.steps / r["wall"] / value}

    if not a.no_3d:
        forms["d3"] = time_3d(a.d3_steps, a.d3_warmup)
        forms["d3_exact_arith"] = time_3d(a.d3_steps, a.d3_warmup, arith=gcb.GCB_ARITH_EXACT)
        if not a.no_mixed:
            forms["d3_mixed"] = time_3d(a.d3_steps, a.d3_warmup, mixed=True)
            forms["d3_mixed"]["speedup_vs_d3_f64"] = (forms["d3_mixed"]["value"]
                                                      / forms["d3"]["value"])

    if not a.no_adjoint:
        forms["fwd_adjoint"] = time_fwd_adjoint(a.adjoint_steps, 32)
        forms["fwd_adjoint"]["speed_vs_f64_forward"] = forms["fwd_adjoint"]["value"] / value
        if a.adjoint_c4_steps > 0:
            # the differentiation workload as stated: 1024^2 grid, 1e6
            # particles, 512 steps, a checkpoint every 32 steps
            c4 = make_config("harris1024")
            log(f"[bench] differentiation workload {c4.name}: n={c4.n}")
            forms["fwd_adjoint_c4"] = time_fwd_adjoint(a.adjoint_c4_steps, 32, wcfg=c4,
                                                       F=c4.fields(), ens=c4.particles())
        if a.adjoint3_steps > 0 and not a.no_3d:
            forms["fwd_adjoint_3d"] = time_fwd_adjoint3(a.adjoint3_steps, 32)

    copy_gbs = copy_bandwidth(dev)
    if a.copy_calib:
        x = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": wall * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.nx}x{cfg.ny} periodic double Harris sheet "
                               f"(guide 0.1 B0, tearing, inflow E, reconnection Ez at X points),"
                               f" {n} electrons MJ theta=1 + Gamma^-2 power law to 1e4, "
                               f"binary64 plain path ({a.arith} arithmetic), curvature on, K={cfg.n_iter}",
                   "particles": n, "grid": [cfg.nx, cfg.ny], "form": "f64",
                   "arith": a.arith,
                   "kernel": ["auto", "global", "tiled"][a.kernel],
                   "sort_every": a.sort_every, "tile": a.tile,
                   "gca_fraction": round(gca_frac, 4)},
        # The roof is the one the push's arithmetic intensity (algorithmic flops
        # per algorithmic byte) puts it under: below the ridge point of the
        # binary64 vector peak and the HBM peak it is HBM.  Both fractions are
        # given; the forward target is 60 % of the HBM peak.
        "roofline": {"bound": "hbm" if hbm_bound else "alu",
                     "achieved": achieved if hbm_bound else alu_tf,
                     "peak": HBM_PEAK_GBS if hbm_bound else FP64_VECTOR_PEAK_TF,
                     "unit": "GB/s" if hbm_bound else "TFLOP/s",
                     "frac": (achieved / HBM_PEAK_GBS) if hbm_bound
                             else (alu_tf / FP64_VECTOR_PEAK_TF),
                     "traffic": traffic,
                     "kernel": ("kern_fast::" if a.arith == "fast" else "kern::")
                               + ("k_push_tiled<double, double, true, 3, 0, false>"
                                  if a.kernel != 1
                                  else "k_push_global<double, double, true, 0, false>"),
                     "kernel_ms": launch_ms,
                     "kernel_ms_per_step": push_ms,
                     "steps_per_launch": steps_per_launch,
                     "algorithmic_flops_per_particle_step": flops,
                     "algorithmic_bytes_per_particle_step": bytes_step / n,
                     "algorithmic_flops_per_launch": flops * n * steps_per_launch,
                     "arithmetic_intensity_flop_per_byte": hroof[
                         "arithmetic_intensity_flop_per_byte"],
                     "alu_achieved_TFLOPs": alu_tf, "alu_peak_TFLOPs": FP64_VECTOR_PEAK_TF,
                     "alu_frac": alu_tf / FP64_VECTOR_PEAK_TF,
                     "hbm_achieved_GBs": achieved, "hbm_peak_GBs": HBM_PEAK_GBS,
                     "hbm_copy_measured_GBs": copy_gbs,
                     "hbm_frac": achieved / HBM_PEAK_GBS,
                     "hbm_target_frac": 0.6,
                     "hbm_frac_of_target": achieved / HBM_PEAK_GBS / 0.6,
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "traffic_over_algorithmic": (traffic / bytes_launch) if traffic else None,
                     "limiter": counter_limiter(cfg.name, n, a.sort_every, a.tile)},
        "sort_ms_per_sort": sort_ms,
        "forms": forms,
    }
    if not a.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(cfg, F, ens)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
