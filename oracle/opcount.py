"""Count the floating-point operations of one oracle step per particle
(TEST INFRASTRUCTURE; a script that calls only the oracle).

Every elementwise torch arithmetic call made by the oracle is intercepted and
charged (number of output elements) x (flops per element): add, sub, mul, div,
sqrt, neg, abs, floor, comparisons and where/maximum each count as one
operation per element; integer index arithmetic is not counted.  Running one
step with the switch forced to one branch (f_rho = 0: every particle Boris;
f_rho = f_E = inf: every particle guiding center) and dividing by the number
of particles gives the per-branch counts used for the arithmetic roofline.

    python -m oracle.opcount
"""
from __future__ import annotations

import math

import numpy as np
import torch
from torch.overrides import TorchFunctionMode

from workloads import make_config

from .fields import GridFields
from .pusher import Params, State, step

_ARITH = {
    "add", "__add__", "__radd__", "sub", "__sub__", "__rsub__", "mul", "__mul__",
    "__rmul__", "div", "__truediv__", "__rtruediv__", "true_divide", "sqrt", "neg",
    "__neg__", "abs", "floor", "maximum", "where", "lt", "le", "gt", "ge", "eq", "ne",
    "__lt__", "__le__", "__gt__", "__ge__", "__eq__", "__ne__", "remainder",
}


class _Count(TorchFunctionMode):
    def __init__(self):
        super().__init__()
        self.flops = 0
        self.by = {}

    def __torch_function__(self, func, types, args=(), kwargs=None):
        out = func(*args, **(kwargs or {}))
        name = getattr(func, "__name__", "")
        if name in _ARITH and isinstance(out, torch.Tensor) and out.is_floating_point():
            self.flops += out.numel()
            self.by[name] = self.by.get(name, 0) + out.numel()
        elif name in _ARITH and isinstance(out, torch.Tensor) and out.dtype == torch.bool:
            # comparisons on floating inputs
            if any(isinstance(a, torch.Tensor) and a.is_floating_point() for a in args):
                self.flops += out.numel()
                self.by[name] = self.by.get(name, 0) + out.numel()
        return out


def count(cfg_name="harris4096", n=4096, **over):
    cfg = make_config(cfg_name)
    F = cfg.fields()
    ens = cfg.particles(n=n)
    p = Params(dt=cfg.dt, c=cfg.c, f_rho=cfg.f_rho, f_E=cfg.f_E, curvature=True,
               n_iter=cfg.n_iter, Lx=cfg.Lx, Ly=cfg.Ly, dl=math.sqrt(cfg.dx * cfg.dy))
    for k, v in over.items():
        setattr(p, k, v)
    prov = GridFields(F, cfg.dx, cfg.dy, cfg.stagger)
    st = State.from_numpy(ens)
    # the sqrt of the oracle goes through numpy; count it explicitly
    import oracle.ieee as ieee
    orig = ieee.sqrt
    calls = {"n": 0}

    def counting_sqrt(x):
        calls["n"] += x.numel()
        return orig(x)
    ieee.sqrt = counting_sqrt
    import oracle.pusher as pusher
    pusher.sqrt = counting_sqrt
    try:
        with _Count() as c:
            _, S, _ = step(prov, st, p)
    finally:
        ieee.sqrt = orig
        pusher.sqrt = orig
    return (c.flops + calls["n"]) / n, c.by, calls["n"] / n


def count3(cfg_name="harris3d128", n=4096, **over):
    """The same count for one step of the 3D oracle."""
    import oracle.pusher as pusher
    import oracle.pusher3d as pusher3d
    from workloads import make_config3
    from .fields3d import GridFields3
    cfg = make_config3(cfg_name)
    F = cfg.fields()
    ens = cfg.particles(n=n)
    p = pusher3d.Params3(dt=cfg.dt, c=cfg.c, f_rho=cfg.f_rho, f_E=cfg.f_E, curvature=True,
                         n_iter=cfg.n_iter, Lx=cfg.Lx, Ly=cfg.Ly, Lz=cfg.Lz, dl=cfg.dl)
    for k, v in over.items():
        setattr(p, k, v)
    prov = GridFields3(F, cfg.dx, cfg.dy, cfg.dz, cfg.stagger)
    st = pusher3d.State3.from_numpy(ens)
    import oracle.ieee as ieee
    orig = ieee.sqrt
    calls = {"n": 0}

    def counting_sqrt(x):
        calls["n"] += x.numel()
        return orig(x)
    pusher.sqrt = pusher3d.sqrt = counting_sqrt
    try:
        with _Count() as c:
            pusher3d.step3(prov, st, p)
    finally:
        pusher.sqrt = pusher3d.sqrt = orig
    return (c.flops + calls["n"]) / n


def count_gr(cfg_name="grbh512", n=4096):
    """Per-branch operations of one curved-spacetime step: the switch part
    (metric, gather and switch at x^n) plus one branch, per particle."""
    import oracle.gr as gr
    from workloads import make_gr_config
    cfg = make_gr_config(cfg_name)
    F = cfg.fields()
    e = cfg.particles(n=n)
    grid = gr.GRGrid(F, cfg.r_min, cfg.r_max)
    met = gr.KerrSchild(cfg.a)
    p = gr.GRParams(dt=cfg.dt, f_rho=cfg.f_rho, f_E=cfg.f_E, n_iter=cfg.n_iter)
    st = gr.GRState.from_numpy(e)
    dl = gr.cell_lengths(met, grid)
    x = (st.r, st.th, st.ph)
    u = (st.ur, st.uth, st.uph)
    import oracle.ieee as ieee
    orig = ieee.sqrt
    calls = {"n": 0}

    def counting_sqrt(v):
        calls["n"] += v.numel()
        return orig(v)
    gr.sqrt = counting_sqrt
    out = {}
    try:
        def switch_part():
            ci, cj, _, _ = grid.cell(x[0], x[1])
            return gr.switch_gca(met.at(x[0], x[1]), *grid.sample(x[0], x[1]), u, st.qm,
                                 dl[cj, ci], p)

        for name, fn in (("switch", switch_part),
                         ("full orbit", lambda: gr.greom_step(met, grid, x, u, st.qm, p)),
                         ("guiding center", lambda: gr.grgca_step(met, grid, x, u, st.qm, p))):
            calls["n"] = 0
            with _Count() as c:
                fn()
            out[name] = ((c.flops + calls["n"]) / n, calls["n"] / n)
    finally:
        gr.sqrt = orig
    return out


def main():
    b, _, bs = count(f_rho=0.0)
    g, by, gs = count(f_rho=math.inf, f_E=math.inf)
    print(f"Boris branch:           {b:8.1f} flops/particle-step ({bs:.1f} sqrt)")
    print(f"Guiding-center branch:  {g:8.1f} flops/particle-step ({gs:.1f} sqrt), K=4, curvature")
    g3, _, _ = count(f_rho=math.inf, f_E=math.inf, n_iter=3)
    print(f"Guiding-center, K=3:    {g3:8.1f}")
    b3 = count3(f_rho=0.0)
    g3d = count3(f_rho=math.inf, f_E=math.inf)
    print(f"3D Boris branch:        {b3:8.1f} flops/particle-step")
    print(f"3D guiding-center:      {g3d:8.1f} flops/particle-step, K=4, curvature")
    gr_counts = count_gr()
    sw = gr_counts["switch"][0]
    for k in ("full orbit", "guiding center"):
        f, sq = gr_counts[k]
        print(f"curved spacetime, {k:15s} {sw + f:8.1f} flops/particle-step "
              f"(switch {sw:.1f} + branch {f:.1f}; {sq:.1f} sqrt in the branch), K=4")


if __name__ == "__main__":
    main()
