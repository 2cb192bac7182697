"""Loss of the differentiation workload and its oracle gradient (TEST INFRASTRUCTURE).

The loss is the mean kinetic energy per unit mass of the final state,
L = (1/N) sum_p (Gamma_p - 1) c^2 with Gamma_p = sqrt(1 + u_p^2/c^2).

`push_gradients` differentiates the oracle's own multi-step push by
reverse-mode automatic differentiation (torch autograd, float64, CPU).  The
switch decision is a comparison, so it carries no derivative: gradients are
those of the branch each particle actually took, i.e. with the switch held
fixed along the forward path.
"""
from __future__ import annotations

import torch

from .ieee import sqrt

from .fields import GridFields
from .fields3d import GridFields3
from .pusher import Params, State, push
from .pusher3d import Params3, State3, push3

F64 = torch.float64


def kinetic_energy(ux, uy, uz, c: float):
    g = sqrt(1.0 + ((ux * ux + uy * uy) + uz * uz) * (1.0 / (c * c)))
    return torch.mean((g - 1.0) * (c * c))


def push_gradients(F, dx, dy, stagger, st0: State, p: Params, n_steps: int):
    """Gradients of the final mean kinetic energy.

    Returns a dict with the loss, dL/dF (shape of F), dL/d(x0, y0, xp0, yp0,
    ux0, uy0, uz0) and the switch trace of the forward pass.
    """
    Ft = torch.as_tensor(F, dtype=F64).clone().requires_grad_(True)
    names = ("x", "y", "xp", "yp", "ux", "uy", "uz")
    leaves = {k: getattr(st0, k).clone().requires_grad_(True) for k in names}
    st = State(**leaves, qm=st0.qm.clone(), status=st0.status.clone())
    prov = GridFields(Ft, dx, dy, stagger)
    out, trace, _ = push(prov, st, p, n_steps, trace=True)
    L = kinetic_energy(out.ux, out.uy, out.uz, p.c)
    grads = torch.autograd.grad(L, [Ft] + [leaves[k] for k in names],
                                allow_unused=True)
    res = {"loss": float(L.detach()), "dF": grads[0], "trace": trace,
           "final": out}
    for k, g in zip(names, grads[1:]):
        res["d" + k] = torch.zeros_like(leaves[k]) if g is None else g
    return res


def push_gradients3(F, dx, dy, dz, stagger, st0: State3, p: Params3, n_steps: int):
    """The 3D counterpart of `push_gradients`: F has shape (6, nz, ny, nx);
    returns the loss, dL/dF and dL/d(x0, y0, z0, xp0, yp0, zp0, ux0, uy0, uz0)
    and the switch trace."""
    Ft = torch.as_tensor(F, dtype=F64).clone().requires_grad_(True)
    names = ("x", "y", "z", "xp", "yp", "zp", "ux", "uy", "uz")
    leaves = {k: getattr(st0, k).clone().requires_grad_(True) for k in names}
    st = State3(**leaves, qm=st0.qm.clone(), status=st0.status.clone())
    prov = GridFields3(Ft, dx, dy, dz, stagger)
    out, trace, _ = push3(prov, st, p, n_steps, trace=True)
    L = kinetic_energy(out.ux, out.uy, out.uz, p.c)
    grads = torch.autograd.grad(L, [Ft] + [leaves[k] for k in names], allow_unused=True)
    res = {"loss": float(L.detach()), "dF": grads[0], "trace": trace, "final": out}
    for k, g in zip(names, grads[1:]):
        res["d" + k] = torch.zeros_like(leaves[k]) if g is None else g
    return res
