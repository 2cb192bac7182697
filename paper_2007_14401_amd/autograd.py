"""torch.autograd wrappers of the push (2D and 3D) and of the kinetic-energy loss.

GcbPush runs n_steps binary64 pushes through libgcb in segments of
`checkpoint` steps, keeping only each segment's start state; its backward
walks the segments in reverse and calls gcb_push_backward on each, which
recomputes the segment's forward steps and applies the hand-written adjoint
with the switch decisions held at their forward values.  Gradients reach the
E and B grids (accumulated in binary32 on the device, returned as float64)
and the initial state (x, y, xp, yp, u).

GcbPush3 / push3 do the same for the 3D push with gcb_push_backward_3d
(state x, y, z, xp, yp, zp, u; fields of shape (3, nz, ny, nx)).

KineticEnergy is the mean (Gamma - 1) c^2 of a state, computed by the
library's reduction kernel; its backward uses dL/du = u/(n Gamma).

A context holds one set of fields at a time.  Each forward records the
context's load generation and keeps E and B; a backward that finds other
fields loaded (a second forward on the same context ran in between, e.g. one
of a finite-difference pair) loads its own again before recomputing.

Argument marshalling and segment bookkeeping only: every step of the push and
of its derivative runs in the library's kernels.  The 2D push sorts in place
(gcb_params keep_order), so the arrays keep their order; so does the 3D push.
Forward and recomputation use the parity arithmetic, so they agree bit for
bit whatever kernel runs them.
"""
from __future__ import annotations

import torch

from . import gcb

_NAMES = ("x", "y", "xp", "yp", "ux", "uy", "uz")


class PushContext:
    """A libgcb context with binary64 fields taken from device tensors."""

    def __init__(self, device: int = 0):
        self.ctx = gcb.gcb_create(device)
        self.generation = 0   # incremented by every load

    def load(self, E: torch.Tensor, B: torch.Tensor, dx=1.0, dy=1.0,
             stagger=gcb.YEE_STAGGER):
        ny, nx = int(E.shape[1]), int(E.shape[2])
        desc = gcb.grid_desc(nx, ny, dx, dy, stagger, gcb.GCB_F64)
        Ec = [E[i].detach().contiguous() for i in range(3)]
        Bc = [B[i].detach().contiguous() for i in range(3)]
        gcb.gcb_load_fields(self.ctx, desc, Ec, Bc, src=gcb.GCB_DEVICE)
        torch.cuda.current_stream().synchronize()
        self.shape = (ny, nx)
        self.generation += 1

    def close(self):
        if self.ctx is not None:
            gcb.gcb_destroy(self.ctx)
            self.ctx = None


def _reload_if_replaced(ctx, pctx):
    """Load the fields of this graph's forward again if another load has
    replaced them on the shared context since."""
    if pctx.generation != ctx.generation:
        E, B = ctx.saved_tensors
        pctx.load(E, B)
        ctx.generation = pctx.generation


def _parts(st: dict, qm):
    d = dict(st)
    d["qm"] = qm
    d["id"] = None
    return gcb.particles(d)


class GcbPush(torch.autograd.Function):
    @staticmethod
    def forward(ctx, E, B, x, y, xp, yp, ux, uy, uz, qm, pctx: PushContext, prm,
                n_steps: int, checkpoint: int):
        pctx.load(E, B)
        n = x.shape[0]
        st = {k: v.detach().clone() for k, v in zip(_NAMES, (x, y, xp, yp, ux, uy, uz))}
        st["status"] = torch.zeros(n, dtype=torch.uint8, device=x.device)
        qmd = qm.detach() if qm is not None else None
        segs = []
        done = 0
        while done < n_steps:
            k = min(checkpoint, n_steps - done)
            segs.append(({kk: v.clone() for kk, v in st.items() if kk != "status"}, k))
            gcb.gcb_push(pctx.ctx, _parts(st, qmd), prm, k)
            done += k
        ctx.pctx, ctx.prm, ctx.segs, ctx.qm = pctx, prm, segs, qmd
        ctx.shape = tuple(E.shape)
        ctx.generation = pctx.generation
        ctx.save_for_backward(E.detach(), B.detach())
        return tuple(st[k] for k in _NAMES)

    @staticmethod
    def backward(ctx, *grads):
        pctx, prm = ctx.pctx, ctx.prm
        _reload_if_replaced(ctx, pctx)
        ref = ctx.segs[0][0]["x"] if ctx.segs else None
        dev = ref.device if ref is not None else torch.device("cuda")
        n = ref.shape[0] if ref is not None else 0
        lam = [g.contiguous() if g is not None else torch.zeros(n, dtype=torch.float64, device=dev)
               for g in grads]
        dE = torch.zeros(ctx.shape, dtype=torch.float32, device=dev)
        dB = torch.zeros(ctx.shape, dtype=torch.float32, device=dev)
        for start, k in reversed(ctx.segs):
            st = dict(start)
            st["status"] = torch.zeros(n, dtype=torch.uint8, device=dev)
            out = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(7)]
            gcb.gcb_push_backward(pctx.ctx, _parts(st, ctx.qm), prm, k, lam, out,
                                  [dE[0], dE[1], dE[2]], [dB[0], dB[1], dB[2]])
            lam = out
        return (dE.double(), dB.double(), *lam, None, None, None, None, None)


def push(E, B, x, y, xp, yp, ux, uy, uz, qm, pctx, prm, n_steps, checkpoint=32):
    """Differentiable push; returns the final (x, y, xp, yp, ux, uy, uz).

    The particles are cell-sorted every prm.sort_every steps (4 when it is 0)
    in place (keep_order), so the tiled kernel does the work and the outputs
    stay in input order; gcb_push_backward recomputes the same way."""
    prm = gcb.gcb_params.from_buffer_copy(prm)
    if prm.sort_every <= 0:
        prm.sort_every = 4
    prm.keep_order = 1
    return GcbPush.apply(E, B, x, y, xp, yp, ux, uy, uz, qm, pctx, prm, int(n_steps),
                         int(checkpoint))


_NAMES3 = ("x", "y", "z", "xp", "yp", "zp", "ux", "uy", "uz")


class PushContext3(PushContext):
    """A libgcb context with binary64 3D fields taken from device tensors, on
    a lattice of cell sizes d = (dx, dy, dz) and component offsets `stagger`."""

    def __init__(self, device: int = 0, d=(1.0, 1.0, 1.0), stagger=gcb.YEE3_STAGGER):
        super().__init__(device)
        self.d, self.stagger = tuple(d), stagger

    def load(self, E: torch.Tensor, B: torch.Tensor):
        nz, ny, nx = (int(v) for v in E.shape[1:])
        desc = gcb.grid3_desc(nx, ny, nz, *self.d, self.stagger, gcb.GCB_F64)
        Ec = [E[i].detach().contiguous() for i in range(3)]
        Bc = [B[i].detach().contiguous() for i in range(3)]
        gcb.gcb_load_fields_3d(self.ctx, desc, Ec, Bc, src=gcb.GCB_DEVICE)
        torch.cuda.current_stream().synchronize()
        self.shape = (nz, ny, nx)
        self.generation += 1


class GcbPush3(torch.autograd.Function):
    @staticmethod
    def forward(ctx, E, B, x, y, z, xp, yp, zp, ux, uy, uz, qm, pctx: PushContext3, prm,
                n_steps: int, checkpoint: int):
        pctx.load(E, B)
        n = x.shape[0]
        st = {k: v.detach().clone() for k, v in zip(_NAMES3, (x, y, z, xp, yp, zp, ux, uy, uz))}
        st["status"] = torch.zeros(n, dtype=torch.uint8, device=x.device)
        qmd = qm.detach() if qm is not None else None
        segs = []
        done = 0
        while done < n_steps:
            k = min(checkpoint, n_steps - done)
            segs.append(({kk: v.clone() for kk, v in st.items() if kk != "status"}, k))
            d = dict(st, qm=qmd, id=None)
            gcb.gcb_push_3d(pctx.ctx, gcb.particles3(d), prm, k)
            done += k
        ctx.pctx, ctx.prm, ctx.segs, ctx.qm = pctx, prm, segs, qmd
        ctx.shape = tuple(E.shape)
        ctx.generation = pctx.generation
        ctx.save_for_backward(E.detach(), B.detach())
        return tuple(st[k] for k in _NAMES3)

    @staticmethod
    def backward(ctx, *grads):
        pctx, prm = ctx.pctx, ctx.prm
        _reload_if_replaced(ctx, pctx)
        ref = ctx.segs[0][0]["x"] if ctx.segs else None
        dev = ref.device if ref is not None else torch.device("cuda")
        n = ref.shape[0] if ref is not None else 0
        lam = [g.contiguous() if g is not None else torch.zeros(n, dtype=torch.float64, device=dev)
               for g in grads]
        dE = torch.zeros(ctx.shape, dtype=torch.float32, device=dev)
        dB = torch.zeros(ctx.shape, dtype=torch.float32, device=dev)
        for start, k in reversed(ctx.segs):
            st = dict(start, qm=ctx.qm, id=None)
            st["status"] = torch.zeros(n, dtype=torch.uint8, device=dev)
            out = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(9)]
            gcb.gcb_push_backward_3d(pctx.ctx, gcb.particles3(st), prm, k, lam, out,
                                     [dE[0], dE[1], dE[2]], [dB[0], dB[1], dB[2]])
            lam = out
        return (dE.double(), dB.double(), *lam, None, None, None, None, None)


def push3(E, B, x, y, z, xp, yp, zp, ux, uy, uz, qm, pctx, prm, n_steps, checkpoint=32):
    """Differentiable 3D push; returns the final (x, y, z, xp, yp, zp, ux, uy, uz)
    in input order.

    As in 2D, the particles are cell-sorted in place (keep_order) every
    prm.sort_every steps (4 when it is 0), in cubic tiles of prm.tile cells (4
    when it is 0), so the tiled kernel does the work; gcb_push_backward_3d
    recomputes the same way."""
    prm = gcb.gcb_params.from_buffer_copy(prm)
    if prm.sort_every <= 0:
        prm.sort_every = 4
    if prm.tile <= 0:
        prm.tile = 4
    prm.keep_order = 1
    return GcbPush3.apply(E, B, x, y, z, xp, yp, zp, ux, uy, uz, qm, pctx, prm, int(n_steps),
                          int(checkpoint))


class KineticEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ux, uy, uz, pctx: PushContext, prm):
        n = ux.shape[0]
        st = {"x": ux, "y": ux, "xp": ux, "yp": ux, "ux": ux.detach(), "uy": uy.detach(),
              "uz": uz.detach(), "status": torch.zeros(n, dtype=torch.uint8, device=ux.device)}
        out = torch.zeros(1, dtype=torch.float64, device=ux.device)
        lam = [torch.empty_like(ux) for _ in range(3)]
        gcb.gcb_kinetic_energy(pctx.ctx, gcb.particles(st), prm, out, lam)
        ctx.save_for_backward(*lam)
        return out[0]

    @staticmethod
    def backward(ctx, g):
        lx, ly, lz = ctx.saved_tensors
        return g * lx, g * ly, g * lz, None, None


def kinetic_energy(ux, uy, uz, pctx, prm):
    return KineticEnergy.apply(ux, uy, uz, pctx, prm)
