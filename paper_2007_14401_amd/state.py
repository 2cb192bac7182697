"""Particle state as device tensors (structure of arrays) for libgcb."""
from __future__ import annotations

import numpy as np
import torch

from . import gcb

_KEYS = ("x", "y", "xp", "yp", "ux", "uy", "uz")
_KEYS3 = ("x", "y", "z", "xp", "yp", "zp", "ux", "uy", "uz")


def to_device(ens, device="cuda", form=gcb.GCB_FORM_F64, per_particle_qm=True,
              with_id=True) -> dict:
    """numpy ensemble (attributes x, y, xp, yp, ux, uy, uz, qm, id, and z, zp
    for a 3D ensemble) -> dict of tensors."""
    udt = torch.float64 if form == gcb.GCB_FORM_F64 else torch.float32
    t = {}
    for k in (_KEYS3 if hasattr(ens, "z") else _KEYS):
        dt = udt if k in ("ux", "uy", "uz") else torch.float64
        t[k] = torch.as_tensor(np.ascontiguousarray(getattr(ens, k)), dtype=dt).to(device)
    n = t["x"].shape[0]
    t["qm"] = (torch.as_tensor(np.ascontiguousarray(ens.qm), dtype=torch.float64).to(device)
               if per_particle_qm else None)
    t["id"] = (torch.arange(n, dtype=torch.int32, device=device) if with_id else None)
    t["status"] = torch.zeros(n, dtype=torch.uint8, device=device)
    return t


def to_host(t: dict) -> dict:
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in t.items()}


def unsort(t: dict) -> dict:
    """Host copy with every array put back in id order."""
    h = to_host(t)
    if h.get("id") is None:
        return h
    order = np.argsort(h["id"], kind="stable")
    return {k: (v[order] if v is not None else None) for k, v in h.items()}


def clone(t: dict) -> dict:
    return {k: (v.clone() if v is not None else None) for k, v in t.items()}
