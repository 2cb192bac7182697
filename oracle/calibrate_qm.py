"""Report the initial guiding-center fraction of the mixed electron ensemble
for a given scalar q/m, and find the q/m giving a target fraction by bisection.

TEST INFRASTRUCTURE (a script that calls only the oracle and the input
generators).  Usage:
    python -m oracle.calibrate_qm [--config harris4096] [--n 200000] [--target 0.7]
"""
from __future__ import annotations

import argparse

import torch

from workloads import make_config

from .fields import GridFields
from .pusher import Params, switch_gca


def gca_fraction(cfg, qm: float, n: int) -> float:
    ens = cfg.with_(qm=qm).particles(n=n)
    F = cfg.fields()
    prov = GridFields(F, cfg.dx, cfg.dy, cfg.stagger)
    p = Params(dt=cfg.dt, c=cfg.c, f_rho=cfg.f_rho, f_E=cfg.f_E,
               Lx=cfg.Lx, Ly=cfg.Ly, dl=(cfg.dx * cfg.dy) ** 0.5)
    t = lambda a: torch.as_tensor(a, dtype=torch.float64)
    s = prov(t(ens.x), t(ens.y))
    g = switch_gca(s, t(ens.ux), t(ens.uy), t(ens.uz), t(ens.qm), p)
    return float(g.double().mean())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="harris4096")
    ap.add_argument("--n", type=int, default=200_000)
    ap.add_argument("--target", type=float, default=0.7)
    ap.add_argument("--qm", type=float, default=None)
    a = ap.parse_args()
    cfg = make_config(a.config)
    if a.qm is not None:
        print(f"qm={a.qm}: GCA fraction {gca_fraction(cfg, a.qm, a.n):.4f}")
        return
    lo, hi = 0.1, 100.0      # |q/m| bracket; the fraction grows with |q/m|
    for _ in range(30):
        mid = (lo * hi) ** 0.5
        f = gca_fraction(cfg, -mid, a.n)
        if f < a.target:
            lo = mid
        else:
            hi = mid
    q = -round((lo * hi) ** 0.5, 3)
    print(f"qm={q}: GCA fraction {gca_fraction(cfg, q, a.n):.4f}")


if __name__ == "__main__":
    main()
