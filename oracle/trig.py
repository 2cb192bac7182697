"""sin and cos for the oracle (test infrastructure: only tests/, the smoke
check and bench.py's CPU baseline use oracle/).

Cody-Waite additive reduction by pi/2 with a two-part constant whose first
part has 33 significant bits (so k * PIO2_HI is exact for |k| < 2^20, i.e.
|x| below about 1.6e6) and Taylor polynomials of degree 19 (sin) and 20
(cos) on [-pi/4, pi/4] in Horner form.  The HIP path evaluates the same
operations, so both sides agree bit for bit; the pins check the result
against the platform's correctly rounded sin/cos.  Used by the curved-
spacetime metric (sin and cos of theta) and by the gyro-phase option of the
guiding-center step (the phase advance of a step).
"""
from __future__ import annotations

import math

import torch

PIO2_HI = 1.57079632673412561417e+00
PIO2_LO = 6.07710050650619224932e-11
TWO_OVER_PI = 2.0 / math.pi
SIN_C = [(-1.0) ** ((n - 1) // 2) / math.factorial(n) for n in range(3, 20, 2)]   # 1/3! .. 1/19!
COS_C = [(-1.0) ** (n // 2) / math.factorial(n) for n in range(2, 21, 2)]        # 1/2! .. 1/20!


def sincos(th: torch.Tensor):
    k = torch.floor(th * TWO_OVER_PI + 0.5)
    y = (th - k * PIO2_HI) - k * PIO2_LO
    z = y * y
    ps = torch.full_like(z, SIN_C[-1])
    for cf in reversed(SIN_C[:-1]):
        ps = ps * z + cf
    s = y + (y * z) * ps
    pc = torch.full_like(z, COS_C[-1])
    for cf in reversed(COS_C[:-1]):
        pc = pc * z + cf
    c = 1.0 + z * pc
    q = k.to(torch.int64) & 3
    sn = torch.where(q == 0, s, torch.where(q == 1, c, torch.where(q == 2, -s, -c)))
    cs = torch.where(q == 0, c, torch.where(q == 1, -s, torch.where(q == 2, -c, s)))
    return sn, cs
