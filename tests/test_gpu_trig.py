"""The library's own binary64 sin and cos (gcb_sincos: the curved-spacetime
metric's sin/cos of theta and the gyro-phase option's phase advance) against
the C library's sin and cos, independently of the oracle, which evaluates
the same published method and is pinned against the C library on its own
(tests/test_oracle_phase_pins.py).  Needs an MI355X.

Bar: within two units in the last place of numpy's (correctly rounded in
practice) sin/cos wherever |value| >= 1e-6, and within 2.3e-16 absolute
next to a zero (where the reduction's absolute error rules), over
|x| <= 1e5 plus multiples of pi/2; and equal bit for bit to the oracle's
evaluation (the parity tests of the curved-spacetime push rest on that)."""
import math

import numpy as np
import pytest
import torch

from gpu_util import log
from oracle.trig import sincos

pytestmark = pytest.mark.gpu


def test_library_sincos_against_libm():
    from paper_2007_14401_amd import gcb
    rng = np.random.default_rng(17)
    x = np.concatenate([rng.uniform(-1e5, 1e5, 400000), rng.uniform(-10.0, 10.0, 100000),
                        np.arange(-4000, 4001) * (math.pi / 2),
                        np.array([0.0, -0.0, 1e-300, -1e-300, 5e-324, 1e-8, math.pi / 4,
                                  3 * math.pi / 4, 1e5])])
    xt = torch.as_tensor(x, device="cuda:0")
    s = torch.empty_like(xt)
    c = torch.empty_like(xt)
    ctx = gcb.gcb_create(0)
    try:
        gcb.gcb_sincos(ctx, xt, s, c)
        torch.cuda.synchronize()
    finally:
        gcb.gcb_destroy(ctx)
    got_s, got_c = s.cpu().numpy(), c.cpu().numpy()
    for got, ref, name in ((got_s, np.sin(x), "sin"), (got_c, np.cos(x), "cos")):
        err = np.abs(got - ref)
        big = np.abs(ref) >= 1e-6
        ulps = err[big] / np.spacing(np.abs(ref[big]))
        log(f"{name}: max {ulps.max():.2f} ulp where |value| >= 1e-6, "
            f"{np.mean(err == 0):.4f} bit-identical to the C library; max abs err {err.max():.2e}")
        assert ulps.max() <= 2.0, name
        assert err.max() <= 2.3e-16, name
    os_, oc = sincos(torch.as_tensor(x))
    assert np.array_equal(got_s, os_.numpy()) and np.array_equal(got_c, oc.numpy())
