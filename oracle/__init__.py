"""CPU oracle for the coupled guiding-center / Boris pusher (TEST INFRASTRUCTURE).

This package is the plain, slow, float64 definition against which the HIP
path is checked.  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product path never does.

It shares no code with the HIP path.  Inputs (fields, particles) come from the
separate ``workloads`` package, which holds no arithmetic of the method.

Layout of the oracle:
  fields.py   field providers: bilinear interpolation with a linear shape
              function and its gradient on a staggered periodic grid (Sec. 4,
              opening paragraph), plus closed-form providers used by the pins.
  pusher.py   the local quantities (b, v_E, kappa, E_par, curvature terms),
              the switch S (Sec. 4.1), the relativistic Boris push (Sec. 2.1),
              the guiding-center leapfrog with and without curvature
              (Sec. 2.2.1, 2.2.2), the variable conversions of the coupled
              scheme (Sec. 3.1) and the multi-step driver.
  loss.py     mean kinetic energy and its gradient by reverse-mode autograd of
              the oracle itself (the oracle gradient of the adjoint checks).
  frame.py    the exact guiding-center frame of Sec. 2.2 (exact v_E, kappa,
              B', E', Psi, eta, xi, b*), used by the zero-curvature scheme
              when Params.exact_frame is set.
  fields3d.py the 3D gather: trilinear interpolation with a linear shape
              function and its gradient on a staggered periodic 3D grid, plus
              closed-form 3D providers used by the pins.
  pusher3d.py the coupled step in three dimensions (trilinear gather,
              gradients along z, three-component guiding-center position);
              reuses the dimension-free functions of pusher.py.
  trig.py     sin and cos by a fixed reduction and polynomial (the curved-
              spacetime metric and the gyro-phase option).
  gr.py       the general-relativistic coupled scheme (Sec. 2.3, 2.4, 3.2) in
              Kerr-Schild coordinates: metric functions and derivatives, the
              (r, theta) grid gather, the local-frame half pushes, the
              implicit-midpoint geodesic iterations, the guiding-center step,
              the switch with the proper cell length, and the driver.

All arithmetic is IEEE binary64 with correctly rounded +, -, *, /, sqrt and
no fused multiply-add: every product and sum is a separate torch operation.
"""
from .fields import (GridFields, UniformFields, LinearFields, CircularFields,
                     FieldSample, YEE, COLLOCATED)
from .pusher import (Params, State, ST_NONFINITE, ST_KAPPA, ST_QUAD, ST_BZERO,
                     ST_FPRES, local, gamma_gca, v_curv, switch_gca, boris,
                     gca_step, step, push, wrap, min_image, parallel_update,
                     GYR_MU, GYR_UPERP, GYR_ZERO, GYR_PHASE, gyration, conserved_mu, uperp_sq,
                     rotate_about, phase_advance,
                     mirror_parallel, mirror_check, ST_MIRROR)
from .loss import kinetic_energy, push_gradients, push_gradients3
from .fields3d import (GridFields3, UniformFields3, LinearFields3, CircularFieldsXZ,
                       FieldSample3, YEE3, COLLOCATED3)
from .frame import exact_frame, local_exact
from .pusher3d import Params3, State3, local3, boris_step3, gca_step3, step3, push3

__all__ = [
    "GridFields", "UniformFields", "LinearFields", "CircularFields",
    "FieldSample", "YEE", "COLLOCATED", "Params", "State", "ST_NONFINITE",
    "ST_KAPPA", "ST_QUAD", "ST_BZERO", "ST_FPRES", "local", "gamma_gca",
    "v_curv", "switch_gca", "boris", "gca_step", "step", "push", "wrap",
    "min_image", "parallel_update", "kinetic_energy", "push_gradients", "push_gradients3",
    "GridFields3", "UniformFields3", "LinearFields3", "CircularFieldsXZ", "FieldSample3",
    "YEE3", "COLLOCATED3", "Params3", "State3", "local3", "boris_step3", "gca_step3",
    "step3", "push3", "exact_frame", "local_exact",
    "GYR_MU", "GYR_UPERP", "GYR_ZERO", "GYR_PHASE", "gyration", "conserved_mu", "uperp_sq",
    "rotate_about", "phase_advance",
    "mirror_parallel", "mirror_check", "ST_MIRROR",
]
