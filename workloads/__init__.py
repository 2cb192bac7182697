"""Seeded synthetic inputs for the coupled guiding-center/Boris pusher.

This package only *draws* inputs: field snapshots sampled from closed-form
Harris-sheet expressions and particle ensembles drawn from seeded numpy
generators.  It contains none of the pusher's arithmetic (no interpolation,
no switch, no Boris or guiding-center update), so both the CPU oracle and the
HIP path can consume the very same arrays.

The paper's own experiments use field snapshots of particle-in-cell runs
(Sec. 4.1 and 4.2), which are not available; the Harris-family fields here are
stand-ins with the same structure (current sheets, X-points, an inflow
electric field, regions where E exceeds B).
"""
from .harris import YEE_STAGGER, COLLOCATED, COMPONENTS, harris_fields
from .particles import (maxwell_juttner_u, power_law_gamma, isotropic_dirs,
                        initial_state, Ensemble)
from .configs import CONFIGS, make_config, Config
from .harris3d import YEE3_STAGGER, harris3d_fields
from .configs3d import CONFIGS3, Config3, Ensemble3, initial_state3, make_config3
from .gr import (GR_CONFIGS, GRConfig, GREnsemble, make_gr_config, magnetosphere_fields,
                 magnetosphere_particles)

__all__ = [
    "YEE_STAGGER", "COLLOCATED", "COMPONENTS", "harris_fields",
    "maxwell_juttner_u", "power_law_gamma", "isotropic_dirs", "initial_state",
    "Ensemble", "CONFIGS", "make_config", "Config", "GR_CONFIGS", "GRConfig",
    "GREnsemble", "make_gr_config", "magnetosphere_fields", "magnetosphere_particles",
    "YEE3_STAGGER", "harris3d_fields", "CONFIGS3", "Config3", "Ensemble3",
    "initial_state3", "make_config3",
]
