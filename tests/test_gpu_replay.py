"""Synthetic replay of the flat-space accuracy experiment of Sec. 4.1 on the
GPU path (paper_2007_14401_amd/replay.py): 5 positrons started at v = v_E
upstream of a reconnecting Harris sheet, pushed for 100 plasma periods with a
gyro-resolving reference Boris push, the Boris push with the PiC-like step,
and the coupled push with the same step.

The claims checked are the paper's qualitative ones (Sec. 4.1): at small
gyro-radii the coupled push follows the gyro-resolved reference while the
Boris push with the large step does not, and the coupled push switches to
the guiding-center equations for most of the run.  The paper's figures are
not in its text, so the thresholds are this workload's, not the paper's
numbers; the full report is written to gpurun_out/replay_report.json.
"""
import json
import os

import pytest

from gpu_util import log

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_replay_coupled_tracks_reference():
    from paper_2007_14401_amd import replay
    reps = [replay.run(r, 1111, log=log) for r in (1e-2, 1e-3)]
    os.makedirs(os.path.join(ROOT, "gpurun_out"), exist_ok=True)
    with open(os.path.join(ROOT, "gpurun_out", "replay_report.json"), "w") as f:
        json.dump(reps, f, indent=1)
    for rep in reps:
        c, b = rep["coupled_curvature"], rep["boris"]
        log(f"rho/d_e={rep['rho_over_de']:g}: coupled max dev {c['max_deviation_de']:.3e} "
            f"d_e, Boris {b['max_deviation_de']:.3e} d_e, GCA fraction {c['gca_fraction']:.2f}")
        assert c["gca_fraction"] > 0.5
    fine = reps[1]
    assert fine["coupled_curvature"]["max_deviation_de"] < fine["boris"]["max_deviation_de"]
