"""Steps after the state is written from outside a step.

Stage 3 leaves the permeability of the state it writes for the next step's magnetic
sweeps. A checkpoint load or a field write replaces the state, so the next step must
compute the permeability from the new state instead: a solver written mid-run has to
give, bit for bit, the fields of a fresh solver given the same state.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2511_10257_amd import lbfs, workloads as wl

pytestmark = pytest.mark.gpu

STATE = ("He", "p", "Mx", "My", "C", "phi", "S", "T", "Fl")


def _same(a, b, what):
    for name in STATE:
        x, y = a.get(name), b.get(name)
        assert np.all(np.isfinite(x)), f"{what}: field {name} is not finite"
        assert np.array_equal(x, y), f"{what}: field {name} differs (max {np.max(np.abs(x - y))})"


def _dip(C, cx, cy, depth=0.05, width=6.0):
    """C lowered by a smooth Gaussian dip of relative depth `depth` around (cx, cy): a
    write that changes the permeability there and keeps the state smooth."""
    ny, nx = C.shape
    y, x = np.mgrid[0:ny, 0:nx]
    return C * (1.0 - depth * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / width ** 2))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_field_write_between_steps_equals_a_fresh_start(precision):
    prob = wl.droplet_problem(96, 24.0, ste=0.1, bo_m=1.5, angle_deg=30.0, precision=precision, ny=72)
    a = lbfs.Solver(prob)
    a.step(20)
    blob = a.save()
    # a smooth dip of the order parameter at the drop's edge: the permeability changes there
    C = _dip(a.get("C"), cx=48 + 24, cy=4)
    a.set("C", C)
    a.step(12)
    b = lbfs.Solver(prob)
    b.load(blob)
    b.set("C", C)
    b.step(12)
    _same(a, b, "written mid-run against loaded and written")
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_checkpoint_load_between_steps_equals_an_uninterrupted_run(precision):
    prob = wl.droplet_problem(80, 20.0, ste=0.1, bo_m=1.0, angle_deg=90.0, precision=precision, ny=64)
    a = lbfs.Solver(prob)
    a.step(15)
    blob = a.save()
    a.step(40)          # the permeability of step 55 is left behind in the solver
    a.load(blob)        # back to step 15
    a.step(25)
    b = lbfs.Solver(prob)
    b.step(40)
    _same(a, b, "loaded back and stepped against uninterrupted")
    a.close()
    b.close()
