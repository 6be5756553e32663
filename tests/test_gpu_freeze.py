"""Freezing time of the GPU path against the oracle's (tests/golden/freeze_time.json):
the first step at which the droplet's liquid fraction is below 1e-3, in FP64 and in
FP32 (FP32 fields, FP64 reductions), within 0.5 %."""
from __future__ import annotations

import json
import os

import pytest

from paper_2511_10257_amd import lbfs, workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "freeze_time.json")))


def _problem(case: dict, precision: str) -> dict:
    return wl.droplet_problem(case["n"], case["radius"], ste=case["ste"], bo_m=case["bo_m"],
                              angle_deg=case["angle_deg"], precision=precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", sorted(GOLDEN))
def test_freezing_time_matches_oracle(name, precision):
    g = GOLDEN[name]
    n_ref = g["freeze_step"]
    s = lbfs.Solver(_problem(g["case"], precision))
    fl_at = {}
    marks = {round(q * n_ref / 4): str(q) for q in (1, 2, 3)}
    step = 0
    start = int(0.97 * n_ref)
    for m in sorted(marks):
        s.step(m - step)
        step = m
        fl_at[marks[m]] = s.observe()["liquid_fraction"]
    s.step(start - step)
    step = start
    fl = s.observe()["liquid_fraction"]
    while fl >= g["threshold"] and step < 2 * n_ref:
        s.step(1)
        step += 1
        fl = s.observe()["liquid_fraction"]
    print(f"{name} {precision}: freeze step {step} (oracle {n_ref}); FL {fl_at} vs {g['fl_at']}")
    assert abs(step - n_ref) <= 0.005 * n_ref
    tol = 1e-9 if precision == "fp64" else 2e-3
    for q, v in g["fl_at"].items():
        assert abs(fl_at[q] - v) <= tol, (q, fl_at[q], v)
    s.close()
