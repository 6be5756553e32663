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


def _freeze_step(s, start, cap):
    """First step at which the liquid fraction is below 1e-3: the solver is stepped to
    `start` (below the freezing time), then one step at a time."""
    s.step(start)
    step = start
    fl = s.observe()["liquid_fraction"]
    while fl >= 1e-3 and step < cap:
        s.step(1)
        step += 1
        fl = s.observe()["liquid_fraction"]
    return step


def test_fp32_freezing_time_matches_fp64_on_the_256_droplet():
    """The benchmark's 256^2 droplet solved to freezing in FP32 (FP64 reductions) and in
    FP64 on the GPU (the FP64 path is held to the oracle at rounding level by the parity
    tests): the freezing steps agree within 0.5 %."""
    p32 = wl.droplet256()
    p64 = wl.with_changes(p32, precision="fp64", init_tol=1e-9)
    probe = lbfs.Solver(p64)
    # coarse search for the FP64 freezing step, then the exact one
    step = 0
    while probe.observe()["liquid_fraction"] >= 1e-3 and step < 400000:
        probe.step(2000)
        step += 2000
    n64 = _freeze_step(lbfs.Solver(p64), max(0, step - 2000), step + 1)
    n32 = _freeze_step(lbfs.Solver(p32), int(0.99 * n64), int(1.02 * n64))
    print(f"256^2 droplet: freezing step FP32 {n32}, FP64 {n64}")
    assert abs(n32 - n64) <= 0.005 * n64
