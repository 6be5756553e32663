"""The oracle's freezing-time goldens: reproducible, and consistent with the quasi-
steady Stefan estimate t ~ R^2 / (2 Ste alpha_s) of a solid front growing from a cold
wall (the conductive limit of the Neumann solution, Sec. 4.1, for small Ste)."""
from __future__ import annotations

import importlib.util
import json
import os

import pytest

HERE = os.path.dirname(__file__)
GOLDEN = json.load(open(os.path.join(HERE, "golden", "freeze_time.json")))


def _maker():
    spec = importlib.util.spec_from_file_location("make_freeze_golden",
                                                  os.path.join(HERE, "golden", "make_freeze_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_golden_reproduces():
    mk = _maker()
    got = mk.freeze(mk.CASES["droplet32"])
    assert got["freeze_step"] == GOLDEN["droplet32"]["freeze_step"]
    for q, v in GOLDEN["droplet32"]["fl_at"].items():
        assert got["fl_at"][q] == pytest.approx(v, rel=1e-12)


def test_freezing_time_follows_the_stefan_estimate():
    from paper_2511_10257_amd import workloads as wl
    for name, g in GOLDEN.items():
        c = g["case"]
        prob = wl.droplet_problem(c["n"], c["radius"], ste=c["ste"], bo_m=c["bo_m"], angle_deg=c["angle_deg"])
        alpha_s = prob["lam"][0] / (prob["rho"][0] * prob["cp"][0])
        est = c["radius"] ** 2 / (2.0 * c["ste"] * alpha_s * prob["dt"])
        assert 0.9 < g["freeze_step"] / est < 1.3, (name, g["freeze_step"], est)
    # doubling the radius at the same Stefan number: about four times longer
    r = GOLDEN["droplet64"]["freeze_step"] / GOLDEN["droplet32"]["freeze_step"]
    assert 3.0 < r < 4.5
