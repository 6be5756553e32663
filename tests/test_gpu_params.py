"""Problem parameters beyond the droplet workloads on the GPU: a melting range
(Ts < Tl, Eq. 8) and the automatic time step, against the oracle."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2511_10257_amd import lbfs, workloads as wl

pytestmark = pytest.mark.gpu


def test_melting_range_matches_oracle():
    prob = wl.droplet_problem(45, 9.0, ste=0.15, bo_m=1.0, angle_deg=60.0, precision="fp64", ny=33)
    prob.update(t_melt=-0.3, t_liquidus=0.2, t_init=0.05)   # the droplet starts mushy
    o = orc.Oracle(prob)
    g = lbfs.Solver(prob)
    for name in ("He", "T", "Fl"):
        assert np.max(np.abs(g.get(name) - o.get(name))) <= 1e-12 * max(1.0, np.max(np.abs(o.get(name)))), name
    st = {k: o.get(k) for k in ("He", "p", "Mx", "My", "C", "phi", "S")}
    g.set_state(st)
    o.step(4)
    g.step(4)
    for name in ("He", "C", "Mx", "T", "Fl"):
        x, y = g.get(name), o.get(name)
        assert np.max(np.abs(x - y)) <= 1e-10 * max(1.0, np.max(np.abs(y))), name


def test_automatic_time_step_matches_oracle():
    prob = wl.droplet_problem(40, 10.0, ste=0.1, bo_m=0.5, angle_deg=90.0, precision="fp64")
    prob = wl.with_changes(prob, dt=0.0, lam=[prob["lam"][0], prob["lam"][1], 0.1])   # gas diffusivity 1
    g = lbfs.Solver(prob)
    g.step(3)
    assert abs(g.observe()["t"] - 3 * 0.4) < 1e-14
    o = orc.Oracle(prob)
    o.step(3)
    assert np.max(np.abs(g.get("He") - o.get("He"))) <= 1e-10 * np.max(np.abs(o.get("He")))
