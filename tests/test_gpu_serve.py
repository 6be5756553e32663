"""Continuous batching (serve.Server) against solves run alone.

Requests arrive while others are on the GPU, wait for memory, are admitted into the
running batch, and retire when frozen (liquid fraction < 1e-3). Each served result -
the fields at retirement, the step count and the observables - must equal the same
problem stepped alone for the same number of steps, bit for bit."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2511_10257_amd import lbfs, serve, workloads as wl

pytestmark = pytest.mark.gpu

FIELDS = ("He", "p", "Mx", "My", "C", "phi", "S")


def _stream():
    # (arrival in batch steps, problem): uneven sizes, angles, Bond and Stefan numbers
    spec = [(0, 16, 4.0, 0.5, 1.5, 90.0), (0, 24, 6.0, 0.3, 0.4, 0.0), (100, 32, 8.0, 0.2, 1.0, 45.0),
            (150, 20, 5.0, 0.4, 0.0, 30.0), (150, 28, 7.0, 0.35, 1.9, 75.0), (600, 16, 4.0, 0.25, 0.8, 10.0)]
    return [(t, wl.droplet_problem(n, r, ste=ste, bo_m=bo, angle_deg=ang, precision="fp32"))
            for t, n, r, ste, bo, ang in spec]


def test_served_results_equal_alone():
    arrivals = _stream()
    biggest = max(lbfs.Batch.instance_bytes(p) for _, p in arrivals)
    captured = {}

    def on_finish(req, view):
        captured[req.rid] = ({f: view.get(f) for f in FIELDS}, req.steps, dict(req.obs))

    srv = serve.Server(hbm_budget=int(2.2 * biggest) + (1 << 16), max_slots=8, chunk=50,
                       max_steps=20000, on_finish=on_finish)
    rep = srv.run(arrivals, clock="steps")
    srv.close()
    print(rep)
    assert rep["completed"] == len(arrivals) and rep["rejected"] == 0 and rep["nonfinite"] == 0
    waited = 0
    for rid, (t, prob) in enumerate(arrivals):
        fields, steps, obs = captured[rid]
        assert obs["liquid_fraction"] < 1e-3
        alone = lbfs.Solver(prob)
        alone.step(steps)
        ref = alone.observe()
        for f in FIELDS:
            assert np.array_equal(fields[f], alone.get(f)), (rid, f)
        for k in ("liquid_fraction", "solid_ratio", "volume", "mag_residual", "umax", "step"):
            assert obs[k] == ref[k], (rid, k)
        alone.close()
    assert rep["p50"] is not None and rep["p99"] >= rep["p50"]


def test_budget_forces_queueing_and_backfill():
    big = wl.droplet_problem(48, 12.0, ste=0.3, bo_m=1.0, angle_deg=0.0)
    small = wl.droplet_problem(16, 4.0, ste=0.5, bo_m=1.0, angle_deg=0.0)
    nb_big, nb_small = lbfs.Batch.instance_bytes(big), lbfs.Batch.instance_bytes(small)
    order = []

    def on_finish(req, view):
        order.append(req.rid)

    # room for one big instance plus one small one
    srv = serve.Server(hbm_budget=nb_big + nb_small + (1 << 16), max_slots=4, chunk=50, max_steps=20000,
                       on_finish=on_finish)
    rep = srv.run([(0, big), (0, big), (0, small)], clock="steps")
    srv.close()
    assert rep["completed"] == 3
    # the small request passes the second big one, which waits for the first to retire
    assert order.index(2) < order.index(1)


def test_request_larger_than_budget_is_rejected():
    prob = wl.droplet_problem(64, 16.0, ste=0.2, bo_m=1.0, angle_deg=0.0)
    small = wl.droplet_problem(16, 4.0, ste=0.5, bo_m=1.0, angle_deg=0.0)
    srv = serve.Server(hbm_budget=lbfs.Batch.instance_bytes(small) + (1 << 16), max_slots=2, chunk=50,
                       max_steps=5000)
    rep = srv.run([(0, prob), (10, small)], clock="steps")
    srv.close()
    assert rep["rejected"] == 1 and rep["completed"] == 1


def test_a_non_finite_solve_is_retired_and_the_others_finish():
    """Failure handling, forced from the host: right after admission one request's state
    gets a non-finite enthalpy in one cell (through its slot handle); the server retires
    it with the non-finite flag at the next observation, and the requests sharing its
    launches still finish with the fields they have alone."""
    arrivals = [(0, wl.droplet_problem(16, 4.0, ste=0.5, bo_m=0.5, angle_deg=90.0, precision="fp32")),
                (0, wl.droplet_problem(20, 5.0, ste=0.3, bo_m=1.0, angle_deg=45.0, precision="fp32")),
                (20, wl.droplet_problem(24, 6.0, ste=0.4, bo_m=1.0, angle_deg=0.0, precision="fp32"))]
    captured = {}

    def on_admit(req, view):
        if req.rid == 1:
            he = view.get("He")
            he[3, 7] = np.inf
            view.set("He", he)

    def on_finish(req, view):
        captured[req.rid] = ({f: view.get(f) for f in FIELDS}, req.steps, dict(req.obs), req.nonfinite)

    budget = sum(lbfs.Batch.instance_bytes(p) for _, p in arrivals) + (1 << 16)
    srv = serve.Server(hbm_budget=budget, max_slots=4, chunk=50, max_steps=20000, on_finish=on_finish,
                       on_admit=on_admit)
    rep = srv.run(arrivals, clock="steps")
    srv.close()
    assert rep["nonfinite"] == 1 and rep["completed"] == 2 and rep["unfinished_live"] == 0, rep
    _, steps_bad, obs_bad, nonfinite = captured[1]
    assert nonfinite and obs_bad["nonfinite"] == 1 and steps_bad == 50
    for rid in (0, 2):
        fields, steps, obs, nonfinite = captured[rid]
        assert not nonfinite and obs["liquid_fraction"] < 1e-3
        alone = lbfs.Solver(arrivals[rid][1])
        alone.step(steps)
        for f in FIELDS:
            assert np.array_equal(fields[f], alone.get(f)), (rid, f)
        alone.close()
