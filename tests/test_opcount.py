"""The operation-counting build of the oracle computes what the oracle computes (so its
count is the count of the same algorithm), and the count per cell is a property of the
method, not of the grid size."""
from __future__ import annotations

import numpy as np

from oracle import opcount, oracle as orc
from paper_2511_10257_amd import workloads as wl


def test_counting_build_reproduces_the_oracle():
    prob = wl.droplet_problem(24, 6.0, ste=0.1, bo_m=1.0, angle_deg=30.0, precision="fp64", ny=20)
    counted = orc.Oracle(prob, library=orc.load(opcount.build()))
    plain = orc.Oracle(prob)
    counted.step(3)
    plain.step(3)
    for name in ("He", "p", "Mx", "My", "C", "phi", "S"):
        a, b = counted.get(name), plain.get(name)
        assert np.allclose(a, b, rtol=1e-12, atol=1e-14 * max(1.0, float(np.max(np.abs(b))))), name


def test_count_per_cell_is_size_independent():
    per = []
    for n in (32, 64):
        prob = wl.droplet_problem(n, n / 4.0, ste=0.1, bo_m=0.5, angle_deg=90.0, precision="fp64")
        c = opcount.count(prob)["per_cell"]
        per.append(c)
        # one step is the magnetic phase plus three right-hand sides and their updates
        assert 3 * c["rhs"]["flops"] < c["step"]["flops"] < 3 * c["rhs"]["flops"] + c["mag"]["flops"] + 200
        assert c["rhs"]["div"] > 0 and c["mag"]["flops"] > 0
    assert abs(per[0]["stage"]["flops"] / per[1]["stage"]["flops"] - 1.0) < 0.02
