"""Parity at the largest grid edge the library accepts (2^20 cells) on a grid of the
smallest height (4 cells), against the FP64 oracle.

The state repeats a seeded 256 x 4 pattern along x (the pattern's modes are periodic
in x with period 256 and the field is vertical, so the potential's applied part does
not depend on x either). A cell's right-hand side depends on the cells within 3 of it,
and one step on those within about 20 (three stages and four red-black sweeps), so:

- columns at least 512 from both x-walls must equal the oracle on the 256 x 4 pattern
  with a periodic x axis, at the same column modulo 256;
- the 512 columns next to each x-wall must equal the oracle on the pattern repeated
  four times (1024 x 4, the same walls), at the same distance from that wall.

This covers every one of the 1,048,576 columns (some 100 thousand stage tiles, rows of
2^20 cells) with oracle runs that take well under a second.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2511_10257_amd import lbfs, workloads as wl

pytestmark = pytest.mark.gpu

NX, NY, P = 1 << 20, 4, 256
FIELDS = ("He", "p", "Mx", "My", "C", "phi", "S")


def problem(nx, precision, periodic=False):
    prob = wl.droplet_problem(nx, 2.0, ste=0.1, bo_m=1.0, angle_deg=90.0, precision=precision, ny=NY)
    prob.update(init_max=0, periodic=[1 if periodic else 0, 0])
    return prob


def pattern_state(seed):
    o = orc.Oracle(problem(P, "fp64", periodic=True), init=False)
    return wl.smooth_state(P, NY, seed, latent=o.params.latent, h0=o.params.h0, angle_deg=90.0)


def tiled(state, reps):
    return {k: np.tile(v, (1, reps)) for k, v in state.items()}


def expected(arrays_per, arrays_walls, name_or_index):
    """The GPU-grid array assembled from the two oracle results."""
    per, walls = arrays_per[name_or_index], arrays_walls[name_or_index]
    mid = np.tile(per, (1, (NX - 2 * 512) // P))
    return np.concatenate([walls[:, :512], mid, walls[:, 512:]], axis=1)


def oracles(st):
    per = orc.Oracle(problem(P, "fp64", periodic=True), init=False)
    per.set_state(st)
    walls = orc.Oracle(problem(4 * P, "fp64"), init=False)
    walls.set_state(tiled(st, 4))
    return per, walls


def test_max_edge_rhs_fp64():
    st = pattern_state(seed=41)
    per, walls = oracles(st)
    g = lbfs.Solver(problem(NX, "fp64"))
    g.set_state(tiled(st, NX // P))
    Rg = g.rhs()
    Rp, Rw = per.rhs(), walls.rhs()
    for k, name in enumerate(("He", "p", "Mx", "My", "C")):
        ref = expected(Rp, Rw, k)
        scale = np.max(np.abs(ref)) + 1e-300
        err = np.max(np.abs(Rg[k] - ref))
        assert err <= 1e-10 * scale, (name, err, scale)


def test_max_edge_step_fp32():
    """One FP32 step (magnetic sweeps and three stages) against one FP64 oracle step:
    relative L2 per field at most 1e-5, and at most 1e-5 on each part of the grid
    (both wall regions and the interior)."""
    st = pattern_state(seed=42)
    per, walls = oracles(st)
    prob = problem(NX, "fp32")
    g = lbfs.Solver(prob)
    g.set_state(tiled(st, NX // P))
    per.step(1)
    walls.step(1)
    g.step(1)
    p = per.params
    fl = dict(He=p.latent, p=p.sigma / 2.0, Mx=p.rho[1] / 3.0 * p.sigma / p.mu[1],
              My=p.rho[1] / 3.0 * p.sigma / p.mu[1], C=1.0, phi=p.h0 * 2.0)
    res_p = {k: per.get(k) for k in fl}
    res_w = {k: walls.get(k) for k in fl}
    parts = dict(west=slice(0, 512), interior=slice(512, NX - 512), east=slice(NX - 512, NX))
    for name, floor in fl.items():
        a = g.get(name)
        b = expected(res_p, res_w, name)
        for part, sl in parts.items():
            d = np.linalg.norm(a[:, sl] - b[:, sl]) / max(np.linalg.norm(b[:, sl]), floor * np.sqrt(b[:, sl].size))
            assert d <= 1e-5, (name, part, d)
    obs = g.observe()
    assert obs["nonfinite"] == 0 and obs["step"] == 1
