"""The locality the maximum-edge parity test relies on, checked on the oracle alone: on
a grid made of a repeated 256 x 4 pattern between two x-walls, one step (magnetic
sweeps and three stages) equals, column by column, the step of the pattern with a
periodic x axis away from the walls, and the step of the pattern repeated four times
within 512 columns of each wall."""
import numpy as np

from oracle import oracle as orc
from paper_2511_10257_amd import workloads as wl

P, NY = 256, 4


def problem(nx, periodic=False):
    prob = wl.droplet_problem(nx, 2.0, ste=0.1, bo_m=1.0, angle_deg=90.0, precision="fp64", ny=NY)
    prob.update(init_max=0, periodic=[1 if periodic else 0, 0])
    return prob


def test_repeated_pattern_step_is_local():
    nx = 16 * P
    per = orc.Oracle(problem(P, periodic=True), init=False)
    st = wl.smooth_state(P, NY, 42, latent=per.params.latent, h0=per.params.h0, angle_deg=90.0)
    per.set_state(st)
    walls = orc.Oracle(problem(4 * P), init=False)
    walls.set_state({k: np.tile(v, (1, 4)) for k, v in st.items()})
    full = orc.Oracle(problem(nx), init=False)
    full.set_state({k: np.tile(v, (1, nx // P)) for k, v in st.items()})
    for o in (per, walls, full):
        o.step(1)
    # Equal up to rounding: cos(90 deg) leaves an x-component of the applied field of
    # 6e-17 H0, so the applied potential, which is subtracted from the stored one, depends
    # on the absolute column at that level.
    for name in ("He", "p", "Mx", "My", "C", "phi", "S"):
        a = full.get(name)
        w, q = walls.get(name), per.get(name)
        mid = np.tile(q, (1, (nx - 1024) // P))
        tol = 1e-12 * np.max(np.abs(a))
        assert np.max(np.abs(a[:, :512] - w[:, :512])) <= tol, name
        assert np.max(np.abs(a[:, nx - 512:] - w[:, 512:])) <= tol, name
        assert np.max(np.abs(a[:, 512:nx - 512] - mid)) <= tol, name
    # the wall regions really differ from the periodic pattern (the comparison is not vacuous)
    assert not np.allclose(full.get("He")[:, :8], per.get("He")[:, :8], rtol=0, atol=1e-9)
