"""Per-step FP32 parity at evolved states (mushy and solid branches active) and on the
1024 x 1024 droplet, through the C ABI.

Both sides take one step from the same state: the FP64 oracle from the state, the FP32
path from the state rounded to its storage (He, p, momentum, potential and S in FP32,
the order parameter in FP64). The bar is the relative L2 norm of the error of each
field against that field's own norm, with no floor; the form floored by the state's
scales is printed beside it. FP64 runs the same steps to rounding.

The 64 x 64 states are those of the oracle's trajectory at a quarter, half and three
quarters of its freezing time (tests/golden/freeze_time.json, written by the oracle):
the FP64 GPU path reaches them and is tied to that trajectory by the liquid fraction
the oracle recorded there (1e-9), before the one-step comparison.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2511_10257_amd import lbfs, workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "freeze_time.json")))
STATE = ("He", "p", "Mx", "My", "C", "phi", "S")
CHECKED = ("He", "p", "Mx", "My", "C", "phi")


def phi0(prob, nx, ny):
    p = orc.make_params(prob)
    th = np.deg2rad(p.angle_deg)
    y, x = np.mgrid[0:ny, 0:nx] + 0.5
    return -p.h0 * (x * np.cos(th) + y * np.sin(th))


def scale_floor(prob):
    p = orc.make_params(prob)
    R = prob["drop"][2]
    m = p.rho[1] / 3.0 * p.sigma / p.mu[1]
    return dict(He=p.latent, p=p.sigma / R, Mx=m, My=m, C=1.0, phi=max(p.h0 * R, 1e-30))


def one_step_errors(prob64, state):
    """Relative L2 errors (unfloored, and floored by the state's scales) of one FP32 and one FP64 GPU
    step against one oracle step, all from `state`."""
    nx, ny = prob64["nx"], prob64["ny"]
    clock = state.get("_clock")
    fields = {k: v for k, v in state.items() if k != "_clock"}
    o = orc.Oracle(dict(prob64, init_max=0), init=False)
    o.set_state(fields)
    if clock:
        o.set_time(*clock)
    o.step(1)
    ref = {k: o.get(k) for k in STATE}
    p0 = phi0(prob64, nx, ny)
    ref["phi"] = ref["phi"] - p0
    out = {}
    for prec in ("fp32", "fp64"):
        g = lbfs.Solver(wl.with_changes(prob64, precision=prec, init_max=0))
        g.set_state(fields)
        if clock:
            g.set_time(*clock)
        g.step(1)
        fl = scale_floor(prob64)
        errs = {}
        for k in STATE:
            a = g.get(k) - (p0 if k == "phi" else 0.0)
            b = ref[k]
            d = np.linalg.norm(a - b)
            nb = np.linalg.norm(b)
            errs[k] = dict(rel=d / nb if nb > 0 else d,
                           floored=d / max(nb, fl[k] * np.sqrt(b.size)) if k in fl else None)
        out[prec] = errs
        g.close()
    return out


def report(tag, errs):
    for prec, e in errs.items():
        print(f"{tag} {prec}: " + "  ".join(
            f"{k} {v['rel']:.2e}" + (f" ({v['floored']:.1e} floored)" if v["floored"] is not None else "")
            for k, v in e.items()), flush=True)


def check(errs):
    for k in CHECKED:
        assert errs["fp32"][k]["rel"] <= 1e-5, ("fp32", k, errs["fp32"][k])
        assert errs["fp64"][k]["rel"] <= 1e-10, ("fp64", k, errs["fp64"][k])


@pytest.fixture(scope="module")
def states64():
    """The 64^2 droplet (Ste 0.1, vertical field, Bo_m 0.5) at 1/4, 1/2 and 3/4 of the
    oracle's freezing time, reached by the FP64 GPU path."""
    g = GOLDEN["droplet64"]
    case = g["case"]
    prob = wl.droplet_problem(case["n"], case["radius"], ste=case["ste"], bo_m=case["bo_m"],
                              angle_deg=case["angle_deg"], precision="fp64")
    s = lbfs.Solver(prob)
    out, step = {}, 0
    for q in (1, 2, 3):
        m = round(q * g["freeze_step"] / 4)
        s.step(m - step)
        step = m
        obs = s.observe()
        assert abs(obs["liquid_fraction"] - g["fl_at"][str(q)]) <= 1e-9, (q, obs["liquid_fraction"])
        st = {k: s.get(k) for k in STATE}
        st["_clock"] = (obs["t"], int(obs["step"]))
        out[q] = (obs["liquid_fraction"], st)
    s.close()
    return prob, out


@pytest.mark.parametrize("quarter", [1, 2, 3])
def test_fp32_step_at_a_fraction_of_the_freezing_time(states64, quarter):
    prob, states = states64
    fl, st = states[quarter]
    # the freezing front is active: part of the droplet frozen, part still liquid
    assert 0.05 < fl < 0.95
    errs = one_step_errors(prob, st)
    report(f"64^2 at {quarter}/4 of the freezing time (liquid fraction {fl:.3f})", errs)
    check(errs)


def test_fp32_step_on_the_1024_droplet():
    """The 1024^2 droplet (R 256, horizontal field, Bo_m 1.5, density ratio 100) after
    2000 FP64 GPU steps; one step of each path from that state."""
    prob = wl.droplet1024("fp64")
    s = lbfs.Solver(prob)
    s.step(2000)
    obs = s.observe()
    st = {k: s.get(k) for k in STATE}
    st["_clock"] = (obs["t"], int(obs["step"]))
    s.close()
    errs = one_step_errors(prob, st)
    report(f"1024^2 after 2000 steps (liquid fraction {obs['liquid_fraction']:.4f})", errs)
    check(errs)
