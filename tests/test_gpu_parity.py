"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Both sides start from the same seeded state; FP64 must agree to rounding, FP32 within
the per-step relative L2 bound 1e-5 against each field's own norm (the helper's floors
only serve FP64 comparisons of fields that can vanish).
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2511_10257_amd import lbfs, workloads as wl

pytestmark = pytest.mark.gpu

NAMES = ("He", "p", "Mx", "My", "C")


def floors(prob):
    """Per-field L2 floors (per cell) for the relative error of near-zero fields."""
    p = orc.make_params(prob)
    R = prob["drop"][2]
    return dict(He=p.latent, p=p.sigma / R, Mx=p.rho[1] / 3.0 * p.sigma / p.mu[1],
                My=p.rho[1] / 3.0 * p.sigma / p.mu[1], C=1.0, phi=max(p.h0 * R, 1e-30), S=1e-6)


def rel_l2(a, b, floor):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), floor * np.sqrt(b.size))


def pair(prob, state=None):
    o = orc.Oracle(prob)
    g = lbfs.Solver(prob)
    if state is None:
        state = {k: o.get(k) for k in ("He", "p", "Mx", "My", "C", "phi", "S")}
    o.set_state(state)
    g.set_state(state)
    return o, g


def smooth_case(nx, ny, seed, precision="fp64", **kw):
    prob = wl.droplet_problem(nx, ny / 4.0, ste=0.1, bo_m=1.0, angle_deg=kw.pop("angle", 60.0),
                              precision=precision, ny=ny)
    prob.update(init_max=0, **kw)
    o = orc.Oracle(prob, init=False)
    st = wl.smooth_state(nx, ny, seed, latent=o.params.latent, h0=o.params.h0,
                         angle_deg=prob["angle_deg"])
    return prob, st


@pytest.mark.parametrize("shape", [(37, 29), (16, 8), (4, 4), (5, 23), (64, 64)])
def test_rhs_fp64_matches_oracle(shape):
    nx, ny = shape
    prob, st = smooth_case(nx, ny, seed=nx * 131 + ny)
    o, g = pair(prob, st)
    Ro, Rg = o.rhs(), g.rhs()
    for k, name in enumerate(NAMES):
        scale = np.max(np.abs(Ro[k])) + 1e-300
        assert np.max(np.abs(Rg[k] - Ro[k])) <= 1e-10 * scale, (name, np.max(np.abs(Rg[k] - Ro[k])), scale)


@pytest.mark.parametrize("variant", ["periodic_x", "periodic_xy", "insulating", "all_fixed_T"])
def test_rhs_fp64_boundary_variants(variant):
    nx, ny = 40, 24
    kw = {}
    if variant == "periodic_x":
        kw = dict(periodic=[1, 0], angle=90.0)
    elif variant == "periodic_xy":
        kw = dict(periodic=[1, 1], bo_m=0.0, angle=90.0)
    elif variant == "insulating":
        kw = dict(mag_bc=["insulating", "insulating", "fixed", "fixed"], angle=90.0)
    else:
        kw = dict(thermal_bc=["fixed"] * 4, thermal_val=[-0.5, -0.2, -1.0, 0.3])
    bo = kw.pop("bo_m", 1.0)
    prob, st = smooth_case(nx, ny, seed=7, **kw)
    prob["bo_m"] = bo
    if bo == 0.0:
        st["phi"] = np.zeros((ny, nx))
    o, g = pair(prob, st)
    Ro, Rg = o.rhs(), g.rhs()
    for k, name in enumerate(NAMES):
        scale = np.max(np.abs(Ro[k])) + 1e-300
        assert np.max(np.abs(Rg[k] - Ro[k])) <= 1e-10 * scale, (variant, name)


def test_rhs_fp32_within_tolerance():
    prob, st = smooth_case(70, 45, seed=3, precision="fp32")
    o, g = pair(prob, st)
    Ro, Rg = o.rhs(), g.rhs()
    for k, name in enumerate(NAMES):
        err = np.linalg.norm(Rg[k] - Ro[k]) / np.linalg.norm(Ro[k])
        assert err < 2e-4, (name, err)


def test_magnetic_sweeps_fp64_match_oracle():
    prob, st = smooth_case(53, 40, seed=11)
    o, g = pair(prob, st)
    for om in (1.0, 1.7):
        ro = o.mag_sweeps(7, om)
        rg = g.mag_sweeps(7, om)
        assert abs(rg - ro) <= 1e-9 * ro
        assert np.max(np.abs(g.get("phi") - o.get("phi"))) <= 1e-12 * np.max(np.abs(o.get("phi")))


def test_initialisation_matches_oracle():
    prob = wl.droplet64()
    o = orc.Oracle(prob)
    g = lbfs.Solver(prob)
    for name in ("He", "C", "p", "Mx", "S"):
        assert np.max(np.abs(g.get(name) - o.get(name))) <= 1e-13
    # both converge the same magnetic system to the 1e-9 relative residual target
    phi_o, phi_g = o.get("phi"), g.get("phi")
    dphi = phi_o - wl_phi0(prob, o)
    assert np.max(np.abs(phi_g - phi_o)) <= 1e-6 * np.max(np.abs(dphi))
    ob, og = o.observe(), g.observe()
    assert og["volume0"] == pytest.approx(ob["volume0"], rel=1e-13)
    assert og["liquid_fraction"] == pytest.approx(ob["liquid_fraction"], rel=1e-13)


def wl_phi0(prob, o):
    th = np.deg2rad(o.params.angle_deg)
    y, x = np.mgrid[0:o.ny, 0:o.nx] + 0.5
    return -o.params.h0 * (x * np.cos(th) + y * np.sin(th))


def test_step_fp64_matches_oracle_on_64x64_states():
    """The 64^2 FP64 droplet: from identical states the GPU step equals the oracle
    step to rounding, at several points of the trajectory."""
    prob = wl.droplet64()
    o = orc.Oracle(prob)
    g = lbfs.Solver(prob)
    for n_before in (0, 30):
        o.step(n_before)
        state = {k: o.get(k) for k in ("He", "p", "Mx", "My", "C", "phi", "S")}
        g.set_state(state)
        clock = o.observe()
        g.set_time(clock["t"], int(clock["step"]))
        o.step(1)
        g.step(1)
        fl = floors(prob)
        for name in ("He", "p", "Mx", "My", "C", "phi", "S"):
            a, b = g.get(name), o.get(name)
            assert rel_l2(a, b, fl[name]) < 1e-11, (n_before, name, rel_l2(a, b, fl[name]))
        ob, og = o.observe(), g.observe()
        for key in ("liquid_fraction", "solid_ratio", "volume", "mag_residual", "umax", "height", "solid_height",
                    "wall_heat", "umax_drop", "fourier", "peclet", "t"):
            assert og[key] == pytest.approx(ob[key], rel=1e-9, abs=1e-14), key


def test_step_fp32_per_step_relative_l2():
    """FP32 step from the FP64 oracle's state (rounded to the FP32 storage) vs the FP64
    oracle step, at steps 1, 10, 100, 1000 and 2000 of the 64^2 droplet: per-step
    relative L2 <= 1e-5 per field against the field's own norm, with no floor (the
    potential as its perturbation phi - phi0)."""
    prob64 = wl.droplet64()
    o = orc.Oracle(prob64)
    p = orc.make_params(prob64)
    th = np.deg2rad(p.angle_deg)
    y, x = np.mgrid[0:prob64["ny"], 0:prob64["nx"]] + 0.5
    phi0 = -p.h0 * (x * np.cos(th) + y * np.sin(th))
    done = 0
    for at in (1, 10, 100, 1000, 2000):
        o.step(at - done)
        done = at
        obs = o.observe()
        state = {k: o.get(k) for k in ("He", "p", "Mx", "My", "C", "phi", "S")}
        o1 = orc.Oracle(dict(prob64, init_max=0), init=False)
        o1.set_state(state)
        o1.set_time(obs["t"], obs["step"])
        g = lbfs.Solver(wl.with_changes(prob64, precision="fp32", init_max=0))
        g.set_state(state)
        g.set_time(obs["t"], int(obs["step"]))
        o1.step(1)
        g.step(1)
        for name in ("He", "p", "Mx", "My", "C", "phi"):
            a, b = g.get(name), o1.get(name)
            if name == "phi":
                a, b = a - phi0, b - phi0
            e = np.linalg.norm(a - b) / np.linalg.norm(b)
            assert e <= 1e-5, (at, name, e)
        g.close()


def test_trajectory_fp64_200_steps():
    prob = wl.droplet_problem(32, 8.0, ste=0.1, bo_m=2.0, angle_deg=0.0, precision="fp64")
    o = orc.Oracle(prob)
    g = lbfs.Solver(prob)
    g.set_state({k: o.get(k) for k in ("phi",)})
    o.step(200)
    g.step(200)
    fl = floors(prob)
    for name in ("He", "p", "Mx", "My", "C", "phi"):
        assert rel_l2(g.get(name), o.get(name), fl[name]) < 1e-9, name
    assert g.observe()["liquid_fraction"] == pytest.approx(o.observe()["liquid_fraction"], rel=1e-10)


def test_checkpoint_resume_is_bitwise():
    prob = wl.droplet_problem(48, 12.0, ste=0.1, bo_m=1.0, angle_deg=90.0, precision="fp32")
    g = lbfs.Solver(prob)
    g.step(5)
    blob = g.save()
    g.step(7)
    ref = {k: g.get(k) for k in ("He", "p", "Mx", "My", "C", "phi", "S")}
    obs_ref = g.observe()
    h = lbfs.Solver(prob)
    h.load(blob)
    assert h.observe()["step"] == 5
    h.step(7)
    for k, v in ref.items():
        assert np.array_equal(h.get(k), v), k
    assert h.observe()["liquid_fraction"] == obs_ref["liquid_fraction"]


def test_nonfinite_state_is_reported():
    prob = wl.droplet_problem(32, 8.0, ste=0.1, bo_m=1.0, angle_deg=90.0, precision="fp32")
    g = lbfs.Solver(prob)
    He = g.get("He")
    He[5, 7] = np.nan
    g.set("He", He)
    g.step(1)
    obs = g.observe(allow_nonfinite=True)
    assert obs["nonfinite"] == 1
    with pytest.raises(lbfs.LbfsError) as e:
        g.observe()
    assert e.value.status == lbfs.LBFS_E_NONFINITE


@pytest.mark.parametrize("which", ["droplet256", "droplet1024"])
def test_rhs_at_full_size(which):
    """Full-size grids in the benchmark's launch configuration: the whole R(W) of a
    seeded state against the oracle (FP32: relative L2 per field)."""
    prob = wl.droplet256() if which == "droplet256" else wl.droplet1024("fp32")
    prob = wl.with_changes(prob, init_max=0)
    nx, ny = prob["nx"], prob["ny"]
    o = orc.Oracle(prob, init=False)
    st = wl.smooth_state(nx, ny, seed=5, latent=o.params.latent, h0=o.params.h0,
                         angle_deg=prob["angle_deg"])
    o.set_state(st)
    g = lbfs.Solver(prob)
    g.set_state(st)
    Ro, Rg = o.rhs(), g.rhs()
    for k, name in enumerate(NAMES):
        err = np.linalg.norm(Rg[k] - Ro[k]) / np.linalg.norm(Ro[k])
        assert err < 2e-4, (which, name, err)


def test_step_fp64_full_size_observables():
    """1024^2 FP64 (some ten thousand stage tiles over all XCDs): one step from the same state,
    fields and the observables reduced by the last workgroup of the last stage."""
    prob = wl.with_changes(wl.droplet1024("fp64"), init_max=0)
    nx, ny = prob["nx"], prob["ny"]
    o = orc.Oracle(prob, init=False)
    # momentum amplitude for |u| ~ 0.015 in the gas of density 0.01
    st = wl.smooth_state(nx, ny, seed=9, latent=o.params.latent, h0=o.params.h0,
                         angle_deg=prob["angle_deg"], amp_u=5e-5)
    o.set_state(st)
    g = lbfs.Solver(prob)
    g.set_state(st)
    o.step(1)
    g.step(1)
    fl = floors(prob)
    for name in ("He", "p", "Mx", "My", "C", "phi", "S"):
        assert rel_l2(g.get(name), o.get(name), fl[name]) < 1e-10, name
    ob, og = o.observe(), g.observe()
    # (the solid ratio is relative to the initial volume, which only the GPU side has here)
    for key in ("liquid_fraction", "volume", "mag_residual", "umax", "height", "solid_height", "wall_heat"):
        assert og[key] == pytest.approx(ob[key], rel=1e-9, abs=1e-14), key
    # a second step exercises the reset of the completion counter
    o.step(1)
    g.step(1)
    assert g.observe()["liquid_fraction"] == pytest.approx(o.observe()["liquid_fraction"], rel=1e-9)


def test_graph_replay_equals_direct_launches(monkeypatch):
    prob = wl.droplet_problem(96, 24.0, ste=0.1, bo_m=1.5, angle_deg=30.0, precision="fp32")
    a = lbfs.Solver(prob)
    monkeypatch.setenv("LBFS_NO_GRAPH", "1")
    b = lbfs.Solver(prob)
    a.step(25)
    b.step(25)
    for k in ("He", "p", "Mx", "My", "C", "phi", "S"):
        assert np.array_equal(a.get(k), b.get(k)), k
    assert a.observe() == b.observe()


@pytest.mark.parametrize("variant", ["sweeps", "sweeps5", "lbfs", "multigrid", "controlled", "fused"])
def test_multi_step_graphs_equal_direct_launches(monkeypatch, variant):
    """Replays of graphs of up to 8 and up to 3 steps (8, 4, 2 and 3, 2, with single steps
    launched directly) give the fields of direct launches bit for bit, for every
    magnetic method: the potential buffer parity after a replay of n steps is that of n
    single steps."""
    prob = wl.droplet_problem(96, 24.0, ste=0.1, bo_m=1.5, angle_deg=30.0, precision="fp32")
    prob.update(dict(sweeps5=dict(sweeps=5), lbfs=dict(mag_method="lbfs", sweeps=3),
                     multigrid=dict(mag_method="multigrid", sweeps=1),
                     controlled=dict(sweeps=4, mag_max_iters=12, mag_tol=1e-30)).get(variant, {}))
    monkeypatch.setenv("LBFS_NO_GRAPH", "1")
    ref = lbfs.Solver(prob)
    monkeypatch.delenv("LBFS_NO_GRAPH")
    runs = []
    for k in ("8", "3"):
        monkeypatch.setenv("LBFS_GRAPH_STEPS", k)
        runs.append(lbfs.Solver(prob))
    monkeypatch.delenv("LBFS_GRAPH_STEPS")
    for g in [ref] + runs:
        if variant == "fused":
            si, _ = g.tile_shapes_in_use()
            g.set_tile_shapes(si, lbfs.mag_fused_index("fp32"))
    for n in (19, 1, 8, 4):
        for g in [ref] + runs:
            g.step(n)
        for g in runs:
            for k in ("He", "p", "Mx", "My", "C", "phi", "S"):
                assert np.array_equal(g.get(k), ref.get(k)), (variant, n, k)
            assert g.observe() == ref.observe()
    # profiled stepping through the same replays
    kr = ref.step_profiled(30, 11)
    for g in runs:
        g.step_profiled(30, 11)
        assert np.array_equal(g.get("phi"), ref.get("phi")) and np.array_equal(g.get("He"), ref.get("He"))
    assert kr["stage3"][1] == 3


def test_multi_step_graphs_in_a_batch(monkeypatch):
    probs = [wl.droplet_problem(e, e / 4.0, ste=0.1, bo_m=1.0, angle_deg=a, precision="fp32")
             for e, a in ((64, 0.0), (96, 45.0), (72, 90.0))]
    budget = sum(lbfs.Batch.instance_bytes(p) for p in probs) + (1 << 20)
    monkeypatch.setenv("LBFS_GRAPH_STEPS", "1")
    b1 = lbfs.Batch(3, budget)
    monkeypatch.setenv("LBFS_GRAPH_STEPS", "8")
    b8 = lbfs.Batch(3, budget)
    monkeypatch.delenv("LBFS_GRAPH_STEPS")
    for b in (b1, b8):
        for p in probs:
            assert b.admit(p) is not None
    for n in (21, 8):
        b1.step(n)
        b8.step(n)
        o1, o8 = b1.observe(), b8.observe()
        assert o1 == o8
    b1.retire(1)
    b8.retire(1)
    b1.step(17)
    b8.step(17)
    for s in (0, 2):
        for k in ("He", "C", "phi"):
            assert np.array_equal(b1.slot(s).get(k), b8.slot(s).get(k)), (s, k)
    b1.close()
    b8.close()


def test_profiled_steps_equal_plain_steps():
    prob = wl.droplet_problem(64, 16.0, ste=0.1, bo_m=1.0, angle_deg=90.0, precision="fp32")
    a = lbfs.Solver(prob)
    b = lbfs.Solver(prob)
    a.step(30)
    kern = b.step_profiled(30, 7)
    assert kern["stage2"][1] == 5 and kern["mag"][0] > 0
    for k in ("He", "C", "phi", "S"):
        assert np.array_equal(a.get(k), b.get(k)), k


def test_profiled_start_and_result():
    """The two-call form: the same steps and timed launches as the one-call form; a second
    start while a run is pending, and a result with none pending, are refused."""
    prob = wl.droplet_problem(64, 16.0, ste=0.1, bo_m=1.0, angle_deg=90.0, precision="fp32")
    a = lbfs.Solver(prob)
    b = lbfs.Solver(prob)
    ka = a.step_profiled(23, 6)
    b.step_profiled_start(23, 6)
    with pytest.raises(lbfs.LbfsError):
        b.step_profiled_start(5, 1)
    with pytest.raises(lbfs.LbfsError):
        b.step_profiled(5, 1)
    kb = b.profile_result()
    with pytest.raises(lbfs.LbfsError):
        b.profile_result()
    assert {k: v[1] for k, v in ka.items()} == {k: v[1] for k, v in kb.items()}
    assert kb["stage3"][1] == 4 and kb["stage3"][0] > 0
    for k in ("He", "p", "Mx", "My", "C", "phi", "S"):
        assert np.array_equal(a.get(k), b.get(k)), k
    assert a.observe() == b.observe()
    a.close()
    b.close()


@pytest.mark.parametrize("sweeps", [0, 1, 9])
def test_sweep_counts_match_oracle(sweeps):
    """The magnetic phase runs in launches of at most four sweeps; any count matches."""
    prob, st = smooth_case(45, 36, seed=21)
    prob["sweeps"] = sweeps
    o, g = pair(prob, st)
    o.step(1)
    g.step(1)
    fl = floors(prob)
    for name in ("phi", "Mx", "He"):
        assert rel_l2(g.get(name), o.get(name), fl[name]) < 1e-11, (sweeps, name)


def test_prepared_graphs_give_the_same_steps():
    """lbfs_prepare captures every step graph up front (no step runs): the state is
    unchanged by it, and the steps that follow equal those of a solver that captures on
    first use, bit for bit; the same for a batch."""
    prob = wl.droplet_problem(96, 24.0, ste=0.1, bo_m=1.5, angle_deg=30.0, precision="fp32")
    a = lbfs.Solver(prob)
    b = lbfs.Solver(prob)
    before = {k: b.get(k) for k in ("He", "phi", "C")}
    b.prepare()
    for k, v in before.items():
        assert np.array_equal(b.get(k), v), k
    assert b.observe()["step"] == 0
    for n in (1, 16, 3, 17):
        a.step(n)
        b.step(n)
    for k in ("He", "p", "Mx", "My", "C", "phi", "S"):
        assert np.array_equal(a.get(k), b.get(k)), k
    probs = [wl.droplet_problem(e, e / 4.0, ste=0.1, bo_m=1.0, angle_deg=ang, precision="fp32")
             for e, ang in ((64, 0.0), (80, 60.0))]
    budget = sum(lbfs.Batch.instance_bytes(p) for p in probs) + (1 << 20)
    b1, b2 = lbfs.Batch(2, budget), lbfs.Batch(2, budget)
    for bb in (b1, b2):
        for p in probs:
            assert bb.admit(p) is not None
    b2.prepare()
    b1.step(21)
    b2.step(21)
    assert b1.observe() == b2.observe()
    b1.close()
    b2.close()
