"""Parity of the magnetic LBFS pseudo-time solve (Sec. 3.1, Eq. 17 by SSP-RK3) on the
GPU with the FP64 oracle, whose face fluxes are the literal m* moments.

FP64 agrees to rounding, FP32 within the relative L2 bound 1e-5 of the other parity
tests. The kernel blocks up to four pseudo-steps per launch in LDS, so step counts
around that limit, every tile shape, ragged grids, periodic and insulating walls and
the full 1024^2 grid are covered.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2511_10257_amd import lbfs, workloads as wl

pytestmark = pytest.mark.gpu


def case(nx, ny, seed, precision, **kw):
    angle = kw.pop("angle", 60.0)
    prob = wl.droplet_problem(nx, ny / 4.0, ste=0.1, bo_m=1.0, angle_deg=angle, precision=precision, ny=ny)
    prob.update(init_max=0, mag_method="lbfs", **kw)
    o = orc.Oracle(prob, init=False)
    st = wl.smooth_state(nx, ny, seed, latent=o.params.latent, h0=o.params.h0, angle_deg=angle)
    o.set_state(st)
    g = lbfs.Solver(prob)
    g.set_state(st)
    return prob, o, g, st


def floor_phi(prob, o):
    return max(o.params.h0 * prob["drop"][2], 1e-30)


def rel_l2(a, b, floor):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), floor * np.sqrt(b.size))


def check_phi(prob, o, g, precision, what):
    po, pg = o.get("phi"), g.get("phi")
    if precision == "fp64":
        err = np.max(np.abs(pg - po))
        assert err <= 1e-12 * np.max(np.abs(po)), (what, err)
    else:
        err = rel_l2(pg, po, floor_phi(prob, o))
        assert err < 1e-5, (what, err)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("nsteps", [0, 1, 4, 5, 9])
def test_pseudo_steps_match_oracle(precision, nsteps):
    prob, o, g, _ = case(150, 70, seed=31 + nsteps, precision=precision)
    D = prob.get("mag_lbfs_d", 1.0)
    ro = o.mag_lbfs(nsteps, D, 0.0)
    rg = g.mag_pseudo_steps(nsteps)
    check_phi(prob, o, g, precision, nsteps)
    assert rg == pytest.approx(ro, rel=1e-9 if precision == "fp64" else 2e-2)


@pytest.mark.parametrize("variant", ["periodic_x", "insulating", "explicit_dtau"])
def test_pseudo_steps_boundary_variants(variant):
    kw = dict(periodic_x=dict(periodic=[1, 0], angle=90.0),
              insulating=dict(mag_bc=["insulating", "insulating", "fixed", "fixed"], angle=90.0),
              explicit_dtau=dict(mag_lbfs_d=2.5, mag_lbfs_dtau=0.04, angle=20.0))[variant]
    prob, o, g, _ = case(66, 41, seed=5, precision="fp64", **kw)
    o.mag_lbfs(5, prob.get("mag_lbfs_d", 1.0), prob.get("mag_lbfs_dtau", 0.0))
    g.mag_pseudo_steps(5)
    check_phi(prob, o, g, "fp64", variant)


def test_every_tile_shape_gives_the_same_potential():
    """Each cell update is the same arithmetic whatever the tile: bitwise equal results."""
    prob, _, g, st = case(201, 77, seed=8, precision="fp32")
    ref = None
    for shape in range(len(lbfs.tile_shapes("mag", "fp32"))):
        g.set_state(st)
        si, _ = g.tile_shapes_in_use()
        g.set_tile_shapes(si, shape)
        g.mag_pseudo_steps(5)
        phi = g.get("phi")
        if ref is None:
            ref = phi
        assert np.array_equal(phi, ref), shape


@pytest.mark.parametrize("sweeps", [0, 2, 5])
def test_step_with_pseudo_time_method_matches_oracle(sweeps):
    prob, o, g, _ = case(45, 36, seed=21, precision="fp64", sweeps=sweeps)
    o.step(3)
    g.step(3)
    fl = dict(He=o.params.latent, Mx=o.params.rho[1] / 3.0 * o.params.sigma / o.params.mu[1],
              phi=floor_phi(prob, o), C=1.0)
    for name in ("phi", "He", "Mx", "C"):
        assert rel_l2(g.get(name), o.get(name), fl[name]) < 1e-10, (sweeps, name)
    ob, og = o.observe(), g.observe()
    assert og["mag_residual"] == pytest.approx(ob["mag_residual"], rel=1e-8)


def test_step_fp32_with_pseudo_time_method():
    prob, o, g, _ = case(70, 45, seed=3, precision="fp32", sweeps=4)
    o.step(1)
    g.step(1)
    assert rel_l2(g.get("phi"), o.get("phi"), floor_phi(prob, o)) < 1e-5
    assert rel_l2(g.get("He"), o.get("He"), o.params.latent) < 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_size_pseudo_steps_match_oracle(precision):
    """The 1024^2 droplet in the launch configuration of the benchmark (64 x 32 magnetic
    tiles): four pseudo-steps (one launch) over the whole grid."""
    prob = wl.with_changes(wl.droplet1024(precision), init_max=0, mag_method="lbfs")
    nx, ny = prob["nx"], prob["ny"]
    o = orc.Oracle(prob, init=False)
    st = wl.smooth_state(nx, ny, seed=12, latent=o.params.latent, h0=o.params.h0, angle_deg=prob["angle_deg"])
    o.set_state(st)
    g = lbfs.Solver(prob)
    g.set_state(st)
    assert g.tile_shapes_in_use()[1] == 1
    o.mag_lbfs(4, 1.0, 0.0)
    g.mag_pseudo_steps(4)
    check_phi(prob, o, g, precision, "1024")


def test_residual_falls_under_repeated_pseudo_steps():
    prob, _, g, _ = case(256, 256, seed=2, precision="fp32")
    res = [g.mag_pseudo_steps(30) for _ in range(8)]
    assert all(b < a for a, b in zip(res, res[1:])), res


def test_batches_reject_the_pseudo_time_method():
    prob = wl.droplet_problem(64, 16.0, ste=0.1, bo_m=0.5, angle_deg=90.0, precision="fp32")
    batch = lbfs.Batch(2, 2 * lbfs.Batch.instance_bytes(prob))
    with pytest.raises(lbfs.LbfsError) as ei:
        batch.admit(wl.with_changes(prob, mag_method="lbfs"))
    assert ei.value.status == lbfs.LBFS_E_INVAL
    slot = batch.admit(prob)
    assert slot is not None
    h = batch.slot(slot)._h
    assert lbfs.lib().lbfs_mag_pseudo_steps(h, 1, None) == lbfs.LBFS_E_STATE
    batch.close()


@pytest.mark.parametrize("method", ["sweeps", "lbfs"])
def test_convergence_control_with_unreachable_target_is_the_fixed_count(method):
    """Every chunk runs when the target is never met: chunks of 4 up to 12 iterations
    equal 12 iterations per step bit for bit (graph replay of the gated launches)."""
    base = wl.droplet_problem(96, 24.0, ste=0.1, bo_m=1.5, angle_deg=30.0, precision="fp32")
    base["mag_method"] = method
    a = lbfs.Solver(wl.with_changes(base, sweeps=4, mag_max_iters=12, mag_tol=0.0))
    b = lbfs.Solver(wl.with_changes(base, sweeps=12))
    a.step(5)
    b.step(5)
    for k in ("He", "p", "Mx", "My", "C", "phi", "S"):
        assert np.array_equal(a.get(k), b.get(k)), k
    assert a.observe()["mag_residual"] == b.observe()["mag_residual"]


@pytest.mark.parametrize("method", ["sweeps", "lbfs"])
def test_convergence_control_matches_oracle(method):
    """A reachable target: the oracle's chunk residuals are computed first and the target
    is put halfway (geometrically) between two of them, so both sides stop after the
    same chunk; then three steps agree to FP64 rounding."""
    prob, o, g, st = case(48, 40, seed=17, precision="fp64", sweeps=2)
    prob["mag_method"] = method
    st = dict(st, phi=st["phi"] * 1.02)
    probe = orc.Oracle(prob, init=False)
    probe.set_state(st)
    res = [probe.mag_sweeps(2, 1.0) if method == "sweeps" else probe.mag_lbfs(2, 1.0, 0.0) for _ in range(6)]
    tol = float(np.sqrt(res[3] * res[4]))
    prob.update(mag_max_iters=200, mag_tol=tol)
    o = orc.Oracle(prob, init=False)
    g = lbfs.Solver(prob)
    o.set_state(st)
    g.set_state(st)
    o.step(1)
    g.step(1)
    assert g.observe()["mag_residual"] <= tol
    assert g.observe()["mag_residual"] == pytest.approx(o.observe()["mag_residual"], rel=1e-8)
    o.step(2)
    g.step(2)
    fl = dict(He=o.params.latent, Mx=o.params.rho[1] / 3.0 * o.params.sigma / o.params.mu[1],
              phi=floor_phi(prob, o), C=1.0)
    for name in ("phi", "He", "Mx", "C"):
        assert rel_l2(g.get(name), o.get(name), fl[name]) < 1e-10, name


def test_convergence_controlled_step_at_full_size():
    """1024^2 FP32 with a target of half the residual at the step start: the step
    ends at or below the target, and its result equals the fixed count of the chunks it
    used (found by hand from the same state)."""
    prob = wl.droplet1024("fp32")
    a = lbfs.Solver(prob)
    a.step(2)
    st = {k: a.get(k) for k in ("He", "p", "Mx", "My", "C", "phi", "S")}
    r_start = a.mag_sweeps(0)
    tol = 0.5 * r_start
    ctl = lbfs.Solver(wl.with_changes(prob, mag_max_iters=400, mag_tol=tol, init_max=0))
    ctl.set_state(st)
    ctl.step(1)
    r = ctl.observe()["mag_residual"]
    assert r <= tol
    # the chunk count it used, found by hand from the same state
    probe = lbfs.Solver(wl.with_changes(prob, init_max=0))
    probe.set_state(st)
    used = 0
    while True:
        used += 4
        if probe.mag_sweeps(4) <= tol or used >= 400:
            break
    fixed = lbfs.Solver(wl.with_changes(prob, sweeps=used, init_max=0))
    fixed.set_state(st)
    fixed.step(1)
    assert np.array_equal(ctl.get("phi"), fixed.get("phi")) and np.array_equal(ctl.get("He"), fixed.get("He"))
