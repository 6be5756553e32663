"""Tile shapes change the time, never the result: every candidate shape of the stage and
magnetic kernels gives the same fields bit for bit, and the autotuner leaves the state
as it found it (solver and batch)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2511_10257_amd import lbfs, workloads as wl

pytestmark = pytest.mark.gpu

FIELDS = ("He", "p", "Mx", "My", "C", "phi", "S")


def _prob(precision):
    # ragged against every candidate tile (77 x 53)
    return wl.droplet_problem(77, 18.0, ste=0.1, bo_m=1.3, angle_deg=35.0, precision=precision, ny=53)


def _fields(s):
    return {f: s.get(f) for f in FIELDS}


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_every_shape_gives_the_same_fields(precision):
    prob = _prob(precision)
    ref = lbfs.Solver(prob)
    ref.step(12)
    want, want_obs = _fields(ref), ref.observe()
    ns, nm = len(lbfs.tile_shapes("stage", precision)), len(lbfs.tile_shapes("mag", precision))
    combos = [(k, 0) for k in range(1, ns)] + [(0, k) for k in range(1, nm)] + [(ns - 1, nm - 1)]
    for si, mi in combos:
        s = lbfs.Solver(prob)
        s.set_tile_shapes(si, mi)
        s.step(12)
        got = _fields(s)
        for f in FIELDS:
            assert np.array_equal(got[f], want[f]), (si, mi, f)
        obs = s.observe()
        for k in ("liquid_fraction", "volume", "umax", "solid_ratio", "mag_residual"):
            assert obs[k] == pytest.approx(want_obs[k], rel=1e-12, abs=1e-300), (si, mi, k)
        s.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_autotune_keeps_the_state(precision):
    prob = _prob(precision)
    a, b = lbfs.Solver(prob), lbfs.Solver(prob)
    a.step(10)
    b.step(10)
    before = a.observe()
    res = a.autotune(reps=3)
    assert all(t > 0 for t in res["stage_ms"] + res["mag_ms"])
    assert (a.observe()["t"], a.observe()["step"]) == (before["t"], before["step"])
    assert len(res["stage_ms"]) == len(lbfs.tile_shapes("stage", precision))
    assert all(t > 0 for t in res["stage_ms"] + res["mag_ms"])
    after = a.observe()
    # the same state, summed over the tuned tiles (another order)
    assert after["umax"] == before["umax"]
    for k in ("liquid_fraction", "volume", "solid_ratio"):
        assert after[k] == pytest.approx(before[k], rel=1e-12, abs=1e-300)
    # the residual is recomputed for the current potential and permeability (a step reports
    # it with the permeability of the step's start); b computes the same one by a
    # sweep-free magnetic call
    assert after["mag_residual"] == pytest.approx(b.mag_sweeps(0), rel=1e-9)
    a.step(10)
    b.step(10)
    for f in FIELDS:
        assert np.array_equal(a.get(f), b.get(f)), f


def test_batch_autotune_keeps_every_member():
    probs = [wl.droplet_problem(n, n / 4.0, ste=0.1 + 0.02 * k, bo_m=0.5 * k, angle_deg=20.0 * k, ny=m)
             for k, (n, m) in enumerate(((64, 64), (96, 48), (40, 72), (128, 128)))]
    batch = lbfs.Batch(4, sum(lbfs.Batch.instance_bytes(p) for p in probs) + (1 << 20))
    slots = [batch.admit(p) for p in probs]
    batch.step(6)
    before = batch.observe()
    res = batch.autotune(reps=3)
    after = batch.observe()
    for k in slots:
        assert (after[k]["t"], after[k]["step"]) == (before[k]["t"], before[k]["step"])
        assert after[k]["umax"] == before[k]["umax"]
        assert after[k]["liquid_fraction"] == pytest.approx(before[k]["liquid_fraction"], rel=1e-12)
    assert 0 <= res["stage_shape"] < len(lbfs.tile_shapes("stage"))
    assert 0 <= res["mag_shape"] < len(lbfs.tile_shapes("mag"))
    batch.step(6)
    for p, k in zip(probs, slots):
        alone = lbfs.Solver(p)
        alone.step(12)
        view = batch.slot(k)
        for f in FIELDS:
            assert np.array_equal(view.get(f), alone.get(f)), (k, f)
        alone.close()
    batch.close()


@pytest.mark.parametrize("axis", ["x", "y"])
def test_magnetic_sweeps_on_a_periodic_axis_shorter_than_the_halo(axis):
    # 6 cells along the periodic axis: the 9-cell halo of the magnetic kernel wraps twice
    nx, ny = (6, 30) if axis == "x" else (30, 6)
    prob = wl.droplet_problem(nx, 4.0, ste=0.1, bo_m=1.0, angle_deg=90.0 if axis == "x" else 0.0,
                              precision="fp64", ny=ny)
    prob.update(init_max=0, periodic=[1, 0] if axis == "x" else [0, 1])
    o = orc.Oracle(prob, init=False)
    st = wl.smooth_state(nx, ny, 5, latent=o.params.latent, h0=o.params.h0, angle_deg=prob["angle_deg"])
    g = lbfs.Solver(prob)
    o.set_state(st)
    g.set_state(st)
    ro, rg = o.mag_sweeps(4, 1.0), g.mag_sweeps(4, 1.0)
    assert abs(rg - ro) <= 1e-9 * ro
    assert np.max(np.abs(g.get("phi") - o.get("phi"))) <= 1e-12 * np.max(np.abs(o.get("phi")))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("variant", ["droplet", "periodic_x", "insulating_wetting", "tiny_periodic"])
def test_sweeps_inside_stage_one_give_the_same_fields(precision, variant):
    """The magnetic "shape" that runs the step's sweeps inside stage 1 (no magnetic
    launch) computes every field bit for bit as the separate magnetic kernel does, with
    graphs and without, for every stage shape; the residual observable is the same sum in
    another order."""
    prob = _prob(precision)
    if variant == "periodic_x":
        prob.update(periodic=[1, 0], angle_deg=90.0, nx=78)
    elif variant == "insulating_wetting":
        prob.update(mag_bc=["insulating", "insulating", "fixed", "fixed"], angle_deg=90.0,
                    contact_angle=[70.0, 110.0, 60.0, 90.0])
    elif variant == "tiny_periodic":
        prob = wl.droplet_problem(6, 2.0, ste=0.1, bo_m=1.0, angle_deg=90.0, precision=precision, ny=30)
        prob.update(periodic=[1, 0])
    fused = lbfs.mag_fused_index(precision)
    ref = lbfs.Solver(prob)
    ref.step(9)
    want, want_obs = _fields(ref), ref.observe()
    for si in range(len(lbfs.tile_shapes("stage", precision))):
        s = lbfs.Solver(prob)
        s.set_tile_shapes(si, fused)
        assert s.tile_shapes_in_use() == (si, fused)
        s.step(9)
        got = _fields(s)
        for f in FIELDS:
            assert np.array_equal(got[f], want[f]), (variant, si, f)
        obs = s.observe()
        for k in ("liquid_fraction", "volume", "umax", "solid_ratio"):
            assert obs[k] == pytest.approx(want_obs[k], rel=1e-12, abs=1e-300), (si, k)
        assert obs["mag_residual"] == pytest.approx(want_obs["mag_residual"], rel=1e-9)
        kern = s.step_profiled(4, 2)
        assert kern["mag"][1] == 0 and kern["stage1"][1] == 2
        s.close()


def test_sweeps_inside_stage_one_need_a_fixed_small_count():
    base = _prob("fp32")
    fused = lbfs.mag_fused_index()
    for kw in (dict(mag_method="lbfs"), dict(sweeps=5), dict(mag_max_iters=40, mag_tol=1e-6)):
        s = lbfs.Solver(wl.with_changes(base, **kw))
        with pytest.raises(lbfs.LbfsError) as ei:
            s.set_tile_shapes(0, fused)
        assert ei.value.status == lbfs.LBFS_E_INVAL
        s.close()
    assert lbfs.shape_name(lbfs.mag_shape(fused)) == "in-stage-1"


@pytest.mark.parametrize("edge, mag_shape", [(256, 0), (362, 0), (363, 2), (512, 2), (513, 1), (1024, 1)])
def test_default_magnetic_shape_by_grid_size(edge, mag_shape):
    """Without autotuning a single solve takes 32 x 8 magnetic tiles up to 2^17 cells,
    64 x 16 up to 512^2 and 64 x 32 above; the stage shape is the table's first."""
    prob = wl.with_changes(wl.droplet_problem(edge, edge / 4.0, ste=0.1, bo_m=0.5, angle_deg=90.0,
                                              precision="fp32"), init_max=0)
    s = lbfs.Solver(prob)
    assert s.tile_shapes_in_use() == (0, mag_shape)


@pytest.mark.parametrize("edge, shapes", [(256, (0, 0)), (512, (0, 2)), (513, (4, 1))])
def test_default_fp64_stage_shape_by_grid_size(edge, shapes):
    """FP64 solves above 512^2 cells start with 12 x 7 stage tiles, smaller ones with the
    table's first; a batch of FP64 instances follows its total cells the same way."""
    prob = wl.with_changes(wl.droplet_problem(edge, edge / 4.0, ste=0.1, bo_m=0.5, angle_deg=90.0,
                                              precision="fp64"), init_max=0)
    s = lbfs.Solver(prob)
    assert s.tile_shapes_in_use() == shapes
    tx, ty, _, _ = lbfs.tile_shapes("stage", "fp64")[shapes[0]]
    assert (tx, ty) == ((12, 7) if edge > 512 else (10, 8))
    s.close()
    if edge == 512:
        two = wl.with_changes(wl.droplet_problem(384, 96.0, ste=0.1, bo_m=0.5, angle_deg=90.0,
                                                 precision="fp64"), init_max=0)
        b = lbfs.Batch(4, 2 * lbfs.Batch.instance_bytes(two) + (1 << 20), precision="fp64")
        b.admit(two)
        assert b.tile_shapes_in_use()[0] == 0
        b.admit(two)   # 2 x 384^2 = 294912 cells, above 512^2
        assert b.tile_shapes_in_use()[0] == 4
        b.close()


def test_batch_magnetic_shape_follows_its_size_until_shapes_are_given():
    """A batch without given shapes takes, after every admission and retirement, the
    magnetic shape a single solve of its total cells would take, except where those tiles
    would cover more than 15% beyond the instances' cells; given shapes stay. The tile
    shapes change no field (checked bit for bit against a solve alone)."""
    def prob(edge):
        return wl.with_changes(wl.droplet_problem(edge, edge / 4.0, ste=0.1, bo_m=0.5, angle_deg=90.0,
                                                  precision="fp32"), init_max=0)

    def budget(probs):
        return sum(lbfs.Batch.instance_bytes(p) for p in probs) + (1 << 20)

    # 3 x 256^2 = 196608 cells: 64 x 16 (above 2^17); a fourth: 262144, still 64 x 16;
    # a 320^2 one more: 364544, 64 x 32 (above 512^2)
    big = [prob(256) for _ in range(4)] + [prob(320)]
    b = lbfs.Batch(8, budget(big))
    slots = [b.admit(p) for p in big[:2]]
    assert b.tile_shapes_in_use() == (0, 0)
    slots.append(b.admit(big[2]))
    assert b.tile_shapes_in_use() == (0, 2)
    slots.append(b.admit(big[3]))
    slots.append(b.admit(big[4]))
    assert b.tile_shapes_in_use() == (0, 1)
    b.step(6)
    b.retire(slots.pop())
    b.retire(slots.pop())
    assert b.tile_shapes_in_use() == (0, 2)
    alone = lbfs.Solver(big[0])
    alone.step(6)
    for name in ("He", "p", "Mx", "My", "C", "phi", "S"):
        assert np.array_equal(b.slot(slots[0]).get(name), alone.get(name)), name
    alone.close()
    b.close()
    # 15 x 96^2 = 138240 cells, above 2^17, but 64 x 16 tiles cover 96 x 96 as 128 x 96
    small = [prob(96) for _ in range(15)]
    b = lbfs.Batch(16, budget(small))
    for p in small:
        b.admit(p)
    assert b.tile_shapes_in_use() == (0, 0)
    b.close()
    # given shapes stay through later admissions
    b = lbfs.Batch(8, budget(big))
    b.set_tile_shapes(0, 0)
    for p in big:
        b.admit(p)
    assert b.tile_shapes_in_use() == (0, 0)
    b.close()


def test_observables_follow_written_and_loaded_states():
    """Writing fields or loading a checkpoint changes what the next observe reports, for a
    single solve and for a batch member written through its borrowed handle."""
    prob = _prob("fp32")
    a = lbfs.Solver(prob)
    a.step(7)
    want = a.observe()
    st = _fields(a)
    b = lbfs.Solver(prob)
    b.observe()
    b.set_state(st)
    got = b.observe()
    for k in ("liquid_fraction", "volume", "umax", "solid_ratio", "height"):
        assert got[k] == want[k], k
    c = lbfs.Solver(prob)
    c.observe()
    c.load(a.save())
    got = c.observe()
    for k in ("liquid_fraction", "volume", "umax", "t", "step"):
        assert got[k] == want[k], k
    batch = lbfs.Batch(1, lbfs.Batch.instance_bytes(prob) + (1 << 20))
    k = batch.admit(prob)
    batch.observe()
    batch.slot(k).set_state(st)
    got = batch.observe()[k]
    for key in ("liquid_fraction", "volume", "umax", "solid_ratio"):
        assert got[key] == want[key], key
    batch.close()
