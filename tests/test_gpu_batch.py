"""Batched instances (lbfs_batch_*) against the same problems solved alone.

A batch runs the same kernels over the concatenated tiles of all live instances, so
every instance must reproduce its stand-alone fields and observables bit for bit,
whatever was admitted or retired around it. One FP64 member is also checked against
the oracle directly.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2511_10257_amd import lbfs, workloads as wl

pytestmark = pytest.mark.gpu

STATE = ("He", "p", "Mx", "My", "C", "phi", "S", "T", "Fl")
OBS = ("liquid_fraction", "solid_ratio", "volume", "volume0", "mag_residual", "umax", "umax_drop",
       "height", "solid_height", "wall_heat", "step", "t")


def _mixed(precision: str):
    """Uneven sizes (ragged tile edges), both field directions, several Bo_m and Ste."""
    shapes = [(37, 29, 9.0, 0.12, 1.3, 90.0), (64, 64, 16.0, 0.1, 0.5, 0.0), (96, 40, 12.0, 0.2, 1.9, 35.0),
              (48, 72, 12.0, 0.07, 0.0, 60.0), (128, 96, 32.0, 0.15, 1.0, 10.0)]
    out = []
    for nx, ny, r, ste, bo, ang in shapes:
        p = wl.droplet_problem(nx, r, ste=ste, bo_m=bo, angle_deg=ang, precision=precision, ny=ny)
        out.append(p)
    return out


def _same(a, b, what):
    for name in STATE:
        x, y = a.get(name), b.get(name)
        assert np.array_equal(x, y), f"{what}: field {name} differs (max {np.max(np.abs(x - y))})"


def _budget(probs, extra=1 << 20):
    return sum(lbfs.Batch.instance_bytes(p) for p in probs) + extra


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_equals_alone_with_admit_and_retire(precision):
    probs = _mixed(precision)
    a, b, c, d, e = probs
    batch = lbfs.Batch(8, _budget(probs), precision=precision)
    sa, sb = batch.admit(a), batch.admit(b)
    batch.step(10)
    sc = batch.admit(c)
    batch.step(10)
    batch.retire(sb)                       # frees memory in the middle of the buffer
    sd = batch.admit(d)
    se = batch.admit(e)
    batch.step(7)
    obs = batch.observe()
    assert set(obs) == {sa, sc, sd, se}
    for prob, slot, steps in ((a, sa, 27), (c, sc, 17), (d, sd, 7), (e, se, 7)):
        alone = lbfs.Solver(prob)
        alone.step(steps)
        ref = alone.observe()
        _same(batch.slot(slot), alone, f"{prob['nx']}x{prob['ny']} after {steps} steps")
        for k in OBS:
            assert obs[slot][k] == ref[k], (k, obs[slot][k], ref[k])
        alone.close()
    batch.close()


def test_batch_member_matches_oracle_fp64():
    from oracle import oracle as orc
    prob = wl.droplet_problem(40, 10.0, ste=0.1, bo_m=1.2, angle_deg=30.0, precision="fp64", ny=33)
    other = wl.droplet_problem(64, 16.0, ste=0.2, bo_m=0.4, angle_deg=90.0, precision="fp64")
    batch = lbfs.Batch(4, _budget([prob, other]), precision="fp64")
    batch.admit(other)
    slot = batch.admit(prob)
    batch.step(20)
    o = orc.Oracle(prob)
    o.step(20)
    view = batch.slot(slot)
    for name in ("He", "p", "Mx", "My", "C", "phi", "S"):
        x, y = view.get(name), o.get(name)
        scale = max(1.0, float(np.max(np.abs(y))))
        assert np.max(np.abs(x - y)) <= 1e-10 * scale, name
    batch.close()


def test_batch_rejections():
    p32 = wl.droplet_problem(64, 16.0, ste=0.1, bo_m=0.5, angle_deg=90.0, precision="fp32")
    need = lbfs.Batch.instance_bytes(p32)
    assert need > 0
    batch = lbfs.Batch(2, need + (1 << 16))
    s0 = batch.admit(p32)
    assert s0 is not None
    assert batch.admit(p32) is None                    # no room in the buffer
    info = batch.info()
    assert info["live"] == 1 and info["cells"] == 64 * 64
    with pytest.raises(lbfs.LbfsError) as ei:
        batch.admit(wl.with_changes(p32, precision="fp64"))
    assert ei.value.status == lbfs.LBFS_E_INVAL
    with pytest.raises(lbfs.LbfsError) as ei:
        batch.admit(wl.with_changes(p32, sweeps=2))
    assert ei.value.status == lbfs.LBFS_E_INVAL
    # a borrowed handle cannot be stepped on its own
    h = batch.slot(s0)._h
    assert lbfs.lib().lbfs_step(h, 1) == lbfs.LBFS_E_STATE
    assert lbfs.lib().lbfs_mag_sweeps(h, 1, 1.0, None) == lbfs.LBFS_E_STATE
    batch.retire(s0)
    assert batch.admit(p32) is not None                # memory and slot reused
    batch.close()

    small = lbfs.Batch(1, 8 * need)
    assert small.admit(p32) is not None
    assert small.admit(p32) is None                    # no free slot
    small.close()


def test_batch_empty_and_idle_calls():
    batch = lbfs.Batch(3, 1 << 20)
    batch.step(5)                                      # nothing live: no launches
    assert batch.observe() == {}
    kern = batch.step_profiled(4, 2)
    assert all(v[1] == 0 for v in kern.values())
    batch.close()


def test_batch_profiled_equals_plain():
    probs = _mixed("fp32")[:3]
    b1 = lbfs.Batch(4, _budget(probs))
    b2 = lbfs.Batch(4, _budget(probs))
    s1 = [b1.admit(p) for p in probs]
    s2 = [b2.admit(p) for p in probs]
    b1.step(12)
    kern = b2.step_profiled(12, 5)
    assert kern["stage1"][1] == 3 and kern["mag"][1] == 3
    for x, y in zip(s1, s2):
        _same(b1.slot(x), b2.slot(y), "profiled batch")
    # the two-call form
    b1.step(9)
    b2.step_profiled_start(9, 4)
    kern = b2.profile_result()
    assert kern["stage2"][1] == 3
    for x, y in zip(s1, s2):
        _same(b1.slot(x), b2.slot(y), "profiled batch, two calls")
    b1.close()
    b2.close()


def test_full_size_batch_members_equal_alone():
    """The 64-instance workload (1.78 M cells) in the benchmark's launch configuration
    (autotuned tile shapes, graph replay): sampled members equal their solves alone,
    with the same shapes, bit for bit."""
    probs = wl.batch64()
    batch = lbfs.Batch(len(probs), _budget(probs, extra=64 << 20))
    slots = [batch.admit(p) for p in probs]
    assert None not in slots
    batch.autotune(reps=3)
    si, mi = batch.tile_shapes_in_use()
    batch.step(6)
    obs = batch.observe()
    assert len(obs) == 64 and not any(o["nonfinite"] for o in obs.values())
    for k in (0, 7, 19, 23, 38, 41, 50, 63):
        alone = lbfs.Solver(probs[k])
        alone.set_tile_shapes(si, mi)
        alone.step(6)
        view = batch.slot(slots[k])
        for f in STATE:
            assert np.array_equal(view.get(f), alone.get(f)), (k, f)
        ref = alone.observe()
        for key in ("liquid_fraction", "volume", "umax", "step"):
            assert obs[slots[k]][key] == ref[key], (k, key)
        alone.close()
    batch.close()
