"""lbfs_step_fields, the entry point that allocates nothing (the library's static
scratch holds the stage fields and lists), against lbfs_step on a solver: the same
state in the same storage, the same number of steps, the same fields bit for bit. Two
calls in a row, the second on a smaller grid (the scratch keeps the first call's
contents), in FP32 and in FP64; a problem larger than the scratch is refused."""
import ctypes as C
import struct

import numpy as np
import pytest
import torch

from paper_2511_10257_amd import lbfs, workloads as wl

pytestmark = pytest.mark.gpu

HEADER = struct.Struct("<IIiiiiddq")   # the checkpoint header of lbfs_save_state


def native_state(solver, prob):
    """The solver's state in its own storage, from its checkpoint: He, p, Mx, My (the
    instance precision), C (FP64), phi - phi0 and S (the instance precision)."""
    blob = solver.save()
    n = prob["nx"] * prob["ny"]
    t = np.float64 if prob["precision"] == "fp64" else np.float32
    off, out = HEADER.size, []
    for k in range(7):
        dt = np.float64 if k == 4 else t
        a = np.frombuffer(blob, dtype=dt, count=n, offset=off).reshape(prob["ny"], prob["nx"]).copy()
        off += a.nbytes
        out.append(a)
    return out


def step_fields(prob, arrays, nsteps):
    dev = [torch.from_numpy(a).to("cuda:0") for a in arrays]
    ptrs = (C.c_void_p * 7)(*[t.data_ptr() for t in dev])
    params = lbfs.make_params(prob)
    stream = torch.cuda.current_stream().cuda_stream
    rc = lbfs.lib().lbfs_step_fields(C.byref(params), ptrs, int(nsteps), C.c_void_p(stream))
    torch.cuda.synchronize()
    return rc, [t.cpu().numpy() for t in dev]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_step_fields_equals_solver_steps_twice_second_smaller(precision):
    cases = [(wl.droplet_problem(96, 20.0, ste=0.1, bo_m=1.5, angle_deg=30.0, precision=precision, ny=80), 19),
             (wl.droplet_problem(64, 14.0, ste=0.15, bo_m=0.7, angle_deg=80.0, precision=precision, ny=48), 6)]
    for prob, nsteps in cases:
        s = lbfs.Solver(prob)
        s.step(5)                          # a state with flow, freezing and a settled potential
        start = native_state(s, prob)
        s.step(nsteps)
        ref = native_state(s, prob)
        rc, got = step_fields(prob, start, nsteps)
        assert rc == lbfs.LBFS_OK, lbfs.strerror(rc)
        for k, (a, b) in enumerate(zip(got, ref)):
            assert np.array_equal(a, b), (prob["nx"], prob["ny"], k, float(np.max(np.abs(a - b))))
        s.close()


def test_step_fields_fp64_above_512_squared():
    """An FP64 grid above 512^2 cells, where the stage kernels take 12 x 7 tiles in both
    entry points, then a small one after it."""
    big = wl.with_changes(wl.droplet_problem(520, 130.0, ste=0.1, bo_m=1.5, angle_deg=0.0, precision="fp64"),
                          init_max=0)
    small = wl.droplet_problem(64, 14.0, ste=0.15, bo_m=0.7, angle_deg=80.0, precision="fp64", ny=48)
    for prob, nsteps in ((big, 3), (small, 4)):
        s = lbfs.Solver(prob)
        s.step(2)
        start = native_state(s, prob)
        s.step(nsteps)
        ref = native_state(s, prob)
        rc, got = step_fields(prob, start, nsteps)
        assert rc == lbfs.LBFS_OK, lbfs.strerror(rc)
        for k, (a, b) in enumerate(zip(got, ref)):
            assert np.array_equal(a, b), (prob["nx"], prob["ny"], k, float(np.max(np.abs(a - b))))
        s.close()


def test_step_fields_refuses_what_does_not_fit():
    prob = wl.droplet_problem(1536, 384.0, ste=0.1, bo_m=1.0, angle_deg=0.0, precision="fp32")
    n = prob["nx"] * prob["ny"]
    arrays = [np.zeros((prob["ny"], prob["nx"]), dtype=np.float64 if k == 4 else np.float32) for k in range(7)]
    rc, _ = step_fields(prob, arrays, 1)
    assert rc == lbfs.LBFS_E_NOMEM and n * 64 > (80 << 20)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_step_fields_replayed_from_a_captured_graph(precision):
    """The entry point captured into a HIP graph (the use it is for: no allocation, no
    memset node, only kernel and copy nodes) and replayed four times, with eager work and
    synchronisation between the replays: every replay equals the same steps taken by a
    solver, bit for bit."""
    prob = wl.droplet_problem(72, 16.0, ste=0.1, bo_m=1.2, angle_deg=45.0, precision=precision, ny=56)
    nsteps = 3   # odd: each replay ends with the copy of the potential back to the caller's field
    s = lbfs.Solver(prob)
    s.step(4)
    dev = [torch.from_numpy(a).to("cuda:0") for a in native_state(s, prob)]
    ptrs = (C.c_void_p * 7)(*[t.data_ptr() for t in dev])
    params = lbfs.make_params(prob)
    # set-up outside the capture (the first call on a device finds the static scratch)
    rc = lbfs.lib().lbfs_step_fields(C.byref(params), ptrs, 0, C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == lbfs.LBFS_OK, lbfs.strerror(rc)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    codes = []
    with torch.cuda.graph(g, stream=side):
        codes.append(lbfs.lib().lbfs_step_fields(C.byref(params), ptrs, nsteps,
                                                 C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    assert codes == [lbfs.LBFS_OK], codes
    torch.cuda.synchronize()
    for replay in range(4):
        g.replay()
        torch.cuda.synchronize()
        s.step(nsteps)
        ref = native_state(s, prob)
        scratch = torch.ones(1 << 20, device="cuda:0").sum()   # eager work between replays
        torch.cuda.synchronize()
        for k, (t, r) in enumerate(zip(dev, ref)):
            a = t.cpu().numpy()
            assert np.array_equal(a, r), (replay, k, float(np.max(np.abs(a - r))))
        assert float(scratch) == float(1 << 20)
    s.close()
