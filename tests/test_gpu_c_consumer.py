"""The library driven from a plain C program (tests/c_consumer.c: the C ABI, the HIP
runtime for device memory, the default stream, no Python or torch in the process)
gives the same results, bit for bit, as the same problem stepped through the Python
binding on a stream of its own (where the steps are graph replays)."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

from paper_2511_10257_amd import lbfs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BIN = os.path.join(ROOT, "tests", "c_consumer.bin")


@pytest.mark.parametrize("nx, ny, precision, steps", [(64, 64, "fp32", 20), (48, 40, "fp64", 10)])
def test_c_program_matches_the_binding(tmp_path, nx, ny, precision, steps):
    assert os.path.exists(BIN), "tests/c_consumer.bin is built by __graft_entry__.build()"
    prec = lbfs.LBFS_FP64 if precision == "fp64" else lbfs.LBFS_FP32
    out = tmp_path / "c_consumer.out"
    print(f"c_consumer {nx}x{ny} {precision} {steps} steps", flush=True)
    r = subprocess.run([BIN, str(nx), str(ny), str(prec), str(steps), str(out)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    got = np.fromfile(out, dtype=np.float64)
    n = nx * ny
    assert got.size == 7 + 2 * n

    p = lbfs.Params()
    assert lbfs.lib().lbfs_params_default(C.byref(p), nx, ny, prec) == lbfs.LBFS_OK
    s = lbfs.Solver(p)
    s.step(steps)
    o = s.observe()
    head = [float(o["step"]), o["t"], o["liquid_fraction"], o["solid_ratio"], o["volume"], o["height"], o["umax"]]
    assert head[0] == steps
    assert np.array_equal(got[:7], np.array(head)), (got[:7], head)
    assert np.array_equal(got[7:7 + n].reshape(ny, nx), s.get("C"))
    assert np.array_equal(got[7 + n:].reshape(ny, nx), s.get("He"))
    s.close()
