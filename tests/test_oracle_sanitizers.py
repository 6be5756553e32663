"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code, CPU): a
build of oracle/lbfs_oracle.c with both runs short problems through every path the
parity tests use (walls and periodic axes, wetting walls, a melting range, the
pseudo-time magnetic solve with convergence control, R(W), face fluxes, the wall heat
profile, observables); any invalid access or undefined operation aborts the run."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

SCRIPT = r'''
import sys
sys.path.insert(0, %(root)r)
import numpy as np
from oracle import oracle as orc
from paper_2511_10257_amd import workloads as wl

def run(prob, steps):
    o = orc.Oracle(prob)
    o.step(steps)
    o.observe()
    o.rhs()
    o.face_fluxes()
    o.wall_heat_profile()
    for k in ("He", "p", "Mx", "My", "C", "phi", "S", "T", "Fl"):
        o.get(k)

base = wl.droplet_problem(20, 5.0, ste=0.1, bo_m=1.0, angle_deg=30.0, precision="fp64", ny=14)
run(base, 3)
run(wl.with_changes(base, periodic=[1, 0], angle_deg=90.0), 3)
run(wl.with_changes(base, contact_angle=[90.0, 90.0, 60.0, 120.0]), 3)
run(wl.with_changes(base, t_liquidus=0.3), 3)
run(wl.with_changes(base, mag_method="lbfs", sweeps=3, mag_max_iters=9, mag_tol=1e-30), 2)
run(wl.with_changes(base, mag_bc=["insulating", "insulating", "fixed", "fixed"], angle_deg=90.0, dt=0.0), 2)
run(wl.droplet_problem(5, 1.5, ste=0.2, bo_m=0.5, angle_deg=0.0, precision="fp64", ny=4), 2)
print("ok")
'''


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no gcc")
    libasan = subprocess.run([cc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("no libasan")
    so = str(tmp_path / "liblbfs_oracle_sanitized.so")
    subprocess.check_call([cc, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-std=c11", "-fPIC", "-shared", "-o", so,
                           os.path.join(ROOT, "oracle", "lbfs_oracle.c"), "-lm"])
    env = dict(os.environ, LD_PRELOAD=libasan, ASAN_OPTIONS="detect_leaks=0", LBFS_ORACLE_LIB=so)
    r = subprocess.run([sys.executable, "-c", SCRIPT % {"root": ROOT}], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr[-4000:]
