"""Host-side checks of the C ABI library (no GPU needed): it loads, exports every
function include/lbfs.h declares, validates parameters and converts Eq. 50 groups."""
import ctypes as C
import math
import os
import re

import pytest

from paper_2511_10257_amd import lbfs, workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lbfs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbfs_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = lbfs.lib()
    names = declared_functions()
    assert len(names) >= 16
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(lbfs.EXPORTS)


def test_state_bytes_and_validation():
    p = lbfs.make_params(wl.droplet256())
    nb = lbfs.state_bytes(p)
    # 18 fields of 256 x 256 float plus metadata
    assert 18 * 256 * 256 * 4 <= nb < 18 * 256 * 256 * 4 + 4 * 1024 * 1024
    p64 = lbfs.make_params(wl.droplet64())
    assert lbfs.state_bytes(p64) >= 18 * 64 * 64 * 8
    for field, bad in (("nx", 3), ("dx", 0.0), ("tau_g", 0.5), ("precision", 7), ("dt", 100.0), ("dt", -1.0),
                       ("t_liquidus", -0.5),
                       ("sor_omega", 2.0), ("dt_stream", 0.3), ("abi_version", 99)):
        q = lbfs.make_params(wl.droplet64())
        setattr(q, field, bad)
        assert lbfs.lib().lbfs_state_bytes(C.byref(q)) == 0, field
    # edges up to 2^20 and at most 2^30 cells (32-bit kernel indices)
    for nx, ny, ok in ((1 << 20, 1024, True), (1 << 20, 1025, False), ((1 << 20) + 1, 8, False),
                       (32768, 32768, True), (32768, 32770, False)):
        q = lbfs.make_params(wl.droplet64())
        q.nx, q.ny = nx, ny
        assert (lbfs.lib().lbfs_state_bytes(C.byref(q)) > 0) == ok, (nx, ny)
    q = lbfs.make_params(wl.neumann_problem(0.1, 250.0))
    assert lbfs.lib().lbfs_state_bytes(C.byref(q)) > 0
    q.ny = 5                     # odd periodic axis: no red-black colouring
    assert lbfs.lib().lbfs_state_bytes(C.byref(q)) == 0
    q = lbfs.make_params(wl.droplet64())
    q.periodic[1] = 1            # vertical applied field across a periodic axis
    assert lbfs.lib().lbfs_state_bytes(C.byref(q)) == 0
    out = C.c_void_p()
    assert lbfs.lib().lbfs_init(C.byref(q), None, 0, None, C.byref(out)) == lbfs.LBFS_E_INVAL
    q = lbfs.make_params(wl.droplet64())
    q.abi_version = lbfs.LBFS_ABI_VERSION - 1
    assert lbfs.lib().lbfs_init(C.byref(q), None, 0, None, C.byref(out)) == lbfs.LBFS_E_ABI
    # the magnetic method and its pseudo-time parameters
    for kw in (dict(mag_method=3), dict(mag_method=1, mag_lbfs_d=0.0), dict(mag_method=1, mag_lbfs_dtau=-1.0),
               dict(mag_method=1, mag_lbfs_d=float("nan")), dict(mag_lbfs_d=-1.0)):
        q = lbfs.make_params(wl.droplet64())
        for k, v in kw.items():
            setattr(q, k, v)
        assert lbfs.lib().lbfs_state_bytes(C.byref(q)) == 0, kw
    q = lbfs.make_params(wl.with_changes(wl.droplet64(), mag_method="lbfs", mag_lbfs_d=2.0, mag_lbfs_dtau=0.05))
    assert (q.mag_method, q.mag_lbfs_d, q.mag_lbfs_dtau) == (1, 2.0, 0.05)
    assert lbfs.lib().lbfs_state_bytes(C.byref(q)) > 0
    # multigrid needs walls on every side and a fixed cycle count
    for kw in (dict(periodic=[1, 0], field_angle_deg=90.0), dict(mag_max_iters=10, mag_tol=1e-3)):
        q = lbfs.make_params(wl.with_changes(wl.droplet64(), mag_method="multigrid"))
        for k, v in kw.items():
            if k == "periodic":
                q.periodic[0], q.periodic[1] = v
            else:
                setattr(q, k, v)
        assert lbfs.lib().lbfs_state_bytes(C.byref(q)) == 0, kw
    q = lbfs.Params()
    assert lbfs.lib().lbfs_params_default(C.byref(q), 64, 64, 0) == 0
    assert (q.mag_method, q.mag_lbfs_d, q.mag_lbfs_dtau) == (0, 1.0, 0.0)
    assert lbfs.lib().lbfs_step(None, 1) == lbfs.LBFS_E_STATE
    assert lbfs.strerror(lbfs.LBFS_E_NOMEM).startswith("buffer")


def test_dimensionless_conversion_matches_eq50():
    prob = wl.droplet64()
    p = lbfs.make_params(prob)
    # Ste = Cp_l (Tm - Tw) / L  and  Bo_m = mu0 H0^2 D / sigma with D = 2R
    assert math.isclose(prob["ste"], p.cp[1] * (p.t_melt - prob["t_wall"]) / p.latent, rel_tol=1e-15)
    assert math.isclose(prob["bo_m"], p.mu0 * p.h0 ** 2 * 2 * p.drop_radius / p.sigma, rel_tol=1e-14)
    assert math.isclose(p.h0, 8.84e-3, rel_tol=1e-3)
    assert p.thermal_bc[2] == 1 and p.thermal_val[2] == -1.0


def test_oracle_and_product_read_the_same_problem():
    from oracle import oracle as orc
    for prob in (wl.droplet64(), wl.droplet256(), wl.droplet1024("fp64"), wl.neumann_problem(0.1, 250.0)):
        a, b = orc.make_params(prob), lbfs.make_params(prob)
        assert (a.nx, a.ny) == (b.nx, b.ny)
        for name in ("dx", "dt", "latent", "h0", "t_melt", "t_init", "sigma", "xi", "mobility", "tau_g",
                     "drop_cx", "drop_cy", "drop_r"):
            other = "drop_radius" if name == "drop_r" else name
            assert getattr(a, name) == pytest.approx(getattr(b, other), rel=1e-15, abs=0), name
        assert a.angle_deg == b.field_angle_deg
        for k in range(3):
            assert a.rho[k] == b.rho[k] and a.mu[k] == b.mu[k] and a.cp[k] == b.cp[k]
            assert a.lam[k] == b.lambda_[k] and a.chi[k] == b.chi[k]
        assert list(a.tbc) == list(b.thermal_bc) and list(a.mbc) == list(b.mag_bc)
        assert list(a.tval) == list(b.thermal_val) and list(a.periodic) == list(b.periodic)
        assert a.sweeps == b.sweeps and a.omega == b.sor_omega


def test_batch_host_checks():
    """Host-side checks of the batch calls (no device work is reached)."""
    p = lbfs.make_params(wl.droplet256())
    nb = lbfs.lib().lbfs_batch_instance_bytes(C.byref(p))
    # the same segments as a solver (tile lists sized for every candidate shape)
    assert lbfs.state_bytes(p) <= nb < lbfs.state_bytes(p) + 64 * 1024
    q = lbfs.make_params(wl.droplet64())
    q.nx = 2
    assert lbfs.lib().lbfs_batch_instance_bytes(C.byref(q)) == 0
    out = C.c_void_p()
    L = lbfs.lib()
    assert L.lbfs_batch_create(0, 0, 4, 1.0, C.c_void_p(1), 1 << 20, None, C.byref(out)) == lbfs.LBFS_E_INVAL
    assert L.lbfs_batch_create(4, 3, 4, 1.0, C.c_void_p(1), 1 << 20, None, C.byref(out)) == lbfs.LBFS_E_INVAL
    assert L.lbfs_batch_create(4, 0, 4, 2.5, C.c_void_p(1), 1 << 20, None, C.byref(out)) == lbfs.LBFS_E_INVAL
    assert L.lbfs_batch_create(4, 0, 4, 1.0, None, 1 << 20, None, C.byref(out)) == lbfs.LBFS_E_INVAL
    slot = C.c_int32()
    assert L.lbfs_batch_admit(None, C.byref(p), C.byref(slot)) == lbfs.LBFS_E_STATE
    assert L.lbfs_batch_step(None, 1) == lbfs.LBFS_E_STATE
    assert L.lbfs_batch_retire(None, 0) == lbfs.LBFS_E_STATE
    L.lbfs_batch_destroy(None)


def test_tile_shape_tables():
    L = lbfs.lib()
    for prec in ("fp32", "fp64"):
        for kind in ("stage", "mag"):
            shapes = lbfs.tile_shapes(kind, prec)
            assert 1 <= len(shapes) <= lbfs.MAX_SHAPES
            for tx, ty, nt, flags in shapes:
                assert nt % 64 == 0 and nt <= 1024 and tx * ty <= (nt if kind == "stage" else 4096)
    assert L.lbfs_tile_shape(2, 0, 0, None, None, None, None) == lbfs.LBFS_E_INVAL
    assert L.lbfs_tile_shape(0, 5, 0, None, None, None, None) == lbfs.LBFS_E_INVAL
    assert L.lbfs_tile_shape(0, 0, 99, None, None, None, None) == lbfs.LBFS_E_INVAL
    assert L.lbfs_set_tile_shapes(None, 0, 0) == lbfs.LBFS_E_STATE
    assert L.lbfs_autotune(None, 5, None, None) == lbfs.LBFS_E_STATE


@pytest.mark.parametrize("compiler, std", [("gcc", "-std=c11"), ("g++", "-std=c++17")])
def test_header_is_plain_iso_c_and_cpp(tmp_path, compiler, std):
    """include/lbfs.h compiles alone as ISO C11 and as C++17 with every warning an error."""
    src = tmp_path / ("h.c" if compiler == "gcc" else "h.cpp")
    src.write_text('#include "lbfs.h"\nint lbfs_header_check(void) { return LBFS_OK + (int)LBFS_ABI_VERSION; }\n')
    import subprocess
    r = subprocess.run([compiler, std, "-Wall", "-Wextra", "-Werror", "-pedantic", "-fsyntax-only",
                        "-I", os.path.join(ROOT, "include"), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_c_consumer_builds_against_the_library(tmp_path):
    """The plain-C test program (the ABI driven from C, no Python) compiles and links
    against liblbfs.so and the HIP runtime alone."""
    import subprocess
    import sys
    sys.path.insert(0, ROOT)
    import __graft_entry__ as ge
    out = str(tmp_path / "c_consumer")
    r = subprocess.run(ge.c_consumer_command(out), capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert os.path.getsize(out) > 0
