"""Pins of the oracle's magnetic LBFS pseudo-time solve (Sec. 3.1, Eqs. 12-18).

The oracle builds every face flux literally: the potential at the nine points
x_f - e_a delta_t by Eq. 44, the face potential by the compatibility sum of Eq. 45,
the equilibria of Eq. 13, m* of Eq. 16 and the moment of Eq. 18, then advances Eq. 17
in pseudo-time by SSP-RK3. These tests pin it against what the mathematics fixes:
the flux the construction reduces to (worked out by hand from Eqs. 13, 16 and 44),
the amplification of a Fourier mode by one RK3 step, a one-dimensional layered medium
whose discrete solution is a series of face resistances, and the fixed point of the
red-black sweeps.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2511_10257_amd import workloads as wl

CS2 = 1.0 / 3.0


def liquid_box(nx, ny, mag_bc, angle=0.0, periodic=(0, 0), dts=0.5):
    """chi = [1, 1, 0]: a liquid cell (Fl = 1) has mu = mu0 (1 + clamp(C))."""
    p = wl.droplet_problem(nx, nx / 8.0, ste=0.1, bo_m=0.5, angle_deg=angle, precision="fp64", ny=ny)
    p.update(init_max=0, h0=1.0, latent=10.0, mag_bc=list(mag_bc), thermal_bc=["adiabatic"] * 4,
             periodic=list(periodic), dt_stream=dts)
    return p


def set_liquid(o, C):
    o.set("C", C)
    o.set("He", 20.0 + np.zeros_like(C))      # above C L = 10 for every C <= 1: Fl = 1


def central_gradients(ph):
    gx = (ph[:, 2:] - ph[:, :-2]) / 2.0
    gy = (ph[2:, :] - ph[:-2, :]) / 2.0
    return gx, gy


@pytest.mark.parametrize("dts", [0.5, 0.3])
def test_literal_flux_is_the_two_point_flux_plus_gradient_term(dts):
    """At an interior x-face the nine m* moments sum to
    ((tau_m - 1/2) / 6) [(phi_L - phi_R) + (dx/2 - delta_t)(g_L + g_R)], tau_m - 1/2 =
    mu_f D / (cs^2 delta_t): the axis and diagonal points of each side carry the cell
    value plus the normal offset (dx/2 - delta_t) times its gradient, the tangential
    offsets of the two diagonals cancel, and the face terms sum to zero against e_a.
    At delta_t = dx/2 this is -D mu_f (phi_R - phi_L) / dx."""
    nx, ny, D = 14, 11, 1.7
    o = orc.Oracle(liquid_box(nx, ny, ["fixed"] * 4, angle=20.0, dts=dts))
    rng = np.random.default_rng(3)
    C = rng.uniform(-0.1, 1.1, (ny, nx))
    set_liquid(o, C)
    phi = rng.standard_normal((ny, nx))
    o.set("phi", phi)
    fx, fy = o.mag_lbfs_fluxes(D)
    mu = 1.0 + np.clip(C, 0.0, 1.0)
    gx, gy = central_gradients(phi)
    a = 0.5 - dts
    # x-faces between interior cells whose gradients are interior: i-1 >= 1, i <= nx-2
    k = (0.5 * (mu[:, 1:] + mu[:, :-1])) * D / (CS2 * dts) / 6.0
    want = k[:, 1:-1] * ((phi[:, 1:-2] - phi[:, 2:-1]) + a * (gx[:, :-1] + gx[:, 1:]))
    got = fx[:, 2:-2]
    assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))
    k = (0.5 * (mu[1:, :] + mu[:-1, :])) * D / (CS2 * dts) / 6.0
    want = k[1:-1, :] * ((phi[1:-2, :] - phi[2:-1, :]) + a * (gy[:-1, :] + gy[1:, :]))
    got = fy[2:-2, :]
    assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))
    if dts == 0.5:
        # every interior face, the compact form
        want = -D * 0.5 * (mu[:, 1:] + mu[:, :-1]) * (phi[:, 1:] - phi[:, :-1])
        assert np.max(np.abs(fx[:, 1:-1] - want)) < 1e-13 * np.max(np.abs(want))


def test_wall_fluxes_at_half_step():
    """Towards a fixed-potential wall the potential difference acts over half a cell:
    -2 D mu_c (phi_wall - phi_c) / dx (outward); an insulating wall carries no flux;
    a periodic axis closes through the opposite side."""
    nx, ny, D = 12, 10, 0.8
    o = orc.Oracle(liquid_box(nx, ny, ["fixed", "insulating", "insulating", "fixed"], angle=35.0))
    rng = np.random.default_rng(4)
    C = rng.uniform(0.0, 1.0, (ny, nx))
    set_liquid(o, C)
    phi = rng.standard_normal((ny, nx))
    o.set("phi", phi)
    fx, fy = o.mag_lbfs_fluxes(D)
    mu = 1.0 + C
    th = math.radians(35.0)
    y = np.arange(ny) + 0.5
    x = np.arange(nx) + 0.5
    phi_w_west = -(0.0 * math.cos(th) + y * math.sin(th))
    phi_w_north = -(x * math.cos(th) + ny * math.sin(th))
    # west wall (x-face 0): flux in +x from the wall into cell 0
    want = -2.0 * D * mu[:, 0] * (phi[:, 0] - phi_w_west)
    assert np.max(np.abs(fx[:, 0] - want)) < 1e-13 * np.max(np.abs(want))
    want = -2.0 * D * mu[-1, :] * (phi_w_north - phi[-1, :])
    assert np.max(np.abs(fy[-1, :] - want)) < 1e-13 * np.max(np.abs(want))
    assert np.max(np.abs(fx[:, -1])) < 1e-13 and np.max(np.abs(fy[0, :])) < 1e-13

    o = orc.Oracle(liquid_box(nx, ny, ["insulating"] * 4, periodic=(1, 0)))
    set_liquid(o, C)
    o.set("phi", phi)
    fx, _ = o.mag_lbfs_fluxes(D)
    want = -D * 0.5 * (mu[:, 0] + mu[:, -1]) * (phi[:, 0] - phi[:, -1])
    assert np.max(np.abs(fx[:, 0] - want)) < 1e-13 * np.max(np.abs(want))
    assert np.array_equal(fx[:, 0], fx[:, -1])


def test_rk3_amplification_of_a_potential_mode():
    """Uniform permeability on a periodic box: a Fourier mode of the potential is an
    eigenvector of the discrete Eq. 17, so one SSP-RK3 pseudo-step multiplies it by
    1 + z + z^2/2 + z^3/6, z = -dtau D mu (2 - 2 cos k dx) / dx^2."""
    n, D, dtau = 32, 1.3, 0.11
    o = orc.Oracle(liquid_box(n, 8, ["insulating"] * 4, periodic=(1, 1)))
    set_liquid(o, np.ones((8, n)))
    x = np.arange(n) + 0.5
    m = 5
    eps = 0.4
    o.set("phi", np.tile(1.5 + eps * np.cos(2 * np.pi * m * x / n), (8, 1)))
    o.mag_lbfs(1, D, dtau)
    k = 2 * np.pi * m / n
    z = -dtau * D * 2.0 * (2.0 - 2.0 * math.cos(k))
    G = 1 + z + z * z / 2 + z ** 3 / 6
    expect = 1.5 + eps * G * np.cos(2 * np.pi * m * x / n)
    got = o.get("phi")
    assert np.max(np.abs(got - expect)) < 1e-13


def test_automatic_pseudo_step_is_stable_for_the_stiffest_mode():
    """The automatic step dx^2 / (4 D mu_max) puts the checkerboard mode (the largest
    eigenvalue, 8 D mu / dx^2) at z = -2, where 1 + z + z^2/2 + z^3/6 = -1/3."""
    n, D = 16, 2.5
    o = orc.Oracle(liquid_box(n, n, ["insulating"] * 4, periodic=(1, 1)))
    set_liquid(o, np.ones((n, n)))
    dtau = o.mag_lbfs_dtau(D)
    assert abs(dtau - 1.0 / (4 * D * 2.0)) < 1e-15
    ii, jj = np.meshgrid(np.arange(n), np.arange(n))
    chk = np.where((ii + jj) % 2 == 0, 1.0, -1.0)
    o.set("phi", chk)
    o.mag_lbfs(1, D, 0.0)
    assert np.max(np.abs(o.get("phi") + chk / 3.0)) < 1e-14


def layered_closed_form(mu, phi_w, phi_e, D=1.0):
    """Discrete Eq. 4 in a medium layered across x between two fixed-potential walls:
    the face flux F is the same through every face, so the potential falls by F times
    a resistance per face (1 / (2 mu_0 D) and 1 / (2 mu_{n-1} D) for the two
    half-cell wall faces, 1 / (mu_f D) inside)."""
    r = np.concatenate([[1 / (2 * mu[0])], 1 / (0.5 * (mu[1:] + mu[:-1])), [1 / (2 * mu[-1])]]) / D
    F = (phi_w - phi_e) / r.sum()
    drops = F * r
    return phi_w - np.cumsum(drops)[:-1]


def test_pseudo_time_reaches_the_layered_closed_form():
    nx, ny = 16, 4
    p = liquid_box(nx, ny, ["fixed", "fixed", "insulating", "insulating"], angle=0.0)
    o = orc.Oracle(p)
    x = np.arange(nx) + 0.5
    Cx = 0.5 + 0.45 * np.sin(2 * np.pi * x / nx) + 0.05 * np.cos(5 * x)
    set_liquid(o, np.tile(Cx, (ny, 1)))
    o.set("phi", np.zeros((ny, nx)))
    mu = 1.0 + np.clip(Cx, 0, 1)
    want = layered_closed_form(mu, 0.0, -float(nx))       # phi_applied = -H0 x, H0 = 1
    r0 = o.mag_residual()
    for _ in range(40):
        r = o.mag_lbfs(500, 0.9)
        if r < 1e-13 * r0:
            break
    assert r < 1e-13 * r0
    got = o.get("phi")
    assert np.max(np.abs(got - want[None, :])) < 1e-10 * nx
    # the red-black sweeps (method 0) reach the same fixed point
    o2 = orc.Oracle(p)
    set_liquid(o2, np.tile(Cx, (ny, 1)))
    o2.set("phi", np.zeros((ny, nx)))
    for _ in range(40):
        if o2.mag_sweeps(200, 1.7) < 1e-13 * r0:
            break
    assert np.max(np.abs(o2.get("phi") - want[None, :])) < 1e-10 * nx


def test_pseudo_time_and_sweeps_share_the_fixed_point_on_a_droplet():
    """Two-dimensional droplet, tilted field, fixed walls: Eq. 17 advanced in pseudo-time
    and the red-black sweeps converge to the same potential."""
    p = wl.droplet_problem(18, 5.0, ste=0.1, bo_m=1.2, angle_deg=30.0, precision="fp64", ny=14)
    p.update(init_max=0)
    a, b = orc.Oracle(p), orc.Oracle(p)
    r0 = a.mag_residual()
    res = []
    for _ in range(60):
        res.append(a.mag_lbfs(200, 1.0))
        if res[-1] < 1e-12 * r0:
            break
    assert res[-1] < 1e-12 * r0
    assert all(y <= x * (1 + 1e-12) for x, y in zip(res, res[1:]))     # never increases
    for _ in range(40):
        if b.mag_sweeps(100, 1.6) < 1e-13 * r0:
            break
    pa, pb = a.get("phi"), b.get("phi")
    assert np.max(np.abs(pa - pb)) < 1e-9 * np.max(np.abs(pb))


def test_step_with_the_pseudo_time_method():
    """A time step with mag_method = lbfs runs the pseudo-time solve in place of the
    sweeps; with both iterated to convergence the steps agree."""
    base = wl.droplet_problem(16, 5.0, ste=0.1, bo_m=1.5, angle_deg=90.0, precision="fp64")
    base.update(init_tol=1e-13)
    a = orc.Oracle(wl.with_changes(base, sweeps=60, omega=1.6))
    b = orc.Oracle(wl.with_changes(base, sweeps=1500, mag_method="lbfs", mag_lbfs_d=1.0))
    a.step(3)
    b.step(3)
    for name in ("phi", "He", "Mx", "My", "C"):
        x, y = a.get(name), b.get(name)
        assert np.max(np.abs(x - y)) <= 1e-8 * max(1.0, np.max(np.abs(x))), name
    assert b.observe()["mag_residual"] < 1e-8


def test_invalid_pseudo_time_parameters_are_rejected():
    p = wl.droplet_problem(16, 4.0, ste=0.1, bo_m=1.0, angle_deg=0.0, precision="fp64")
    with pytest.raises(ValueError):
        orc.Oracle(wl.with_changes(p, mag_method="lbfs", mag_lbfs_d=0.0))


@pytest.mark.parametrize("method", ["sweeps", "lbfs"])
def test_convergence_controlled_step_is_a_whole_number_of_chunks(method):
    """With a residual target the magnetic phase repeats chunks of `sweeps` iterations
    until ||r||_2 <= mag_tol or mag_max_iters: with an unreachable target it is the
    fixed count mag_max_iters, and otherwise the fixed count of the chunks it used."""
    base = wl.droplet_problem(20, 5.0, ste=0.1, bo_m=1.5, angle_deg=90.0, precision="fp64")
    base.update(mag_method=method, init_tol=1e-6)
    a = orc.Oracle(wl.with_changes(base, sweeps=4, mag_max_iters=12, mag_tol=0.0))
    b = orc.Oracle(wl.with_changes(base, sweeps=12))
    a.step(2)
    b.step(2)
    for name in ("phi", "He", "Mx", "C"):
        assert np.array_equal(a.get(name), b.get(name)), name
    # a reachable target: count the chunks on a copy of the state, then compare with the
    # fixed count
    probe = orc.Oracle(base)
    probe.step(1)
    state = {k: probe.get(k) for k in ("He", "p", "Mx", "My", "C", "phi", "S")}
    state["phi"] = state["phi"] * 1.01          # away from the fixed point
    counter = orc.Oracle(base, init=False)
    counter.set_state(state)
    tol = 0.02 * counter.mag_sweeps(0, 1.0)
    chunks = 0
    while True:
        r = counter.mag_sweeps(2, 1.0) if method == "sweeps" else counter.mag_lbfs(2, 1.0, 0.0)
        chunks += 1
        if r <= tol or chunks >= 500:
            break
    assert 1 < chunks < 500
    c = orc.Oracle(wl.with_changes(base, sweeps=2, mag_max_iters=1000, mag_tol=tol), init=False)
    d = orc.Oracle(wl.with_changes(base, sweeps=2 * chunks), init=False)
    for o in (c, d):
        o.set_state(state)
        o.step(1)
    assert c.observe()["mag_residual"] <= tol
    for name in ("phi", "He", "Mx", "C"):
        assert np.array_equal(c.get(name), d.get(name)), name
