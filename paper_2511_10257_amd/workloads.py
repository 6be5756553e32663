"""Seeded synthetic workloads shaped like the paper's freezing-droplet study.

This module only describes inputs: grid sizes, droplet geometry, the dimensionless
groups (Ste, Bo_m, field angle) and the property table in lattice units. It holds none
of the solver's arithmetic and is shared by the HIP product binding, the CPU oracle
wrapper, the tests and the benchmark.

The paper (Sec. 5, Fig. 8) studies a half droplet sitting on a cold bottom wall with a
90 degree contact angle, in a vertical or horizontal uniform field; the wall
temperature sets the Stefan number and the field the magnetic Bond number (Eq. 50).
Property ratios follow the ferrofluid table of Sec. 5 (solid/liquid density
1450/1580, heat capacity 1670/3000, conductivity 2.32/0.72); the remaining lattice
values (viscosities, gas conductivity, interface width, mobility, time step) are
choices stable for the explicit scheme, listed in the design notes. There is no
dataset or checkpoint: every field is generated here.
"""
from __future__ import annotations

import copy

import numpy as np

# property table [solid, liquid, gas] in lattice units (dx = 1)
RHO_S = 1450.0 / 1580.0
CP_S = 1670.0 / 3000.0
LAM_L = 0.05
LAM_S = LAM_L * 2.32 / 0.72
GAS_DIFFUSIVITY = 0.4


def _props(rho_ratio: float = 10.0, visc_ratio: float = 10.0, gas_lambda_ratio: float | None = None) -> dict:
    """Gas conductivity: by default that of a gas of diffusivity GAS_DIFFUSIVITY and
    heat capacity 1 (lambda_g / lambda_l = 0.8); with gas_lambda_ratio the conductivity
    is that fraction of the liquid's (air against a water-based ferrofluid: about
    0.036) at the same diffusivity, through a lower gas heat capacity."""
    rho_g = 1.0 / rho_ratio
    mu_l = 0.02
    if gas_lambda_ratio is None:
        lam_g, cp_g = GAS_DIFFUSIVITY * rho_g * 1.0, 1.0
    else:
        lam_g = gas_lambda_ratio * LAM_L
        cp_g = lam_g / (rho_g * GAS_DIFFUSIVITY)
    return dict(
        rho=[RHO_S, 1.0, rho_g],
        mu=[mu_l, mu_l, mu_l / visc_ratio],
        cp=[CP_S, 1.0, cp_g],
        lam=[LAM_S, LAM_L, lam_g],
        chi=[1.0, 1.0, 0.0],
    )


def droplet_problem(n: int, radius: float, ste: float, bo_m: float, angle_deg: float,
                    rho_ratio: float = 10.0, visc_ratio: float = 10.0,
                    precision: str = "fp32", ny: int | None = None,
                    gas_lambda_ratio: float | None = None) -> dict:
    """Half droplet on the cold south wall of an n x ny box (Sec. 5, Fig. 8)."""
    ny = n if ny is None else ny
    prob = dict(
        nx=n, ny=ny, dx=1.0, dt=0.5, dt_stream=0.5,
        t_melt=0.0, t_init=0.0, t_wall=-1.0, ste=ste, bo_m=bo_m, angle_deg=angle_deg,
        mu0=1.0, grav=[0.0, 0.0], sigma=0.005, xi=4.0, mobility=0.05, tau_g=1.0,
        drop=[n / 2.0, 0.0, float(radius)], init_kind="droplet", c_init=1.0,
        periodic=[0, 0],
        thermal_bc=["adiabatic", "adiabatic", "fixed", "adiabatic"],
        thermal_val=[0.0, 0.0, -1.0, 0.0],
        mag_bc=["fixed", "fixed", "fixed", "fixed"],
        sweeps=4, omega=1.0, init_omega=0.0,
        init_tol=1e-9 if precision == "fp64" else 1e-4, init_max=20 * max(n, ny) + 1000,
        init_check=50,
        precision=precision,
    )
    prob.update(_props(rho_ratio, visc_ratio, gas_lambda_ratio))
    return prob


def droplet64() -> dict:
    """64^2 FP64 case: R=16, vertical field, Bo_m=0.5, Ste=0.1, 2000 steps."""
    p = droplet_problem(64, 16, ste=0.1, bo_m=0.5, angle_deg=90.0, precision="fp64")
    p["steps"] = 2000
    p["name"] = "droplet-64x64-R16-vertical-Bo0.5-Ste0.1-fp64"
    return p


def droplet256(seed: int = 0) -> dict:
    """256^2 FP32 case: R=64, angle 0 or 90 and Bo_m ~ U[0,2] drawn with the seed."""
    rng = np.random.default_rng(seed)
    angle = (0.0, 90.0)[int(rng.integers(0, 2))]
    bo = float(rng.uniform(0.0, 2.0))
    p = droplet_problem(256, 64, ste=0.1, bo_m=bo, angle_deg=angle, precision="fp32")
    p["steps"] = 20000
    p["name"] = f"droplet-256x256-R64-angle{angle:g}-Bo{bo:.4f}-Ste0.1-fp32"
    return p


def droplet1024(precision: str = "fp32") -> dict:
    """1024^2 case: R=256, horizontal field, Bo_m=1.5, density ratio 100, K=4."""
    p = droplet_problem(1024, 256, ste=0.1, bo_m=1.5, angle_deg=0.0, rho_ratio=100.0,
                        precision=precision)
    p["steps"] = 1000
    p["name"] = f"droplet-1024x1024-R256-horizontal-Bo1.5-rho100-{precision}"
    return p


def droplet4096(precision: str = "fp32") -> dict:
    """4096^2 case with the physics of the 1024^2 one (R=1024): its 1.2 GB of FP32 state
    exceeds the 256 MB last-level cache, so every step streams from HBM."""
    p = droplet_problem(4096, 1024, ste=0.1, bo_m=1.5, angle_deg=0.0, rho_ratio=100.0,
                        precision=precision)
    p["steps"] = 100
    p["name"] = f"droplet-4096x4096-R1024-horizontal-Bo1.5-rho100-{precision}"
    return p


def deformation_problem(n: int, bo_m: float, precision: str = "fp32", radius: float | None = None) -> dict:
    """Suspended ferrofluid droplet in a carrier liquid, no freezing (Sec. 4.3, Table 2):
    an n x n box, droplet of radius n/5 at the centre, relative permeability 2.2 inside
    (chi = 1.2) and 1 outside, density ratio 1580/800 and viscosity ratio 0.016/0.0008
    of Table 2. The field is vertical, imposed through the potential on the top and
    bottom walls, with magnetically insulating side walls; every wall is no-slip and
    adiabatic and the whole box stays liquid (T above the melting point), so only the
    magnetic, capillary and viscous forces act. H0 follows Bo_m = mu0 H0^2 D / sigma
    (Eq. 50) with D the droplet diameter."""
    R = n / 5.0 if radius is None else float(radius)
    sigma, mu0 = 0.005, 1.0
    mu_l = 0.02
    prob = dict(
        nx=n, ny=n, dx=1.0, dt=0.5, dt_stream=0.5,
        t_melt=0.0, t_init=1.0, latent=1.0, h0=float(np.sqrt(bo_m * sigma / (mu0 * 2.0 * R))),
        ste=None, bo_m=float(bo_m), angle_deg=90.0,
        mu0=mu0, grav=[0.0, 0.0], sigma=sigma, xi=4.0, mobility=0.05, tau_g=1.0,
        drop=[n / 2.0, n / 2.0, R], init_kind="droplet", c_init=1.0,
        periodic=[0, 0],
        thermal_bc=["adiabatic"] * 4, thermal_val=[0.0] * 4,
        mag_bc=["insulating", "insulating", "fixed", "fixed"],
        sweeps=4, omega=1.0, init_omega=0.0,
        init_tol=1e-9 if precision == "fp64" else 1e-4, init_max=20 * n + 1000, init_check=50,
        precision=precision,
        rho=[RHO_S, 1.0, 800.0 / 1580.0],
        mu=[mu_l, mu_l, mu_l * 0.0008 / 0.016],
        cp=[CP_S, 1.0, 1.0],
        lam=[LAM_S, LAM_L, LAM_L],
        chi=[1.2, 1.2, 0.0],
        name=f"deformation-{n}x{n}-R{R:g}-Bo{bo_m:g}-{precision}",
    )
    return prob


def sessile_radius(R0: float, theta_deg: float) -> float:
    """Radius of the circular cap of contact angle theta whose area equals the half disc
    of radius R0 (the 90 degree droplet): R^2 (theta - sin theta cos theta) = pi R0^2 / 2."""
    th = np.deg2rad(theta_deg)
    return float(R0 * np.sqrt((np.pi / 2.0) / (th - np.sin(th) * np.cos(th))))


def static_droplet_problem(theta_deg: float, nx: int = 400, ny: int = 200, R0: float | None = None,
                           precision: str = "fp32") -> dict:
    """Water droplet freezing on a cold wall at contact angle theta (Sec. 4.2): Ste 0.19,
    Bond number g R0 (rho_l - rho_g) / sigma = 0.22 with gravity towards the wall,
    solid / liquid / gas densities 0.9 / 1 / 0.05, no magnetic field, a 400 x 200 box;
    the droplet starts at the melting point as the circular cap of that contact angle
    with the area of a half disc of radius R0 (nx / 8 by default). The Prandtl number of
    the paper (13.47) is not matched (explicit stability), as for the other workloads."""
    R0 = nx / 8.0 if R0 is None else float(R0)
    R = sessile_radius(R0, theta_deg)
    p = droplet_problem(nx, R0, ste=0.19, bo_m=0.0, angle_deg=90.0, precision=precision, ny=ny)
    rho_g = 0.05
    sigma = p["sigma"]
    g = 0.22 * sigma / (R0 * (1.0 - rho_g))
    p.update(
        rho=[0.9, 1.0, rho_g],
        lam=[LAM_S, LAM_L, GAS_DIFFUSIVITY * rho_g * 1.0],
        chi=[0.0, 0.0, 0.0], h0=0.0,
        grav=[0.0, -g],
        drop=[nx / 2.0, -R * float(np.cos(np.deg2rad(theta_deg))), R],
        contact_angle=[90.0, 90.0, float(theta_deg), 90.0],
        name=f"static-droplet-{nx}x{ny}-R0{R0:g}-theta{theta_deg:g}-Ste0.19-Bo0.22-{precision}",
    )
    p["r0"] = R0
    return p


def batch64(seed: int = 1, count: int = 64) -> list[dict]:
    """Batch of uneven instances: edge in {64..256}, R=edge/4, random angle/Bo_m/Ste."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        edge = int(rng.choice([64, 96, 128, 192, 256]))
        angle = float(rng.uniform(0.0, 90.0))
        bo = float(rng.uniform(0.0, 2.0))
        ste = float(rng.uniform(0.05, 0.2))
        out.append(droplet_problem(edge, edge / 4.0, ste=ste, bo_m=bo, angle_deg=angle,
                                   precision="fp32"))
    return out


def request_stream(seed: int = 2, rate_hz: float = 20.0, horizon_s: float = 300.0,
            edges=(96, 128, 256, 512)) -> list[tuple[float, dict]]:
    """Poisson request stream: (arrival time in s, problem) pairs."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= horizon_s:
            break
        edge = int(rng.choice(list(edges)))
        angle = float(rng.uniform(0.0, 90.0))
        bo = float(rng.uniform(0.0, 2.0))
        ste = float(rng.uniform(0.05, 0.2))
        out.append((t, droplet_problem(edge, edge / 4.0, ste=ste, bo_m=bo, angle_deg=angle,
                                       precision="fp32")))
    return out


def neumann_problem(dx: float, latent: float, length: float = 20.0, ny: int = 4) -> dict:
    """One-dimensional conductive freezing (Sec. 4.1): rho = Cp = 1, alpha = 0.4,
    T_b = -1 at x = 0, T_0 = 1 initially and at the far wall, T_m = 0; y periodic."""
    nx = int(round(length / dx))
    alpha = 0.4
    prob = dict(
        nx=nx, ny=ny, dx=dx, dt=0.25 * dx * dx / alpha, dt_stream=0.5 * dx,
        rho=[1.0, 1.0, 1.0], mu=[0.02, 0.02, 0.02], cp=[1.0, 1.0, 1.0],
        lam=[alpha, alpha, alpha], chi=[0.0, 0.0, 0.0],
        latent=latent, h0=0.0, t_melt=0.0, t_init=1.0, t_wall=-1.0,
        angle_deg=0.0, mu0=1.0, grav=[0.0, 0.0], sigma=0.005, xi=4.0, mobility=0.05,
        tau_g=1.0, drop=[0.0, 0.0, 1.0], init_kind="uniform", c_init=1.0,
        periodic=[0, 1],
        thermal_bc=["fixed", "fixed", "adiabatic", "adiabatic"],
        thermal_val=[-1.0, 1.0, 0.0, 0.0],
        mag_bc=["insulating"] * 4, sweeps=0, omega=1.0, init_omega=0.0,
        init_tol=1e-12, init_max=0, init_check=50, precision="fp64",
    )
    return prob


def with_changes(prob: dict, **kw) -> dict:
    p = copy.deepcopy(prob)
    p.update(kw)
    return p


def smooth_state(nx: int, ny: int, seed: int, latent: float, h0: float,
                 angle_deg: float = 90.0, amp_u: float = 0.02, droplet: bool = True) -> dict:
    """Seeded smooth state (conserved fields, potential, lagged source) that exercises
    every branch of the enthalpy map: a droplet-like order parameter with noise, an
    enthalpy spanning solid, mushy and liquid values, small random pressure and
    momentum, and a perturbed applied-field potential. Returned arrays are (ny, nx)."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64) + 0.5

    def modes(k: int, scale: float) -> np.ndarray:
        f = np.zeros((ny, nx))
        for _ in range(k):
            kx, ky = rng.integers(1, 4, size=2)
            ph1, ph2 = rng.uniform(0, 2 * np.pi, size=2)
            f += rng.normal() * np.sin(2 * np.pi * kx * x / nx + ph1) * np.cos(2 * np.pi * ky * y / ny + ph2)
        return scale * f / max(1.0, np.sqrt(k))

    if droplet:
        r = np.hypot(x - nx / 2.0, y - 0.1 * ny)
        rad = 0.35 * min(nx, ny)
        C = 0.5 * (1.0 + np.tanh(2.0 * (rad - r) / 3.0)) + modes(3, 0.02)
    else:
        C = 0.5 + modes(3, 0.2)
    frac = 0.5 + modes(4, 0.9)            # spans < 0, (0,1) and > 1
    He = latent * np.clip(C, 0.0, 1.0) * frac + modes(2, 0.3)
    p = modes(3, 1e-3)
    Mx = modes(3, amp_u)
    My = modes(3, amp_u)
    th = np.deg2rad(angle_deg)
    phi = -h0 * (x * np.cos(th) + y * np.sin(th)) + modes(3, 0.05 * h0 * max(nx, ny))
    S = modes(2, 1e-3)
    return dict(He=He, p=p, Mx=Mx, My=My, C=C, phi=phi, S=S)
