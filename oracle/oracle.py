"""ctypes wrapper of the FP64 CPU oracle (liblbfs_oracle.so).

TEST INFRASTRUCTURE: imported only by the tests, the smoke check and the CPU-baseline
leg of the benchmark. The HIP product never imports this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liblbfs_oracle.so")

HE, P, MX, MY, CC, PHI, S, T, FL, FMGX, FMGY, MUC = range(12)
FIELDS = dict(He=HE, p=P, Mx=MX, My=MY, C=CC, phi=PHI, S=S, T=T, Fl=FL,
              Fmgx=FMGX, Fmgy=FMGY, muc=MUC)


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int),
        ("dx", C.c_double), ("dt", C.c_double), ("dt_stream", C.c_double),
        ("rho", C.c_double * 3), ("mu", C.c_double * 3), ("cp", C.c_double * 3),
        ("lam", C.c_double * 3), ("chi", C.c_double * 3),
        ("latent", C.c_double), ("t_melt", C.c_double), ("t_init", C.c_double),
        ("mu0", C.c_double), ("h0", C.c_double), ("angle_deg", C.c_double),
        ("grav", C.c_double * 2),
        ("sigma", C.c_double), ("xi", C.c_double), ("mobility", C.c_double), ("tau_g", C.c_double),
        ("drop_cx", C.c_double), ("drop_cy", C.c_double), ("drop_r", C.c_double),
        ("init_kind", C.c_int), ("c_init", C.c_double),
        ("periodic", C.c_int * 2),
        ("tbc", C.c_int * 4), ("tval", C.c_double * 4), ("mbc", C.c_int * 4),
        ("sweeps", C.c_int), ("omega", C.c_double),
        ("init_omega", C.c_double), ("init_tol", C.c_double),
        ("init_max", C.c_int), ("init_check", C.c_int),
        ("mag_method", C.c_int), ("mag_lbfs_d", C.c_double), ("mag_lbfs_dtau", C.c_double),
        ("mag_max_iters", C.c_int), ("mag_tol", C.c_double),
        ("contact_angle", C.c_double * 4), ("t_liquidus", C.c_double),
    ]


class Obs(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "t", "step", "liquid_fraction", "solid_ratio", "volume", "volume0",
        "mag_residual", "umax", "nonfinite", "height", "umax_drop", "wall_heat", "fourier", "peclet",
        "centroid_x", "centroid_y", "semi_axis_x", "semi_axis_y", "semi_axis_major", "semi_axis_minor",
        "major_axis_deg", "solid_height")]


def build(force: bool = False) -> str:
    src = os.path.join(HERE, "lbfs_oracle.c")
    newest = max(os.path.getmtime(src), os.path.getmtime(os.path.join(HERE, "lbfs_oracle.h")))
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < newest:
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared",
                               "-o", LIB, src, "-lm"])
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        # LBFS_ORACLE_LIB: another build of the same source (the sanitizer test's)
        alt = os.environ.get("LBFS_ORACLE_LIB")
        if alt:
            _lib = load(alt)
        else:
            build()               # rebuilds only when the source is newer than the library
            _lib = load(LIB)
    return _lib


def load(path: str):
    """Open a build of the oracle source (the FP64 library, or its operation-counting
    build) and declare the argument types of its API."""
    L = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    L.orc_new.restype = C.c_void_p
    L.orc_new.argtypes = [C.POINTER(Params)]
    L.orc_free.argtypes = [C.c_void_p]
    L.orc_init.argtypes = [C.c_void_p]
    L.orc_init.restype = C.c_int
    L.orc_step.argtypes = [C.c_void_p, C.c_int]
    L.orc_rhs.argtypes = [C.c_void_p, dp]
    L.orc_face_fluxes.argtypes = [C.c_void_p, dp, dp]
    L.orc_face_inputs.argtypes = [C.c_void_p, dp]
    L.orc_get.argtypes = [C.c_void_p, C.c_int, dp]
    L.orc_set.argtypes = [C.c_void_p, C.c_int, dp]
    L.orc_set_time.argtypes = [C.c_void_p, C.c_double, C.c_double]
    L.orc_observe.argtypes = [C.c_void_p, C.POINTER(Obs)]
    L.orc_mag_sweeps.argtypes = [C.c_void_p, C.c_int, C.c_double]
    L.orc_mag_sweeps.restype = C.c_double
    L.orc_mag_residual.argtypes = [C.c_void_p]
    L.orc_mag_residual.restype = C.c_double
    L.orc_mag_lbfs.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double]
    L.orc_mag_lbfs.restype = C.c_double
    L.orc_mag_lbfs_fluxes.argtypes = [C.c_void_p, C.c_double, dp, dp]
    L.orc_mag_lbfs_dtau.argtypes = [C.POINTER(Params), C.c_double]
    L.orc_mag_lbfs_dtau.restype = C.c_double
    L.orc_wall_heat_profile.argtypes = [C.c_void_p, dp]
    L.orc_lattice.argtypes = [dp, dp, dp]
    L.orc_enthalpy_state.argtypes = [C.POINTER(Params), C.c_double, C.c_double, dp, dp]
    L.orc_equilibria.argtypes = [C.POINTER(Params)] + [C.c_double] * 9 + [dp, dp, dp]
    L.orc_params_from_dimless.argtypes = [C.POINTER(Params), C.c_double, C.c_double, C.c_double]
    return L


_TBC = {"adiabatic": 0, "fixed": 1}
_MBC = {"insulating": 0, "fixed": 1}


def make_params(prob: dict) -> Params:
    """Oracle parameter block from a workload description (Eq. 50 conversions here)."""
    p = Params()
    p.nx, p.ny = int(prob["nx"]), int(prob["ny"])
    p.dx = float(prob["dx"])
    p.dt = float(prob["dt"])
    p.dt_stream = float(prob.get("dt_stream", 0.5 * p.dx)) or 0.5 * p.dx
    for name in ("rho", "mu", "cp", "lam", "chi"):
        arr = getattr(p, name)
        for k in range(3):
            arr[k] = float(prob[name][k])
    p.t_melt = float(prob.get("t_melt", 0.0))
    p.t_init = float(prob.get("t_init", 0.0))
    p.mu0 = float(prob.get("mu0", 1.0))
    p.angle_deg = float(prob.get("angle_deg", 0.0))
    p.grav[0], p.grav[1] = [float(g) for g in prob.get("grav", [0.0, 0.0])]
    p.sigma, p.xi = float(prob["sigma"]), float(prob["xi"])
    p.mobility, p.tau_g = float(prob["mobility"]), float(prob["tau_g"])
    p.drop_cx, p.drop_cy, p.drop_r = [float(v) for v in prob["drop"]]
    p.init_kind = 0 if prob.get("init_kind", "droplet") == "droplet" else 1
    p.c_init = float(prob.get("c_init", 1.0))
    p.periodic[0], p.periodic[1] = [int(v) for v in prob.get("periodic", [0, 0])]
    for k in range(4):
        p.tbc[k] = _TBC[prob["thermal_bc"][k]]
        p.tval[k] = float(prob["thermal_val"][k])
        p.mbc[k] = _MBC[prob["mag_bc"][k]]
    p.sweeps = int(prob.get("sweeps", 4))
    p.omega = float(prob.get("omega", 1.0))
    p.init_omega = float(prob.get("init_omega", 0.0))
    p.init_tol = float(prob.get("init_tol", 1e-12))
    p.init_max = int(prob.get("init_max", 200000))
    p.init_check = int(prob.get("init_check", 50))
    p.mag_method = {"sweeps": 0, "lbfs": 1}[prob.get("mag_method", "sweeps")]
    p.mag_lbfs_d = float(prob.get("mag_lbfs_d", 1.0))
    p.mag_lbfs_dtau = float(prob.get("mag_lbfs_dtau", 0.0))
    p.mag_max_iters = int(prob.get("mag_max_iters", 0))
    p.mag_tol = float(prob.get("mag_tol", 0.0))
    for k, a in enumerate(prob.get("contact_angle", [90.0] * 4)):
        p.contact_angle[k] = float(a)
    p.t_liquidus = float(prob.get("t_liquidus", p.t_melt))
    if "latent" in prob and "h0" in prob:
        p.latent, p.h0 = float(prob["latent"]), float(prob["h0"])
    else:
        # Eq. 50: Ste = Cp_l (Tm - Tw) / L and Bo_m = mu0 H0^2 D / sigma, D = 2 R
        lib().orc_params_from_dimless(C.byref(p), float(prob["ste"]), float(prob["t_wall"]),
                                      float(prob["bo_m"]))
        if "latent" in prob:
            p.latent = float(prob["latent"])
        if "h0" in prob:
            p.h0 = float(prob["h0"])
    return p


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Oracle:
    """One FP64 CPU solve of a workload description."""

    def __init__(self, prob: dict, init: bool = True, library=None):
        self.prob = prob
        self._L = library if library is not None else lib()
        self.params = make_params(prob)
        self.nx, self.ny = self.params.nx, self.params.ny
        self._h = self._L.orc_new(C.byref(self.params))
        if not self._h:
            raise ValueError("oracle rejected the parameters")
        self.init_sweeps = self._L.orc_init(self._h) if init else 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.orc_free(h)
            self._h = None

    @property
    def n(self) -> int:
        return self.nx * self.ny

    def step(self, n: int = 1) -> None:
        self._L.orc_step(self._h, int(n))

    def rhs(self) -> np.ndarray:
        out = np.zeros(5 * self.n)
        self._L.orc_rhs(self._h, _dp(out))
        return out.reshape(5, self.ny, self.nx)

    def face_fluxes(self):
        fx = np.zeros(5 * (self.nx + 1) * self.ny)
        fy = np.zeros(5 * self.nx * (self.ny + 1))
        self._L.orc_face_fluxes(self._h, _dp(fx), _dp(fy))
        return fx.reshape(5, self.ny, self.nx + 1), fy.reshape(5, self.ny + 1, self.nx)

    def face_inputs(self) -> np.ndarray:
        """Inputs of the face fluxes per cell, (27, ny, nx): p, u, v, rho, C, mu_c, T, He,
        their x gradients, their y gradients, then mu, lambda and Cp."""
        out = np.zeros(27 * self.n)
        self._L.orc_face_inputs(self._h, _dp(out))
        return out.reshape(27, self.ny, self.nx)

    def get(self, name: str) -> np.ndarray:
        out = np.zeros(self.n)
        self._L.orc_get(self._h, FIELDS[name], _dp(out))
        return out.reshape(self.ny, self.nx)

    def set(self, name: str, arr) -> None:
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(arr, dtype=np.float64), (self.ny, self.nx)))
        self._L.orc_set(self._h, FIELDS[name], _dp(a))

    def set_state(self, state: dict) -> None:
        for k, v in state.items():
            self.set(k, v)

    def set_time(self, t: float, step: float) -> None:
        self._L.orc_set_time(self._h, float(t), float(step))

    def observe(self) -> dict:
        o = Obs()
        self._L.orc_observe(self._h, C.byref(o))
        return {n: getattr(o, n) for n, _ in Obs._fields_}

    def mag_sweeps(self, n: int, omega: float = 1.0) -> float:
        return self._L.orc_mag_sweeps(self._h, int(n), float(omega))

    def mag_residual(self) -> float:
        return self._L.orc_mag_residual(self._h)

    def mag_lbfs(self, n: int, D: float = 1.0, dtau: float = 0.0) -> float:
        """n pseudo-time RK3 steps of the magnetic LBFS (Eq. 17); returns ||r||_2."""
        return self._L.orc_mag_lbfs(self._h, int(n), float(D), float(dtau))

    def mag_lbfs_fluxes(self, D: float = 1.0):
        """Normal m* fluxes (Eq. 18) of the current potential: (ny, nx+1), (ny+1, nx)."""
        fx = np.zeros((self.nx + 1) * self.ny)
        fy = np.zeros(self.nx * (self.ny + 1))
        self._L.orc_mag_lbfs_fluxes(self._h, float(D), _dp(fx), _dp(fy))
        return fx.reshape(self.ny, self.nx + 1), fy.reshape(self.ny + 1, self.nx)

    def wall_heat_profile(self) -> np.ndarray:
        """Local heat flux -lambda dT/dy on the south wall, one value per column."""
        out = np.zeros(self.nx)
        self._L.orc_wall_heat_profile(self._h, _dp(out))
        return out

    def mag_lbfs_dtau(self, D: float = 1.0) -> float:
        return self._L.orc_mag_lbfs_dtau(C.byref(self.params), float(D))


def lattice():
    ex, ey, w = np.zeros(9), np.zeros(9), np.zeros(9)
    lib().orc_lattice(_dp(ex), _dp(ey), _dp(w))
    return ex, ey, w


def enthalpy_state(prob: dict, He: float, Cval: float):
    p = make_params(prob)
    T, Fl = C.c_double(), C.c_double()
    lib().orc_enthalpy_state(C.byref(p), float(He), float(Cval), C.byref(T), C.byref(Fl))
    return T.value, Fl.value


def equilibria(prob: dict, pr, rho, u, v, Cval, muc, He, T, cp):
    p = make_params(prob)
    f, g, h = np.zeros(9), np.zeros(9), np.zeros(9)
    lib().orc_equilibria(C.byref(p), pr, rho, u, v, Cval, muc, He, T, cp, _dp(f), _dp(g), _dp(h))
    return f, g, h

