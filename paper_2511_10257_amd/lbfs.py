"""Python binding of the C ABI in include/lbfs.h (argument marshalling only).

Every step of the solver runs in the gfx950 kernels of liblbfs.so; PyTorch only
provides the device buffer and the stream. Importing works without a GPU (the
host-only calls such as lbfs_state_bytes can be used for validation); creating a
Solver needs the built library and a ROCm device and raises otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblbfs.so")

LBFS_ABI_VERSION = 3
LBFS_OK, LBFS_E_INVAL, LBFS_E_NOMEM, LBFS_E_NONFINITE, LBFS_E_DEVICE, LBFS_E_STATE, LBFS_E_ABI = (
    0, -1, -2, -3, -4, -5, -6)
LBFS_FP32, LBFS_FP64 = 0, 1
FIELDS = dict(He=0, p=1, Mx=2, My=3, C=4, phi=5, S=6, T=7, Fl=8)
KERNELS = ("mag", "stage1", "stage2", "stage3", "reduce")
NKERNELS = len(KERNELS)

# every symbol include/lbfs.h declares
EXPORTS = (
    "lbfs_params_default", "lbfs_params_from_dimless", "lbfs_state_bytes", "lbfs_init",
    "lbfs_step", "lbfs_step_profiled", "lbfs_step_profiled_start", "lbfs_profile_result", "lbfs_prepare",
    "lbfs_observe", "lbfs_rhs", "lbfs_mag_sweeps",
    "lbfs_mag_pseudo_steps", "lbfs_mag_multigrid", "lbfs_wall_heat_profile", "lbfs_read_field",
    "lbfs_write_field", "lbfs_set_time", "lbfs_checkpoint_bytes", "lbfs_save_state",
    "lbfs_load_state", "lbfs_destroy", "lbfs_strerror", "lbfs_step_fields",
    "lbfs_tile_shape", "lbfs_set_tile_shapes", "lbfs_tile_shapes_in_use", "lbfs_autotune",
    "lbfs_batch_instance_bytes", "lbfs_batch_create", "lbfs_batch_admit", "lbfs_batch_retire",
    "lbfs_batch_step", "lbfs_batch_step_profiled", "lbfs_batch_step_profiled_start", "lbfs_batch_profile_result",
    "lbfs_batch_prepare", "lbfs_batch_observe", "lbfs_batch_slot",
    "lbfs_batch_info", "lbfs_batch_destroy", "lbfs_batch_set_tile_shapes", "lbfs_batch_autotune",
    "lbfs_batch_tile_shapes_in_use",
)
MAX_SHAPES = 8


class Params(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("nx", C.c_int32), ("ny", C.c_int32), ("precision", C.c_int32),
        ("dx", C.c_double), ("dt", C.c_double), ("dt_stream", C.c_double),
        ("rho", C.c_double * 3), ("mu", C.c_double * 3), ("cp", C.c_double * 3),
        ("lambda_", C.c_double * 3), ("chi", C.c_double * 3),
        ("latent", C.c_double), ("t_melt", C.c_double), ("t_init", C.c_double),
        ("mu0", C.c_double), ("h0", C.c_double), ("field_angle_deg", C.c_double),
        ("gravity", C.c_double * 2), ("sigma", C.c_double), ("xi", C.c_double),
        ("mobility", C.c_double), ("tau_g", C.c_double),
        ("drop_cx", C.c_double), ("drop_cy", C.c_double), ("drop_radius", C.c_double),
        ("init_kind", C.c_int32), ("c_init", C.c_double),
        ("periodic", C.c_int32 * 2), ("thermal_bc", C.c_int32 * 4), ("thermal_val", C.c_double * 4),
        ("mag_bc", C.c_int32 * 4), ("sweeps", C.c_int32), ("sor_omega", C.c_double),
        ("init_omega", C.c_double), ("init_tol", C.c_double), ("init_max", C.c_int32),
        ("init_check", C.c_int32),
        ("mag_method", C.c_int32), ("mag_lbfs_d", C.c_double), ("mag_lbfs_dtau", C.c_double),
        ("mag_max_iters", C.c_int32), ("mag_tol", C.c_double),
        ("contact_angle_deg", C.c_double * 4), ("t_liquidus", C.c_double),
    ]


class Observables(C.Structure):
    _fields_ = [
        ("t", C.c_double), ("liquid_fraction", C.c_double), ("solid_ratio", C.c_double),
        ("volume", C.c_double), ("volume0", C.c_double), ("mag_residual", C.c_double),
        ("umax", C.c_double), ("umax_drop", C.c_double), ("height", C.c_double),
        ("wall_heat", C.c_double), ("fourier", C.c_double), ("peclet", C.c_double),
        ("centroid_x", C.c_double), ("centroid_y", C.c_double), ("semi_axis_x", C.c_double),
        ("semi_axis_y", C.c_double), ("semi_axis_major", C.c_double), ("semi_axis_minor", C.c_double),
        ("major_axis_deg", C.c_double), ("solid_height", C.c_double),
        ("step", C.c_int64), ("nonfinite", C.c_int32),
    ]


class LbfsError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {strerror(status)} ({status})")
        self.status = status


_lib = None


def lib():
    """Load liblbfs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        # PyTorch ships its own HIP runtime under the same soname as the system one that
        # liblbfs.so links against; loading torch first makes both use that one runtime
        # (two runtimes in one process do not share devices, streams or memory)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, dp, i32 = C.c_void_p, C.POINTER(C.c_double), C.c_int32
        sig = {
            "lbfs_params_default": (C.c_int, [C.POINTER(Params), i32, i32, i32]),
            "lbfs_params_from_dimless": (C.c_int, [C.POINTER(Params), C.c_double, C.c_double, C.c_double, C.c_double]),
            "lbfs_state_bytes": (C.c_size_t, [C.POINTER(Params)]),
            "lbfs_init": (C.c_int, [C.POINTER(Params), vp, C.c_size_t, vp, C.POINTER(vp)]),
            "lbfs_step": (C.c_int, [vp, i32]),
            "lbfs_step_profiled": (C.c_int, [vp, i32, i32, dp, C.POINTER(C.c_int32)]),
            "lbfs_step_profiled_start": (C.c_int, [vp, i32, i32]),
            "lbfs_profile_result": (C.c_int, [vp, dp, C.POINTER(C.c_int32)]),
            "lbfs_prepare": (C.c_int, [vp]),
            "lbfs_observe": (C.c_int, [vp, C.POINTER(Observables)]),
            "lbfs_rhs": (C.c_int, [vp, dp]),
            "lbfs_mag_sweeps": (C.c_int, [vp, i32, C.c_double, dp]),
            "lbfs_mag_pseudo_steps": (C.c_int, [vp, i32, dp]),
            "lbfs_mag_multigrid": (C.c_int, [vp, i32, dp]),
            "lbfs_wall_heat_profile": (C.c_int, [vp, dp, C.c_size_t]),
            "lbfs_read_field": (C.c_int, [vp, i32, dp, C.c_size_t]),
            "lbfs_write_field": (C.c_int, [vp, i32, dp, C.c_size_t]),
            "lbfs_set_time": (C.c_int, [vp, C.c_double, C.c_int64]),
            "lbfs_checkpoint_bytes": (C.c_size_t, [vp]),
            "lbfs_save_state": (C.c_int, [vp, vp, C.c_size_t]),
            "lbfs_load_state": (C.c_int, [vp, vp, C.c_size_t]),
            "lbfs_destroy": (None, [vp]),
            "lbfs_step_fields": (C.c_int, [C.POINTER(Params), C.POINTER(vp), i32, vp]),
            "lbfs_strerror": (C.c_char_p, [C.c_int]),
            "lbfs_tile_shape": (C.c_int, [i32, i32, i32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                          C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
            "lbfs_set_tile_shapes": (C.c_int, [vp, i32, i32]),
            "lbfs_tile_shapes_in_use": (C.c_int, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
            "lbfs_batch_tile_shapes_in_use": (C.c_int, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
            "lbfs_autotune": (C.c_int, [vp, i32, C.POINTER(C.c_int32), dp]),
            "lbfs_batch_set_tile_shapes": (C.c_int, [vp, i32, i32]),
            "lbfs_batch_autotune": (C.c_int, [vp, i32, C.POINTER(C.c_int32), dp]),
            "lbfs_batch_instance_bytes": (C.c_size_t, [C.POINTER(Params)]),
            "lbfs_batch_create": (C.c_int, [i32, i32, i32, C.c_double, vp, C.c_size_t, vp, C.POINTER(vp)]),
            "lbfs_batch_admit": (C.c_int, [vp, C.POINTER(Params), C.POINTER(C.c_int32)]),
            "lbfs_batch_retire": (C.c_int, [vp, i32]),
            "lbfs_batch_step": (C.c_int, [vp, i32]),
            "lbfs_batch_step_profiled": (C.c_int, [vp, i32, i32, dp, C.POINTER(C.c_int32)]),
            "lbfs_batch_step_profiled_start": (C.c_int, [vp, i32, i32]),
            "lbfs_batch_profile_result": (C.c_int, [vp, dp, C.POINTER(C.c_int32)]),
            "lbfs_batch_prepare": (C.c_int, [vp]),
            "lbfs_batch_observe": (C.c_int, [vp, C.POINTER(Observables), C.POINTER(C.c_uint8)]),
            "lbfs_batch_slot": (C.c_int, [vp, i32, C.POINTER(vp)]),
            "lbfs_batch_info": (C.c_int, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]),
            "lbfs_batch_destroy": (None, [vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return lib().lbfs_strerror(int(status)).decode()


def _check(status: int, what: str) -> None:
    if status != LBFS_OK:
        raise LbfsError(status, what)


_TBC = {"adiabatic": 0, "fixed": 1}
_MBC = {"insulating": 0, "fixed": 1}
_MAG = {"sweeps": 0, "lbfs": 1, "multigrid": 2}


def make_params(prob: dict) -> Params:
    """lbfs_params from a workload description (see workloads.py)."""
    prec = LBFS_FP64 if prob.get("precision", "fp32") == "fp64" else LBFS_FP32
    p = Params()
    _check(lib().lbfs_params_default(C.byref(p), int(prob["nx"]), int(prob["ny"]), prec), "params_default")
    p.dx = float(prob.get("dx", 1.0))
    p.dt = float(prob.get("dt", 0.5))
    p.dt_stream = float(prob.get("dt_stream", 0.0))
    for name, key in (("rho", "rho"), ("mu", "mu"), ("cp", "cp"), ("lambda_", "lam"), ("chi", "chi")):
        if key in prob:
            arr = getattr(p, name)
            for k in range(3):
                arr[k] = float(prob[key][k])
    for key in ("t_melt", "t_init", "mu0", "sigma", "xi", "mobility", "tau_g", "c_init",
                "init_omega", "init_tol"):
        if key in prob:
            setattr(p, key, float(prob[key]))
    if "grav" in prob:
        p.gravity[0], p.gravity[1] = [float(g) for g in prob["grav"]]
    if "drop" in prob:
        p.drop_cx, p.drop_cy, p.drop_radius = [float(v) for v in prob["drop"]]
    p.init_kind = 0 if prob.get("init_kind", "droplet") == "droplet" else 1
    if "periodic" in prob:
        p.periodic[0], p.periodic[1] = [int(v) for v in prob["periodic"]]
    for k in range(4):
        if "thermal_bc" in prob:
            p.thermal_bc[k] = _TBC[prob["thermal_bc"][k]]
        if "thermal_val" in prob:
            p.thermal_val[k] = float(prob["thermal_val"][k])
        if "mag_bc" in prob:
            p.mag_bc[k] = _MBC[prob["mag_bc"][k]]
    p.sweeps = int(prob.get("sweeps", 4))
    p.sor_omega = float(prob.get("omega", 1.0))
    p.mag_method = _MAG[prob.get("mag_method", "sweeps")]
    p.mag_lbfs_d = float(prob.get("mag_lbfs_d", 1.0))
    p.mag_lbfs_dtau = float(prob.get("mag_lbfs_dtau", 0.0))
    p.mag_max_iters = int(prob.get("mag_max_iters", 0))
    p.mag_tol = float(prob.get("mag_tol", 0.0))
    for k, a in enumerate(prob.get("contact_angle", [90.0] * 4)):
        p.contact_angle_deg[k] = float(a)
    p.t_liquidus = float(prob.get("t_liquidus", p.t_melt))
    for key in ("init_max", "init_check"):
        if key in prob:
            setattr(p, key, int(prob[key]))
    angle = float(prob.get("angle_deg", p.field_angle_deg))
    if "latent" in prob and "h0" in prob:
        p.latent, p.h0 = float(prob["latent"]), float(prob["h0"])
        p.field_angle_deg = angle
    else:
        # Eq. 50 conversions happen in the library; they also set the fixed south wall
        tbc2, tval2 = p.thermal_bc[2], p.thermal_val[2]
        _check(lib().lbfs_params_from_dimless(C.byref(p), float(prob["ste"]), float(prob["t_wall"]),
                                              float(prob["bo_m"]), angle), "params_from_dimless")
        p.thermal_bc[2], p.thermal_val[2] = tbc2, tval2
        if "latent" in prob:
            p.latent = float(prob["latent"])
        if "h0" in prob:
            p.h0 = float(prob["h0"])
    return p


def tile_shapes(kind: str, precision: str = "fp32") -> list:
    """Candidate tile shapes (tx, ty, threads, flags) of the "stage" or "mag" kernels."""
    k = 0 if kind == "stage" else 1
    prec = LBFS_FP64 if precision == "fp64" else LBFS_FP32
    n = lib().lbfs_tile_shape(k, prec, -1, None, None, None, None)
    out = []
    for i in range(n):
        tx, ty, nt, fl = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().lbfs_tile_shape(k, prec, i, C.byref(tx), C.byref(ty), C.byref(nt), C.byref(fl)),
               "lbfs_tile_shape")
        out.append((tx.value, ty.value, nt.value, fl.value))
    return out


def mag_fused_index(precision: str = "fp32") -> int:
    """The magnetic "shape" index that runs the step's sweeps inside stage 1."""
    return len(tile_shapes("mag", precision))


def shape_name(shape: tuple) -> str:
    """'TXxTY/threads', with an 'e' for the early owned-cell loads of the first stages;
    'in-stage-1' for the sweeps run inside stage 1."""
    if shape[3] & 2:
        return "in-stage-1"
    return f"{shape[0]}x{shape[1]}/{shape[2]}" + ("e" if shape[3] & 1 else "")


def mag_shape(index: int, precision: str = "fp32") -> tuple:
    """(tx, ty, threads, flags) of a magnetic shape index, the fused index included."""
    k = 1
    prec = LBFS_FP64 if precision == "fp64" else LBFS_FP32
    tx, ty, nt, fl = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().lbfs_tile_shape(k, prec, int(index), C.byref(tx), C.byref(ty), C.byref(nt), C.byref(fl)),
           "lbfs_tile_shape")
    return (tx.value, ty.value, nt.value, fl.value)


def _tune_result(chosen, ms, precision: str) -> dict:
    """ms per whole step for each stage shape and each magnetic shape, and (where it was
    a candidate) the step with the sweeps inside stage 1 minus the best other step."""
    ns, nm = len(tile_shapes("stage", precision)), len(tile_shapes("mag", precision))
    out = {"stage_shape": chosen[0], "mag_shape": chosen[1],
           "stage_ms": [ms[k] for k in range(ns)], "mag_ms": [ms[MAX_SHAPES + k] for k in range(nm)]}
    if ms[MAX_SHAPES + nm] != 0.0:
        out["fused_step_minus_best_ms"] = ms[MAX_SHAPES + nm]
    return out


def state_bytes(prob_or_params) -> int:
    p = prob_or_params if isinstance(prob_or_params, Params) else make_params(prob_or_params)
    return int(lib().lbfs_state_bytes(C.byref(p)))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class _Instance:
    """Calls on one instance handle (owned by a Solver, or borrowed from a Batch slot)."""

    _h = None
    nx = ny = 0

    @property
    def n(self) -> int:
        return self.nx * self.ny

    def observe(self, allow_nonfinite: bool = False) -> dict:
        o = Observables()
        st = lib().lbfs_observe(self._h, C.byref(o))
        if not (st == LBFS_OK or (allow_nonfinite and st == LBFS_E_NONFINITE)):
            _check(st, "lbfs_observe")
        return _obs_dict(o)

    def rhs(self) -> np.ndarray:
        out = np.zeros(5 * self.n)
        _check(lib().lbfs_rhs(self._h, _dp(out)), "lbfs_rhs")
        return out.reshape(5, self.ny, self.nx)

    def get(self, name: str) -> np.ndarray:
        out = np.zeros(self.n)
        _check(lib().lbfs_read_field(self._h, FIELDS[name], _dp(out), self.n), "lbfs_read_field")
        return out.reshape(self.ny, self.nx)

    def set(self, name: str, arr) -> None:
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(arr, dtype=np.float64), (self.ny, self.nx)))
        _check(lib().lbfs_write_field(self._h, FIELDS[name], _dp(a), self.n), "lbfs_write_field")

    def set_state(self, state: dict) -> None:
        for k, v in state.items():
            self.set(k, v)

    def wall_heat_profile(self) -> np.ndarray:
        """Local heat flux -lambda dT/dy on the south wall, one value per column."""
        out = np.zeros(self.nx)
        _check(lib().lbfs_wall_heat_profile(self._h, out.ctypes.data_as(C.POINTER(C.c_double)), out.size),
               "lbfs_wall_heat_profile")
        return out

    def set_time(self, t: float, step: int) -> None:
        _check(lib().lbfs_set_time(self._h, float(t), int(step)), "lbfs_set_time")

    def save(self) -> bytes:
        nb = int(lib().lbfs_checkpoint_bytes(self._h))
        buf = C.create_string_buffer(nb)
        _check(lib().lbfs_save_state(self._h, buf, nb), "lbfs_save_state")
        return buf.raw

    def load(self, blob: bytes) -> None:
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().lbfs_load_state(self._h, buf, len(blob)), "lbfs_load_state")


def _obs_dict(o: Observables) -> dict:
    return {n: getattr(o, n) for n, _ in Observables._fields_}


def _kernel_times(ms, cnt) -> dict:
    return {KERNELS[k]: (ms[k], cnt[k]) for k in range(NKERNELS)}


class Solver(_Instance):
    """One LBFS solve resident on a ROCm device; state lives in a torch uint8 buffer."""

    def __init__(self, prob, device: str = "cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the LBFS solver needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.params = prob if isinstance(prob, Params) else make_params(prob)
        self.nx, self.ny = self.params.nx, self.params.ny
        nbytes = int(lib().lbfs_state_bytes(C.byref(self.params)))
        if nbytes == 0:
            raise LbfsError(LBFS_E_INVAL, "lbfs_state_bytes")
        self.device = torch.device(device)
        self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        # a stream of its own (default priority) so that a step can be replayed as a graph
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().lbfs_init(C.byref(self.params), C.c_void_p(self.buffer.data_ptr()), nbytes,
                                   C.c_void_p(self.stream.cuda_stream), C.byref(h)), "lbfs_init")
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().lbfs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1) -> None:
        _check(lib().lbfs_step(self._h, int(n)), "lbfs_step")

    def prepare(self) -> None:
        """Capture every step graph now (no step runs; the state is unchanged)."""
        _check(lib().lbfs_prepare(self._h), "lbfs_prepare")

    def step_profiled(self, n: int, sample_every: int = 10) -> dict:
        """Steps with HIP events around the kernels of every sample_every-th step;
        returns {kernel kind: (mean ms per launch, timed launches)}."""
        ms = (C.c_double * NKERNELS)()
        cnt = (C.c_int32 * NKERNELS)()
        _check(lib().lbfs_step_profiled(self._h, int(n), int(sample_every), ms, cnt), "lbfs_step_profiled")
        return _kernel_times(ms, cnt)

    def step_profiled_start(self, n: int, sample_every: int = 10) -> None:
        """step_profiled without waiting: enqueue the steps and their timing events."""
        _check(lib().lbfs_step_profiled_start(self._h, int(n), int(sample_every)), "lbfs_step_profiled_start")

    def profile_result(self) -> dict:
        """Wait for the run step_profiled_start enqueued; its kernel times as step_profiled."""
        ms = (C.c_double * NKERNELS)()
        cnt = (C.c_int32 * NKERNELS)()
        _check(lib().lbfs_profile_result(self._h, ms, cnt), "lbfs_profile_result")
        return _kernel_times(ms, cnt)

    def mag_sweeps(self, n: int, omega: float = 1.0) -> float:
        r = C.c_double()
        _check(lib().lbfs_mag_sweeps(self._h, int(n), float(omega), C.byref(r)), "lbfs_mag_sweeps")
        return r.value

    def mag_multigrid(self, n: int) -> float:
        """n multigrid V(2,2) cycles of the compact magnetic system; returns ||r||_2."""
        r = C.c_double()
        _check(lib().lbfs_mag_multigrid(self._h, int(n), C.byref(r)), "lbfs_mag_multigrid")
        return r.value

    def mag_pseudo_steps(self, n: int) -> float:
        """n pseudo-time steps of the magnetic LBFS solve (Eq. 17); returns ||r||_2."""
        r = C.c_double()
        _check(lib().lbfs_mag_pseudo_steps(self._h, int(n), C.byref(r)), "lbfs_mag_pseudo_steps")
        return r.value

    def set_tile_shapes(self, stage_shape: int, mag_shape: int) -> None:
        _check(lib().lbfs_set_tile_shapes(self._h, int(stage_shape), int(mag_shape)), "lbfs_set_tile_shapes")

    def tile_shapes_in_use(self) -> tuple:
        """(stage shape index, magnetic shape index) of the next launches."""
        a, b = C.c_int32(), C.c_int32()
        _check(lib().lbfs_tile_shapes_in_use(self._h, C.byref(a), C.byref(b)), "lbfs_tile_shapes_in_use")
        return a.value, b.value

    def autotune(self, reps: int = 20) -> dict:
        """Time the candidate tile shapes on the current state and keep the fastest."""
        chosen = (C.c_int32 * 2)()
        ms = (C.c_double * (2 * MAX_SHAPES))()
        _check(lib().lbfs_autotune(self._h, int(reps), chosen, ms), "lbfs_autotune")
        return _tune_result(chosen, ms, "fp64" if self.params.precision == LBFS_FP64 else "fp32")


class _SlotView(_Instance):
    """Borrowed handle of a batch slot (valid until the slot is retired)."""

    def __init__(self, handle, nx: int, ny: int):
        self._h, self.nx, self.ny = handle, nx, ny


class Batch:
    """Many independent solves advanced by the same launches (lbfs_batch_*); the state of
    every instance is carved from one torch uint8 buffer of `nbytes` bytes."""

    def __init__(self, max_slots: int, nbytes: int, precision: str = "fp32", sweeps: int = 4,
                 omega: float = 1.0, device: str = "cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the LBFS batch needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.max_slots = int(max_slots)
        self.precision = precision
        self.device = torch.device(device)
        self.buffer = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self._dims = {}
        h = C.c_void_p()
        prec = LBFS_FP64 if precision == "fp64" else LBFS_FP32
        with torch.cuda.device(self.device):
            _check(lib().lbfs_batch_create(self.max_slots, prec, int(sweeps), float(omega),
                                           C.c_void_p(self.buffer.data_ptr()), int(nbytes),
                                           C.c_void_p(self.stream.cuda_stream), C.byref(h)), "lbfs_batch_create")
        self._h = h

    @staticmethod
    def instance_bytes(prob) -> int:
        p = prob if isinstance(prob, Params) else make_params(prob)
        return int(lib().lbfs_batch_instance_bytes(C.byref(p)))

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().lbfs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, prob):
        """Admit a problem; returns its slot, or None when the batch has no room."""
        p = prob if isinstance(prob, Params) else make_params(prob)
        slot = C.c_int32(-1)
        st = lib().lbfs_batch_admit(self._h, C.byref(p), C.byref(slot))
        if st == LBFS_E_NOMEM:
            return None
        _check(st, "lbfs_batch_admit")
        self._dims[slot.value] = (p.nx, p.ny)
        return slot.value

    def retire(self, slot: int) -> None:
        _check(lib().lbfs_batch_retire(self._h, int(slot)), "lbfs_batch_retire")
        self._dims.pop(int(slot), None)

    def step(self, n: int = 1) -> None:
        _check(lib().lbfs_batch_step(self._h, int(n)), "lbfs_batch_step")

    def prepare(self) -> None:
        """Capture the step graphs of the live instances now (no step runs)."""
        _check(lib().lbfs_batch_prepare(self._h), "lbfs_batch_prepare")

    def step_profiled(self, n: int, sample_every: int = 10) -> dict:
        ms = (C.c_double * NKERNELS)()
        cnt = (C.c_int32 * NKERNELS)()
        _check(lib().lbfs_batch_step_profiled(self._h, int(n), int(sample_every), ms, cnt),
               "lbfs_batch_step_profiled")
        return _kernel_times(ms, cnt)

    def step_profiled_start(self, n: int, sample_every: int = 10) -> None:
        _check(lib().lbfs_batch_step_profiled_start(self._h, int(n), int(sample_every)),
               "lbfs_batch_step_profiled_start")

    def profile_result(self) -> dict:
        ms = (C.c_double * NKERNELS)()
        cnt = (C.c_int32 * NKERNELS)()
        _check(lib().lbfs_batch_profile_result(self._h, ms, cnt), "lbfs_batch_profile_result")
        return _kernel_times(ms, cnt)

    def observe(self, allow_nonfinite: bool = False) -> dict:
        """{slot: observables} of the live instances."""
        out = (Observables * self.max_slots)()
        live = (C.c_uint8 * self.max_slots)()
        st = lib().lbfs_batch_observe(self._h, out, live)
        if not (st == LBFS_OK or (allow_nonfinite and st == LBFS_E_NONFINITE)):
            _check(st, "lbfs_batch_observe")
        return {k: _obs_dict(out[k]) for k in range(self.max_slots) if live[k]}

    def slot(self, k: int) -> _SlotView:
        h = C.c_void_p()
        _check(lib().lbfs_batch_slot(self._h, int(k), C.byref(h)), "lbfs_batch_slot")
        nx, ny = self._dims[int(k)]
        return _SlotView(h, nx, ny)

    def set_tile_shapes(self, stage_shape: int, mag_shape: int) -> None:
        _check(lib().lbfs_batch_set_tile_shapes(self._h, int(stage_shape), int(mag_shape)),
               "lbfs_batch_set_tile_shapes")

    def tile_shapes_in_use(self) -> tuple:
        a, b = C.c_int32(), C.c_int32()
        _check(lib().lbfs_batch_tile_shapes_in_use(self._h, C.byref(a), C.byref(b)),
               "lbfs_batch_tile_shapes_in_use")
        return a.value, b.value

    def autotune(self, reps: int = 20) -> dict:
        """Time the candidate tile shapes over all live instances and keep the fastest."""
        chosen = (C.c_int32 * 2)()
        ms = (C.c_double * (2 * MAX_SHAPES))()
        _check(lib().lbfs_batch_autotune(self._h, int(reps), chosen, ms), "lbfs_batch_autotune")
        return _tune_result(chosen, ms, self.precision)

    def info(self) -> dict:
        n, c, f = C.c_int32(), C.c_int64(), C.c_size_t()
        _check(lib().lbfs_batch_info(self._h, C.byref(n), C.byref(c), C.byref(f)), "lbfs_batch_info")
        return {"live": n.value, "cells": c.value, "largest_free": f.value}
