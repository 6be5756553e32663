"""Benchmark of the coupled LBFS time step on one MI355X.

Workload (default): the 256 x 256 freezing droplet (radius 64, Ste 0.1, field angle
0 or 90 deg and magnetic Bond number ~ U[0, 2] drawn with seed 0), FP32 fields with
FP64 reductions, 4 red-black sweeps per step. One "step" is the whole hot path: the
magnetic sweeps and residual, three fused Runge-Kutta stages with the Kelvin force,
the end-of-step Eq. 8 update and the FP64 reductions.

Other workloads: droplet64 (64 x 64, FP64), droplet1024 / droplet1024-fp64 (1024 x 1024),
batch64 (64 uneven instances advanced by the same launches) and serve (a Poisson stream
of freezing requests served by continuous batching, FP32, beside the same stream served
one solve at a time in FP64).

Prints one JSON line: throughput in MLUPS (cell updates per second / 1e6; solves/s for
serve) with the state resident in HBM, the roofline of the dominant kernel (its mean
launch duration from HIP events recorded on the solver's stream inside the timed
region), and the FP64 CPU oracle timed on a bounded sample of the same workload on the
host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coupled LBFS step MLUPS (FP32 vs FP64 at stated err); solves/s + p99 latency"
HBM_PEAK_GBS = 8000.0
# vector ALU peaks of MI355X: 256 CUs x 64 lanes x 2 (FMA) x 2.4 GHz = 78.6 TFLOP/s per
# issued instruction stream; FP32 doubles that with packed FP32 instructions (157.3)
VALU_PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}
VALU_PEAK_NONPACKED_TFLOPS = 78.6

# algorithmic field accesses per cell and launch (one field = one value per cell)
FIELD_ACCESSES = {
    "mag": 4.0,       # read C, He, phi'; write phi' (permeability, sweeps, residual in LDS)
    "stage1": 12.0,   # read W, phi', S; write W1
    "stage2": 17.0,   # read W1, W, phi', S; write W2
    "stage3": 18.0,   # read W2, W, phi', S; write W, S (plus per-tile partial sums)
    "reduce": 0.0,
}
# algorithmic floating-point operations per cell and launch: the operation count of the
# definitional algorithm (per-direction equilibria at the nine Eq. 44 points, Eq. 45 face
# state, star distributions, moments, sources, the Runge-Kutta combination; a division
# or square root counts as one), measured by compiling the oracle with a counting number
# type (oracle/opcount.py) on the 256 x 256 droplet: 13993 per cell-step, of which the
# magnetic phase (permeability, 4 sweeps, residual) takes 152.7 and each stage 4613.4
ALG_FLOPS = {"mag": 152.7, "stage1": 4613.4, "stage2": 4613.4, "stage3": 4613.4, "reduce": 0.0}
# the magnetic phase by the LBFS pseudo-time solve, counted the same way on the oracle's
# literal m* construction (nine reconstructed points, compatibility sum, equilibria and
# star distributions per face): 51.8 per cell for the permeability and residual plus
# 1682.5 per cell and pseudo-step. The kernel evaluates the exact reduction of that
# construction at delta_t = dx/2 (about 45 operations per cell and pseudo-step), so
# this count measures the definitional algorithm, not the instructions issued.
ALG_FLOPS_MAG_LBFS = (51.8, 1682.5)
# and by the sweeps: 51.8 per cell for the permeability and residual, 25.2 per sweep
ALG_FLOPS_MAG_SWEEPS = (51.8, 25.23)
# the resource that bounds each kernel: the sweeps stream fields with little arithmetic,
# the stages are far above the ridge point (68 FLOP/B against 19.7 FP32 / 9.8 FP64)
BOUND = {"mag": "hbm", "stage1": "alu", "stage2": "alu", "stage3": "alu", "reduce": "hbm"}


DEFAULT_STEPS = {"droplet64": 2000, "droplet256": 20000, "droplet1024": 1000, "droplet1024-fp64": 1000,
                 "droplet4096": 200, "batch64": 1000}
DEFAULT_WARMUP = {"droplet64": 100, "droplet256": 200, "droplet1024": 100, "droplet1024-fp64": 100,
                  "droplet4096": 10, "batch64": 100}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default per workload)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default per workload)")
    ap.add_argument("--workload", default="droplet256",
                    choices=["droplet64", "droplet256", "droplet1024", "droplet1024-fp64", "droplet4096", "batch64",
                             "serve"])
    ap.add_argument("--sample-every", type=int, default=97,
                    help="bracket the kernels of every n-th timed step with HIP events (the 96 steps "
                         "between two sampled ones run as six 16-step graph replays)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--freeze-check", action="store_true",
                    help="solve the workload to freezing in FP32 and in FP64 and report both freezing steps "
                         "(single solves; about 17 minutes for droplet1024)")
    ap.add_argument("--no-freeze-check", action="store_true",
                    help="droplet256: skip solving the workload to freezing in FP32 and FP64 (about 10 s; "
                         "also skipped with --no-cpu-baseline)")
    ap.add_argument("--no-host-io", action="store_true",
                    help="skip the rates with per-step observables or checkpoints over PCIe")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run a plain device copy of this size (HBM counter calibration)")
    ap.add_argument("--tile-shapes", default=None, metavar="STAGE,MAG",
                    help="use these tile-shape indices instead of the defaults or the autotuner (counter "
                         "runs: collecting counters distorts the autotuner's timings)")
    ap.add_argument("--autotune", choices=["auto", "on", "off"], default="auto",
                    help="time the candidate tile shapes first (auto: for the batch only; single solves "
                         "keep the default shapes, so that runs and profiles use the same kernels)")
    # serving
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="arrivals are cut after this time")
    ap.add_argument("--serve-drain", type=float, default=60.0, help="hard cap after the last arrival")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="mean arrivals per second")
    ap.add_argument("--serve-edges", default="96,128,256,512", help="grid edges the requests draw from")
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-budget-gib", type=float, default=32.0)
    ap.add_argument("--serve-chunk", type=int, default=200, help="steps between observations")
    ap.add_argument("--no-serve-baseline", action="store_true")
    ap.add_argument("--mag-method", choices=["sweeps", "lbfs", "multigrid"], default="sweeps",
                    help="per-step magnetic update of the single-solve workloads: red-black sweeps, "
                         "the LBFS pseudo-time solve (Eq. 17) or multigrid V-cycles (--mag-steps of them)")
    ap.add_argument("--mag-steps", type=int, default=None,
                    help="sweeps or pseudo-steps per time step (default: the workload's)")
    ap.add_argument("--mag-in-stage1", choices=["auto", "on", "off"], default="auto",
                    help="run the step's sweeps inside Runge-Kutta stage 1 (no magnetic launch): on, off, "
                         "or the library's default for the grid")
    ap.add_argument("--mag-max-iters", type=int, default=0,
                    help="convergence control: repeat chunks of --mag-steps iterations per step until the "
                         "magnetic residual is at most --mag-tol, at most this many iterations (0: off)")
    ap.add_argument("--mag-tol", type=float, default=0.0, help="absolute ||r||_2 target of the convergence control")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = DEFAULT_STEPS.get(args.workload, 0)
    if args.warmup is None:
        args.warmup = DEFAULT_WARMUP.get(args.workload, 0)
    return args


def kernel_sources_digest() -> str:
    h = hashlib.sha256()
    # the kernel sources and the build script (its compiler flags shape the kernels too)
    for name in ("csrc/lbfs_kernels.hip", "csrc/lbfs_internal.hpp", "build.py"):
        with open(os.path.join(ROOT, "paper_2511_10257_amd", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, shape: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel sources with the same tile shape."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_sources_sha256_16:\s*([0-9a-f]+)", text)
    if not m or m.group(1) != kernel_sources_digest():
        return None
    m = re.search(rf"^\|\s*{kernel}\s*\|\s*([^|]*?)\s*\|[^|]*\|[^|]*\|\s*([0-9.eE+]+)\s*\|", text, re.M)
    return float(m.group(2)) if m and m.group(1) == shape else None


def shape_names(lbfs, precision: str, in_use: tuple) -> dict:
    return {"stage": lbfs.shape_name(lbfs.tile_shapes("stage", precision)[in_use[0]]),
            "mag": lbfs.shape_name(lbfs.mag_shape(in_use[1], precision))}


def cpu_baseline(prob: dict, budget_s: float, solver=None) -> dict:
    """The FP64 oracle on one host thread over about budget_s of steps of the same
    workload. Grids above 1024^2 start from the solver's current state instead of the
    oracle's own initialisation, whose converged magnetic solve alone would take many
    minutes there; one step of 4096^2 takes about half a minute."""
    from oracle import oracle as orc
    p64 = dict(prob, precision="fp64", init_tol=1e-9)
    cells = prob["nx"] * prob["ny"]
    large = solver is not None and cells > 1024 * 1024
    print(f"bench: timing the FP64 oracle on the host ({prob['nx']}x{prob['ny']})", file=sys.stderr, flush=True)
    if large:
        o = orc.Oracle(dict(p64, init_max=0), init=False)
        o.set_state({k: solver.get(k) for k in ("He", "p", "Mx", "My", "C", "phi", "S")})
    else:
        o = orc.Oracle(p64)
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter()
    n = max(0, int(budget_s / max(t1 - t0, 1e-6)) - 1)   # (none more when one step used the budget)
    t2 = time.perf_counter()
    if n:
        o.step(n)
    t3 = time.perf_counter()
    steps = n + 1
    secs = (t1 - t0) + (t3 - t2)
    start = "the GPU solver's state after the timed steps" if large else "its initial state"
    return {"value": cells * steps / secs / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of the {prob['nx']}x{prob['ny']} droplet from {start}, "
                      f"FP64, single thread, {secs:.1f} s (init excluded)",
            "host": host_cpu()}


def host_cpu() -> dict:
    """The host's CPU model and the logical CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        ncpu = os.cpu_count()
    return {"cpu_model": model, "logical_cpus_available": ncpu}


def kernel_shape(kernel: str, shapes: dict) -> str:
    """Shape of one kernel kind: stages 2 and 3 always load the owned cells late, so the
    early-load mark of a stage shape applies to stages 0 and 1 only."""
    if kernel == "mag":
        return shapes["mag"]
    return shapes["stage"] if kernel in ("stage0", "stage1") else shapes["stage"].rstrip("e")


def error_vs_oracle(solver, prob: dict) -> dict:
    """One step of the GPU path against one step of the FP64 oracle from the same state
    (the solver's own current state, read back): relative L2 error per field, with the
    floors of near-zero fields (He ~ L, C ~ 1, phi ~ H0 R, p ~ sigma/R, momentum ~
    rho_l cs^2 sigma / mu_l)."""
    import numpy as np
    from oracle import oracle as orc
    names = ("He", "p", "Mx", "My", "C", "phi", "S")
    state = {k: solver.get(k) for k in names}
    t0 = solver.observe()["t"]
    o = orc.Oracle(dict(prob, precision="fp64", init_max=0), init=False)
    o.set_state(state)
    solver.set_state(state)          # the same values in the solver's own precision
    o.step(1)
    solver.step(1)
    p = o.params
    R = prob["drop"][2]
    floor = dict(He=p.latent, p=p.sigma / R, Mx=p.rho[1] / 3.0 * p.sigma / p.mu[1],
                 My=p.rho[1] / 3.0 * p.sigma / p.mu[1], C=1.0, phi=max(p.h0 * R, 1e-30))
    err = {}
    for k in ("He", "p", "Mx", "My", "C", "phi"):
        a, b = solver.get(k), o.get(k)
        err[k] = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), floor[k] * np.sqrt(b.size)))
    return {"per_step_rel_l2": err, "max": max(err.values()), "bound": 1e-5 if prob["precision"] == "fp32" else 1e-10,
            "state": f"the solver's state at t = {t0:g} after the timed steps"}


def host_boundary(solver, lbfs, cells: int, n: int) -> dict:
    """Rates with host traffic over PCIe inside the loop (never the headline value): each
    step followed by lbfs_observe (FP64 reductions, the observables struct to the host,
    as the serving loop does between chunks), and each step followed by lbfs_save_state
    (the whole state to a host buffer, a checkpoint every step)."""
    import ctypes as C
    lib = lbfs.lib()
    nb = int(lib.lbfs_checkpoint_bytes(solver._h))
    buf = C.create_string_buffer(nb)
    solver.step(1)
    solver.observe()
    t0 = time.perf_counter()
    for _ in range(n):
        solver.step(1)
        solver.observe()
    t1 = time.perf_counter()
    lbfs._check(lib.lbfs_save_state(solver._h, buf, nb), "lbfs_save_state")
    t2 = time.perf_counter()
    for _ in range(n):
        solver.step(1)
        lbfs._check(lib.lbfs_save_state(solver._h, buf, nb), "lbfs_save_state")
    t3 = time.perf_counter()
    return {"observe_each_step_mlups": cells * n / (t1 - t0) / 1e6,
            "checkpoint_each_step_mlups": cells * n / (t3 - t2) / 1e6,
            "checkpoint_bytes": nb, "steps": n,
            "note": "before the warm-up, outside the timed region; the timed value keeps the state resident"}


def freezing_fp32_vs_fp64(lbfs, wl, prob: dict) -> dict:
    """The workload solved to freezing (liquid fraction below 1e-3) in FP32 and in FP64 on
    the GPU; the FP64 path is held to the oracle at rounding level by the parity tests.
    FP64 is stepped in chunks of 2000 with a checkpoint before each, then one step at a
    time from the last checkpoint; FP32 is stepped to 99% of the FP64 step, then one step
    at a time."""
    def exact(s, start, cap):
        step = start
        fl = s.observe()["liquid_fraction"]
        while fl >= 1e-3 and step < cap:
            s.step(1)
            step += 1
            fl = s.observe()["liquid_fraction"]
        return step
    t0 = time.perf_counter()
    # chunks of about a hundredth of the freezing time (which grows as R^2)
    chunk = 2000 * max(1, prob["nx"] // 256) ** 2
    s64 = lbfs.Solver(wl.with_changes(prob, precision="fp64", init_tol=1e-9))
    step, blob = 0, s64.save()
    while s64.observe()["liquid_fraction"] >= 1e-3 and step < 500 * chunk:
        blob = s64.save()
        s64.step(chunk)
        step += chunk
        print(f"bench: freezing check, FP64 step {step}", file=sys.stderr, flush=True)
    s64.load(blob)
    n64 = exact(s64, max(0, step - chunk), step + 1)
    s64.close()
    s32 = lbfs.Solver(prob)
    start, step = int(0.99 * n64), 0
    while step < start:
        k = min(chunk, start - step)
        s32.step(k)
        step += k
        s32.observe()
        print(f"bench: freezing check, FP32 step {step}", file=sys.stderr, flush=True)
    n32 = exact(s32, start, int(1.02 * n64))
    s32.close()
    # the FP64 path's own throughput on the same workload (graph replays, state resident)
    p64 = lbfs.Solver(wl.with_changes(prob, precision="fp64", init_tol=1e-9))
    p64.step(200)
    p64.observe()
    n = 2000
    t1 = time.perf_counter()
    p64.step(n)
    p64.observe()
    t2 = time.perf_counter()
    p64.close()
    return {"fp32_freeze_step": n32, "fp64_freeze_step": n64, "rel_diff": abs(n32 - n64) / n64, "bound": 0.005,
            "fp64_mlups": prob["nx"] * prob["ny"] * n / (t2 - t1) / 1e6,
            "seconds": time.perf_counter() - t0}


def roofline(kern: dict, cells: int, precision: str, workload: str, shapes: dict, mag_flops=None,
             mag_launches: int = 1, exclude=()) -> dict:
    """Roofline of the kernel kind with the largest mean duration per step. The magnetic
    phase streams its fields once per launch (mag_launches per step). Kinds in `exclude`
    (a multigrid magnetic phase, many small launches with no algorithmic count) are not
    candidates."""
    share = {k: kern[k][0] for k in kern if k not in exclude}
    dominant = max(share, key=share.get)
    esize = 8 if precision == "fp64" else 4
    accesses = dict(FIELD_ACCESSES, mag=FIELD_ACCESSES["mag"] * mag_launches)
    alg_bytes = accesses[dominant] * esize * cells
    flops = dict(ALG_FLOPS, **({"mag": mag_flops} if mag_flops is not None else {}))
    alg_flops = flops[dominant] * cells
    dur_s = kern[dominant][0] * 1e-3
    gbs = alg_bytes / dur_s / 1e9
    tflops = alg_flops / dur_s / 1e12
    traffic = measured_traffic(dominant, workload, kernel_shape(dominant, shapes))
    hbm = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": gbs / HBM_PEAK_GBS, "traffic": traffic, "algorithmic_bytes_per_launch": alg_bytes}
    vpeak = VALU_PEAK_TFLOPS[precision]
    alu = {"bound": "alu", "achieved": tflops, "peak": vpeak, "unit": "TFLOP/s", "frac": tflops / vpeak,
           "traffic": traffic, "algorithmic_flops_per_launch": alg_flops,
           "frac_of_nonpacked_peak": tflops / VALU_PEAK_NONPACKED_TFLOPS}
    roof = dict(alu if BOUND[dominant] == "alu" else hbm)
    roof.update({"kernel": dominant, "tile_shape": kernel_shape(dominant, shapes),
                 "mean_launch_us": kern[dominant][0] * 1e3,
                 "timed_launches": kern[dominant][1],
                 "other_ceiling": hbm if BOUND[dominant] == "alu" else alu})
    return roof


def kernel_fields(kern: dict) -> dict:
    share = {k: kern[k][0] for k in kern}
    total = sum(share.values()) or 1.0
    return {"kernels_us": {k: round(v[0] * 1e3, 3) for k, v in kern.items()},
            "step_share": {k: round(v / total, 4) for k, v in share.items()}}


def line(args, value, unit, ms_per_step, dtype, config, higher=True) -> dict:
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": higher,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def copy_calibration(torch, mib: int) -> None:
    if mib <= 0:
        return
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def run_single(args, torch, lbfs, wl) -> dict:
    prob = {"droplet64": wl.droplet64, "droplet256": wl.droplet256, "droplet1024": lambda: wl.droplet1024("fp32"),
            "droplet1024-fp64": lambda: wl.droplet1024("fp64"), "droplet4096": wl.droplet4096}[args.workload]()
    if args.mag_method != "sweeps" or args.mag_steps is not None or args.mag_max_iters > 0:
        prob = wl.with_changes(prob, mag_method=args.mag_method,
                               sweeps=prob["sweeps"] if args.mag_steps is None else args.mag_steps,
                               mag_max_iters=args.mag_max_iters, mag_tol=args.mag_tol)
        prob["name"] += f"-mag-{args.mag_method}{prob['sweeps']}"
        if args.mag_max_iters > 0:
            prob["name"] += f"-upto{args.mag_max_iters}-tol{args.mag_tol:g}"
    # per step, at the fixed count (with convergence control, at the most chunks)
    iters = max(prob["sweeps"], args.mag_max_iters)
    base, per = ALG_FLOPS_MAG_LBFS if args.mag_method == "lbfs" else ALG_FLOPS_MAG_SWEEPS
    mag_flops = base + per * iters
    # launches of the magnetic phase: up to 4 sweeps or 4 pseudo-steps each, times the
    # chunks of the convergence control (an upper bound: converged chunks only copy)
    kmax = 4
    chunks = -(-args.mag_max_iters // max(1, prob["sweeps"])) if args.mag_max_iters > 0 else 1
    mag_launches = max(1, -(-prob["sweeps"] // kmax)) * chunks
    cells = prob["nx"] * prob["ny"]
    copy_calibration(torch, args.copy_calibration_mib)
    solver = lbfs.Solver(prob, device="cuda:0")
    if args.mag_in_stage1 != "auto":
        si, mi = solver.tile_shapes_in_use()
        fused = lbfs.mag_fused_index(prob["precision"])
        solver.set_tile_shapes(si, fused if args.mag_in_stage1 == "on" else (mi if mi != fused else 0))
    if args.tile_shapes:
        solver.set_tile_shapes(*(int(v) for v in args.tile_shapes.split(",")))
        tuned = None
    else:
        tuned = solver.autotune() if args.autotune == "on" else None
    shapes = shape_names(lbfs, prob["precision"], solver.tile_shapes_in_use())
    host_io = None if args.no_host_io else host_boundary(solver, lbfs, cells, max(5, min(200, args.steps // 10)))
    solver.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern = solver.step_profiled(args.steps, args.sample_every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    obs = solver.observe()
    secs = t1 - t0
    out = line(args, cells * args.steps / secs / 1e6, "MLUPS", secs * 1e3 / args.steps,
               "f64" if prob["precision"] == "fp64" else "f32",
               {"workload": prob["name"], "nx": prob["nx"], "ny": prob["ny"], "precision": prob["precision"],
                "angle_deg": prob["angle_deg"], "bo_m": prob["bo_m"], "ste": prob["ste"],
                "mag_method": prob.get("mag_method", "sweeps"),
                "mag_max_iters": prob.get("mag_max_iters", 0), "mag_tol": prob.get("mag_tol", 0.0),
                "sweeps_per_step": prob["sweeps"], "reductions": "f64",
                "tile_shapes": dict(shapes, chosen_by="autotuner" if tuned else
                                    ("given" if args.tile_shapes else "default"))})
    profile_key = args.workload + ("-mag-lbfs" if args.mag_method == "lbfs" else "")
    out["roofline"] = roofline(kern, cells, prob["precision"], profile_key, shapes, mag_flops, mag_launches,
                               exclude=("mag",) if args.mag_method == "multigrid" else ())
    out.update(kernel_fields(kern))
    if tuned:
        out["autotune"] = tuned
    out["liquid_fraction_reached"] = obs["liquid_fraction"]
    out["mag_residual_after_last_step"] = obs["mag_residual"]
    if host_io is not None:
        out["host_boundary"] = host_io
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds, solver)
        if cells <= 1024 * 1024:
            out["error_vs_oracle"] = error_vs_oracle(solver, prob)
        if args.workload == "droplet256" and args.mag_method == "sweeps" and not args.no_freeze_check:
            out["freezing_fp32_vs_fp64"] = freezing_fp32_vs_fp64(lbfs, wl, prob)
    if args.freeze_check and "freezing_fp32_vs_fp64" not in out:
        out["freezing_fp32_vs_fp64"] = freezing_fp32_vs_fp64(lbfs, wl, prob)
    return out


def run_batch(args, torch, lbfs, wl) -> dict:
    probs = wl.batch64()
    cells = sum(p["nx"] * p["ny"] for p in probs)
    budget = sum(lbfs.Batch.instance_bytes(p) for p in probs) + (64 << 20)
    copy_calibration(torch, args.copy_calibration_mib)
    batch = lbfs.Batch(len(probs), budget, precision="fp32", sweeps=probs[0]["sweeps"], omega=probs[0]["omega"])
    for p in probs:
        if batch.admit(p) is None:
            raise RuntimeError("the batch buffer is too small for the workload")
    if args.tile_shapes:
        batch.set_tile_shapes(*(int(v) for v in args.tile_shapes.split(",")))
        tuned = None
    else:
        tuned = batch.autotune(reps=10) if args.autotune in ("auto", "on") else None
    shapes = shape_names(lbfs, "fp32", batch.tile_shapes_in_use())
    batch.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern = batch.step_profiled(args.steps, args.sample_every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    obs = batch.observe()
    secs = t1 - t0
    fl = [o["liquid_fraction"] for o in obs.values()]
    out = line(args, cells * args.steps / secs / 1e6, "MLUPS", secs * 1e3 / args.steps, "f32",
               {"workload": f"batch of {len(probs)} droplets, edges 64-256 (seed 1), FP32", "instances": len(probs),
                "cells": cells, "edges": sorted({p["nx"] for p in probs}), "precision": "fp32",
                "sweeps_per_step": probs[0]["sweeps"], "reductions": "f64",
                "tile_shapes": dict(shapes, chosen_by="autotuner" if tuned else ("given" if args.tile_shapes else "default")),
                "launches_per_step": "one graph replay"})
    out["roofline"] = roofline(kern, cells, "fp32", args.workload, shapes)
    out.update(kernel_fields(kern))
    if tuned:
        out["autotune"] = tuned
    out["liquid_fraction_range"] = [min(fl), max(fl)]
    if not args.no_cpu_baseline:
        # the oracle on one instance of the mix (the largest edge), per-cell rate
        big = max(probs, key=lambda p: p["nx"] * p["ny"])
        out["cpu_baseline"] = cpu_baseline(big, args.cpu_seconds)
    return out


def run_serve(args, torch, lbfs, wl) -> dict:
    from paper_2511_10257_amd import serve
    edges = tuple(int(e) for e in args.serve_edges.split(","))
    stream = wl.request_stream(rate_hz=args.serve_rate, horizon_s=args.serve_seconds, edges=edges)
    budget = int(args.serve_budget_gib * (1 << 30))
    cap = args.serve_seconds + args.serve_drain
    srv = serve.Server(budget, max_slots=args.serve_slots, precision="fp32", chunk=args.serve_chunk)
    rep = srv.run(stream, clock="wall", horizon=args.serve_seconds, cap=cap, progress_every=20.0)
    srv.close()
    out = line(args, rep["solves_per_unit"], "solves/s", None, "f32",
               {"workload": f"Poisson stream {args.serve_rate:g}/s for {args.serve_seconds:g} s (seed 2), edges "
                            f"{args.serve_edges}, run to liquid fraction < 1e-3, FP32 continuous batching",
                "edges": list(edges), "rate_per_s": args.serve_rate,
                "slots": args.serve_slots, "budget_gib": args.serve_budget_gib, "chunk_steps": args.serve_chunk,
                "drain_cap_s": args.serve_drain})
    out["serve"] = rep
    if not args.no_serve_baseline:
        base = serve.Server(budget, max_slots=1, precision="fp64", chunk=args.serve_chunk)
        rb = base.run(stream, clock="wall", horizon=args.serve_seconds, cap=cap, progress_every=20.0)
        base.close()
        out["serve_fp64_one_at_a_time"] = rb
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the library runs each "
              f"solve or batch on a single MI355X, and sharding across GPUs exists as a design only",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2511_10257_amd import lbfs, workloads as wl

    if args.workload == "batch64":
        out = run_batch(args, torch, lbfs, wl)
    elif args.workload == "serve":
        out = run_serve(args, torch, lbfs, wl)
    else:
        out = run_single(args, torch, lbfs, wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
