"""Benchmark of the coupled LBFS time step on one MI355X.

Workload (default): the 1024 x 1024 freezing droplet (radius 256, horizontal field,
magnetic Bond number 1.5, density ratio 100, Ste 0.1, 4 red-black sweeps per step), the
configuration on which the roofline of the fused flux and update kernels is measured.
One "step" is the whole hot path: the magnetic sweeps and residual, three fused
Runge-Kutta stages with the Kelvin force, and the end-of-step Eq. 8 update with the
lagged dFs/dt. The FP64 observables (liquid fraction, volume, max |u|) are reduced only
when they are read, Table 1's "if output required" branch, and are not part of the
timed step. The FP32 path keeps the order parameter in FP64.

The line times FP32 (the value) and FP64 on the same workload, each with its per-step
error against the FP64 oracle; it adds a bounded serving run (continuous batching in
FP32 against the plain FP64 per-solve path), the FP32 against FP64 freezing time of the
256 x 256 droplet, and the oracle timed on the host (one thread, and all cores).

Other workloads: droplet64 (64 x 64, FP64), droplet256 (256 x 256, FP32), droplet1024-fp64,
droplet4096 (HBM-resident), batch64 (64 uneven instances advanced by the same launches)
and serve (the Poisson stream of requests, FP32 continuous batching beside the same
stream served one solve at a time in FP64).

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
import math
import multiprocessing as mp
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

# Algorithmic work and traffic per cell and launch, from an operation count of the
# definitional algorithm: about 780 FLOP per face for the nine
# surrounding equilibria, the Eq. 45 face state, the star distributions and the moments,
# two faces per cell, plus about 250 of cell work, i.e. about 1.8k per cell and stage
# (5.5k per cell-step); the magnetic phase about 1 % of a step. Bytes: one 4-byte FP32
# value per field access with perfect on-chip reuse (12, 17, 18 accesses for stages
# 1-3: W, the stage input, phi', S in and the stage output; 13 for the magnetic phase:
# mu written, and phi, mu read and phi written by each of 4 sweeps); FP64 doubles them.
ALG_FLOPS = {"mag": 55.0, "stage1": 1800.0, "stage2": 1800.0, "stage3": 1800.0, "reduce": 0.0}
ALG_BYTES_FP32 = {"mag": 52.0, "stage1": 48.0, "stage2": 68.0, "stage3": 72.0, "reduce": 0.0}
# The bytes these kernels have to move at the least (each field once, the order
# parameter in FP64 in both precisions; stage 1 also writes the step's Kelvin force and
# step-start liquid fraction, which stages 2 and 3 read instead of the potential; stage 3
# also writes the permeability of the new state, which the sweeps read instead of He and
# C): FP32 and FP64
MIN_BYTES = {"fp32": {"mag": 12.0, "stage1": 68.0, "stage2": 84.0, "stage3": 96.0, "reduce": 0.0},
             "fp64": {"mag": 24.0, "stage1": 120.0, "stage2": 144.0, "stage3": 168.0, "reduce": 0.0}}
# a magnetic phase that computes the permeability from He and C (the pseudo-time solve)
MIN_BYTES_MAG_FROM_STATE = {"fp32": 20.0, "fp64": 32.0}


def min_bytes(precision: str, kind: str, workload: str = "") -> float:
    """Least bytes per cell of one launch of `kind` (MIN_BYTES), for the magnetic phase
    of a workload whose name ends in -mag-lbfs the figure with He and C read."""
    if kind == "mag" and workload.endswith("-mag-lbfs"):
        return MIN_BYTES_MAG_FROM_STATE[precision]
    return MIN_BYTES[precision][kind]
# The operation count of the oracle's literal per-face procedure (nine equilibria of
# each kind built point by point), measured by compiling the oracle with a counting
# number type (oracle/opcount.py) on the 256 x 256 droplet: 13993 per cell-step, of which
# the magnetic phase (permeability, 4 sweeps, residual) takes 152.7 and each stage
# 4613.4; reported beside the roofline, never as its figure
ORACLE_OPCOUNT = {"mag": 152.7, "stage1": 4613.4, "stage2": 4613.4, "stage3": 4613.4, "reduce": 0.0}
# the magnetic phase by the LBFS pseudo-time solve, counted the same way on the oracle's
# literal m* construction: 51.8 per cell for the permeability and residual plus 1682.5
# per cell and pseudo-step (the kernel evaluates the exact reduction of that
# construction at delta_t = dx/2, about 45 operations per cell and pseudo-step)
ALG_FLOPS_MAG_LBFS = (51.8, 1682.5)
# and by the sweeps: 51.8 per cell for the permeability and residual, 25.2 per sweep
ALG_FLOPS_MAG_SWEEPS = (51.8, 25.23)
# the resource that bounds each kernel: the sweeps stream fields with little arithmetic,
# the stages lie above the ridge point (1800/68 = 26 FLOP/B against 19.7 FP32 / 9.8 FP64)
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
    ap.add_argument("--workload", default="droplet1024",
                    choices=["droplet64", "droplet256", "droplet1024", "droplet1024-fp64", "droplet4096", "batch64",
                             "serve"])
    ap.add_argument("--sample-every", type=int, default=None,
                    help="bracket the kernels of every n-th timed step with HIP events (default: 97, "
                         "the 96 steps between two sampled ones running as six 16-step graph replays on "
                         "grids under 2^19 cells and as direct launches on larger ones, "
                         "or fewer, so that at least three steps are sampled)")
    ap.add_argument("--settle-seconds", type=float, default=1.0,
                    help="untimed steps for about this long before the warm-up, so that the GPU runs at its "
                         "sustained clock when the timed steps begin (a few milliseconds of steps after an "
                         "idle period run about 10%% slower)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle sample")
    ap.add_argument("--cpu-all-seconds", type=float, default=10.0,
                    help="budget of the all-core oracle runs (one single-thread oracle per CPU)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true",
                    help="droplet1024: skip the FP64 path beside the FP32 one")
    ap.add_argument("--no-serve-leg", action="store_true",
                    help="droplet1024: skip the bounded serving run (FP32 continuous batching against "
                         "FP64 one solve at a time, about 80 s)")
    ap.add_argument("--serve-leg-seconds", type=float, default=30.0,
                    help="arrivals of the bounded serving run (the sustainable variant)")
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
    if args.sample_every is None:
        args.sample_every = sample_every_for(args.steps)
    return args


def sample_every_for(steps: int) -> int:
    """97 (six 16-step graph replays between sampled steps on small grids), or fewer so that at least
    three of the timed steps are sampled."""
    return max(1, min(97, -(-steps // 3)))


def _code_only(src: str) -> str:
    """C++ source without its comments and with runs of white space made one space (the
    sources hold no string literal with comment markers)."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_sources_digest() -> str:
    """Hash of the code the kernels are built from: the kernel sources without their
    comments, and the build script (its compiler flags shape the kernels too)."""
    h = hashlib.sha256()
    for name in ("csrc/lbfs_kernels.hip", "csrc/lbfs_face.hpp", "csrc/lbfs_internal.hpp", "build.py"):
        with open(os.path.join(ROOT, "paper_2511_10257_amd", name), encoding="utf-8") as f:
            text = f.read()
        h.update((text if name.endswith(".py") else _code_only(text)).encode())
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
    workload. Grids of 512^2 and up start from the solver's current state instead of
    the oracle's own initialisation, whose converged magnetic solve alone would take
    minutes there; one step of 4096^2 takes about half a minute."""
    from oracle import oracle as orc
    p64 = dict(prob, precision="fp64", init_tol=1e-9)
    cells = prob["nx"] * prob["ny"]
    large = solver is not None and cells >= 512 * 512
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


def _oracle_worker(args):
    """One single-thread FP64 oracle process: steps its share of the problems round
    robin, one step each, until the budget is spent; returns (cell updates, seconds)."""
    probs, budget = args
    from oracle import oracle as orc
    sims = [(orc.Oracle(dict(p, precision="fp64", init_max=0)), p["nx"] * p["ny"]) for p in probs]
    done, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget:
        for o, n in sims:
            o.step(1)
            done += n
    return done, time.perf_counter() - t0


def cpu_cores() -> int:
    """Host threads for the all-core oracle runs: the CPUs this process may use, at most
    16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def all_cores_rate(probs: list, budget_s: float, cores: int) -> dict:
    """Aggregate FP64 oracle rate of `cores` independent single-thread processes, each
    stepping its share of `probs` (initialised without the magnetic solve, whose cost
    is not a step's) for about budget_s."""
    shares = [probs[k::cores] for k in range(cores)]
    shares = [sh for sh in shares if sh]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(len(shares)) as pool:
        res = pool.map(_oracle_worker, [(sh, budget_s) for sh in shares])
    wall = time.perf_counter() - t0
    cells = sum(r[0] for r in res)
    slowest = max(r[1] for r in res)
    return {"value": cells / slowest / 1e6, "unit": "MLUPS", "cores": len(shares),
            "cell_updates": cells, "seconds": slowest, "wall_s_with_start": wall}


def all_cores_baseline(wl, budget_s: float, serve_edges=(96, 128)) -> dict:
    """The oracle on every host core (one single-thread solve per core) for the instance
    mixes of the 64-instance batch (edges 64-256) and of the bounded serving run (its edges). Runs
    before the GPU is touched. Solves/s of the serving mix follows from this rate and the
    cell updates a served request needed on the GPU (filled in after the serving run)."""
    cores = cpu_cores()
    print(f"bench: all-core oracle runs on {cores} host threads", file=sys.stderr, flush=True)
    batch = all_cores_rate(wl.batch64(), budget_s, cores)
    stream = wl.request_stream(rate_hz=9.0, horizon_s=60.0, edges=tuple(serve_edges))
    mix = [p for _, p in stream][: 4 * cores]
    serve = all_cores_rate(mix, budget_s, cores)
    return {"cores": cores, "kind": "oracle",
            "batch64": dict(batch, sample=f"the 64 instances of the batch (edges 64-256), round robin over "
                                         f"{batch['cores']} single-thread processes, {budget_s:g} s each"),
            "serve_mix": dict(serve, sample=f"{len(mix)} requests of the serving mix (edges "
                                            f"{','.join(map(str, serve_edges))}), {budget_s:g} s per process")}


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
    return shapes["stage"] if kernel in ("stage0", "stage1") else shapes["stage"].replace("e", "")


def error_vs_oracle(source, solvers: dict, prob: dict) -> dict:
    """One step of each GPU path against one step of the FP64 oracle, all from the same
    state (the source solver's current state, read back; each solver receives it in its
    own storage precision). Per field: the relative L2 error against the field's own
    norm (for the potential, its perturbation phi - phi0), and the same with the floors
    of the state's scales (He ~ L, C ~ 1, phi ~ H0 R, p ~ sigma/R, momentum ~
    rho_l cs^2 sigma / mu_l). The bound applies to the unfloored value."""
    import numpy as np
    from oracle import oracle as orc
    names = ("He", "p", "Mx", "My", "C", "phi", "S")
    state = {k: source.get(k) for k in names}
    obs = source.observe()
    o = orc.Oracle(dict(prob, precision="fp64", init_max=0), init=False)
    o.set_state(state)
    o.set_time(obs["t"], obs["step"])
    print(f"bench: one oracle step of the {prob['nx']}x{prob['ny']} state", file=sys.stderr, flush=True)
    o.step(1)
    p = o.params
    R = prob["drop"][2]
    th = math.radians(p.angle_deg)
    y, x = np.mgrid[0:p.ny, 0:p.nx] + 0.5
    phi0 = -p.h0 * (x * math.cos(th) + y * math.sin(th))
    ref = {k: o.get(k) for k in names}
    ref["phi"] = ref["phi"] - phi0
    m = p.rho[1] / 3.0 * p.sigma / p.mu[1]
    floor = dict(He=p.latent, p=p.sigma / R, Mx=m, My=m, C=1.0, phi=max(p.h0 * R, 1e-30))
    out = {}
    for prec, solver in solvers.items():
        solver.set_state(state)          # the same values in the solver's own precision
        solver.set_time(obs["t"], int(obs["step"]))
        solver.step(1)
        rel, floored = {}, {}
        for k in names:
            a = solver.get(k) - (phi0 if k == "phi" else 0.0)
            b = ref[k]
            d, nb = float(np.linalg.norm(a - b)), float(np.linalg.norm(b))
            rel[k] = d / nb if nb > 0 else d
            if k in floor:
                floored[k] = d / max(nb, floor[k] * math.sqrt(b.size))
        checked = [rel[k] for k in floor]
        out[prec] = {"per_step_rel_l2": rel, "max": max(checked), "per_step_rel_l2_floored": floored,
                     "bound": 1e-5 if prec == "fp32" else 1e-10,
                     "note": "bound on the unfloored error of He, p, Mx, My, C and phi - phi0; "
                             "S (a difference of liquid fractions) is reported only"}
    out["state"] = f"the FP32 solver's state at t = {obs['t']:g} after the timed steps"
    return out


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
    """Roofline of the kernel kind with the largest mean duration among the sampled
    steps. `achieved` is the algorithmic per-cell figure (ALG_FLOPS, or ALG_BYTES_FP32 times
    2 in FP64) times the cells of one launch over the mean launch duration; the bound is
    the kernel's (ALU for the stages, HBM for the magnetic phase), the other ceiling is
    given beside it. A magnetic phase of other than 4 sweeps (mag_launches launches per
    step, the definitional count mag_flops) scales the magnetic figures. Kinds in
    `exclude` (a multigrid magnetic phase: many small launches with no per-cell figure)
    are not candidates."""
    share = {k: kern[k][0] for k in kern if k not in exclude and kern[k][1] > 0}
    dominant = max(share, key=share.get)
    scale = 2.0 if precision == "fp64" else 1.0
    alg_bytes = ALG_BYTES_FP32[dominant] * scale * cells
    least = min_bytes(precision, dominant, workload) * cells
    alg_flops = ALG_FLOPS[dominant] * cells
    if dominant == "mag" and (mag_flops is not None or mag_launches != 1):
        alg_bytes *= mag_launches
        least *= mag_launches
        alg_flops = (mag_flops if mag_flops is not None else ALG_FLOPS["mag"]) * cells
    dur_s = kern[dominant][0] * 1e-3
    gbs = alg_bytes / dur_s / 1e9
    tflops = alg_flops / dur_s / 1e12
    traffic = measured_traffic(dominant, workload, kernel_shape(dominant, shapes))
    hbm = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": gbs / HBM_PEAK_GBS, "traffic": traffic, "algorithmic_bytes_per_launch": alg_bytes,
           "min_bytes_per_launch": least,
           "min_bytes_frac": least / dur_s / 1e9 / HBM_PEAK_GBS}
    vpeak = VALU_PEAK_TFLOPS[precision]
    alu = {"bound": "alu", "achieved": tflops, "peak": vpeak, "unit": "TFLOP/s", "frac": tflops / vpeak,
           "traffic": traffic, "algorithmic_flops_per_launch": alg_flops,
           "frac_of_nonpacked_peak": tflops / VALU_PEAK_NONPACKED_TFLOPS,
           "oracle_opcount_flops_per_launch": ORACLE_OPCOUNT[dominant] * cells,
           "oracle_opcount_tflops": ORACLE_OPCOUNT[dominant] * cells / dur_s / 1e12}
    roof = dict(alu if BOUND[dominant] == "alu" else hbm)
    roof.update({"kernel": dominant, "tile_shape": kernel_shape(dominant, shapes),
                 "mean_launch_us": kern[dominant][0] * 1e3,
                 "timed_launches": kern[dominant][1],
                 "figures": "algorithmic per-cell figures: 1.8k FLOP per cell and stage; 48/68/72 B per cell for "
                            "stages 1/2/3 and 52 B for 4 sweeps (FP32; x2 in FP64)",
                 "other_ceiling": hbm if BOUND[dominant] == "alu" else alu})
    return roof


def measured_valu(workload: str) -> float | None:
    """Issued VALU lane-operations per cell and stage (mean of the three stage kernels)
    from the committed rocprofv3 counter summary, if it was taken on the current kernel
    sources."""
    path = os.path.join(ROOT, "profiles", f"valu_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_sources_sha256_16:\s*([0-9a-f]+)", text)
    if not m or m.group(1) != kernel_sources_digest():
        return None
    vals = [float(x) for x in re.findall(r"^\|\s*stage[123]\s*\|[^|]*\|[^|]*\|[^|]*\|\s*([0-9.]+)\s*\|", text, re.M)]
    return sum(vals) / len(vals) if vals else None


def whole_step(cells: int, precision: str, ms_per_step: float, workload: str) -> dict:
    """The whole step against the HBM peak: the algorithmic bytes per cell-step (63 field
    accesses of 4 B with perfect on-chip reuse; 8 B in FP64) and the least bytes of this
    layout (each kernel's fields once, the order parameter in FP64), over the measured
    time per step; and the issued VALU lane-operations per cell and stage when a counter
    summary of the current kernels exists."""
    scale = 2.0 if precision == "fp64" else 1.0
    alg = sum(ALG_BYTES_FP32.values()) * scale
    least = sum(min_bytes(precision, k, workload) for k in MIN_BYTES[precision])
    step_s = ms_per_step * 1e-3
    return {"algorithmic_bytes_per_cell_step": alg, "least_bytes_per_cell_step": least,
            "hbm_frac_algorithmic_bytes": alg * cells / step_s / 1e9 / HBM_PEAK_GBS,
            "hbm_frac_least_bytes": least * cells / step_s / 1e9 / HBM_PEAK_GBS,
            "issued_valu_lane_ops_per_cell_stage": measured_valu(workload) if precision == "fp32" else None,
            "algorithmic_flop_per_cell_stage": ALG_FLOPS["stage1"]}


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


def settle(args, torch, stepper) -> int:
    """Untimed steps (16 at a time) for about args.settle_seconds; returns their count."""
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < args.settle_seconds:
        stepper.step(16)
        n += 16
        if n % 256 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    return n


def timed_steps(args, torch, solver) -> tuple:
    """Capture every step graph, settle the clock, run the warm-up steps, then time
    exactly args.steps steps (kernels of every sample_every-th step bracketed by HIP
    events on the solver's stream), synchronised on both sides. Returns (kernel times,
    seconds, settle steps)."""
    solver.prepare()
    nsettle = settle(args, torch, solver)
    solver.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step_profiled_start(args.steps, args.sample_every)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    # (the sampled launches' event times are read after the clock stopped)
    return solver.profile_result(), secs, nsettle


def single_problem(args, wl, workload: str) -> tuple:
    prob = {"droplet64": wl.droplet64, "droplet256": wl.droplet256, "droplet1024": lambda: wl.droplet1024("fp32"),
            "droplet1024-fp64": lambda: wl.droplet1024("fp64"), "droplet4096": wl.droplet4096}[workload]()
    if args.mag_method != "sweeps" or args.mag_steps is not None or args.mag_max_iters > 0:
        prob = wl.with_changes(prob, mag_method=args.mag_method,
                               sweeps=prob["sweeps"] if args.mag_steps is None else args.mag_steps,
                               mag_max_iters=args.mag_max_iters, mag_tol=args.mag_tol)
        prob["name"] += f"-mag-{args.mag_method}{prob['sweeps']}"
        if args.mag_max_iters > 0:
            prob["name"] += f"-upto{args.mag_max_iters}-tol{args.mag_tol:g}"
    # per step, at the fixed count (with convergence control, at the most chunks)
    iters = max(prob["sweeps"], args.mag_max_iters)
    mag_flops = None
    if args.mag_method != "sweeps" or iters != 4:
        base, per = ALG_FLOPS_MAG_LBFS if args.mag_method == "lbfs" else ALG_FLOPS_MAG_SWEEPS
        mag_flops = base + per * iters
    # launches of the magnetic phase: up to 4 sweeps or 4 pseudo-steps each, times the
    # chunks of the convergence control (an upper bound: converged chunks only copy)
    kmax = 4
    chunks = -(-args.mag_max_iters // max(1, prob["sweeps"])) if args.mag_max_iters > 0 else 1
    mag_launches = max(1, -(-prob["sweeps"] // kmax)) * chunks
    return prob, mag_flops, mag_launches


def make_solver(args, lbfs, prob):
    solver = lbfs.Solver(prob, device="cuda:0")
    if args.mag_in_stage1 != "auto":
        si, mi = solver.tile_shapes_in_use()
        fused = lbfs.mag_fused_index(prob["precision"])
        solver.set_tile_shapes(si, fused if args.mag_in_stage1 == "on" else (mi if mi != fused else 0))
    tuned = None
    if args.tile_shapes:
        solver.set_tile_shapes(*(int(v) for v in args.tile_shapes.split(",")))
    elif args.autotune == "on":
        tuned = solver.autotune()
    return solver, tuned


def serving_leg(args, lbfs, wl, cpu_all: dict | None) -> dict:
    """The sustainable variant of the serving stream, bounded: Poisson arrivals at 9
    requests/s (about 80 % of the estimated FP32 capacity for these sizes) of droplets
    with edges 96 and 128 (seed 2, per-request angle, Bo_m and Ste), arrivals for
    --serve-leg-seconds, each solve to liquid fraction < 1e-3. FP32 continuous batching
    (up to 64 resident solves) against the plain FP64 path, one solve at a time; the
    hard cap after the last arrival is 30 s for the first and 15 s for the second."""
    from paper_2511_10257_amd import serve
    edges, rate, horizon = (96, 128), 9.0, args.serve_leg_seconds
    stream = wl.request_stream(rate_hz=rate, horizon_s=horizon, edges=edges)
    budget = 8 << 30
    print(f"bench: serving {len(stream)} requests in FP32 (continuous batching)", file=sys.stderr, flush=True)
    srv = serve.Server(budget, max_slots=64, precision="fp32", chunk=args.serve_chunk)
    rep32 = srv.run(stream, clock="wall", horizon=horizon, cap=horizon + 30.0, progress_every=10.0)
    srv.close()
    print("bench: the same stream in FP64, one solve at a time", file=sys.stderr, flush=True)
    base = serve.Server(budget, max_slots=1, precision="fp64", chunk=args.serve_chunk)
    rep64 = base.run(stream, clock="wall", horizon=horizon, cap=horizon + 15.0, progress_every=10.0)
    base.close()
    keys = ("requests", "completed", "unfinished", "solves_per_unit", "p50", "p99", "elapsed", "mlups",
            "cell_steps_per_completed", "nonfinite", "rejected")
    out = {"workload": f"Poisson stream {rate:g}/s for {horizon:g} s (seed 2), edges {edges[0]} and {edges[1]}, "
                       f"R = edge/4, each run to liquid fraction < 1e-3",
           "fp32_continuous_batching": {k: rep32.get(k) for k in keys},
           "fp64_one_at_a_time": {k: rep64.get(k) for k in keys},
           "units": "solves_per_unit in solves/s; p50, p99 and elapsed in s (arrival to result)"}
    if rep64["solves_per_unit"]:
        out["solves_per_s_ratio"] = rep32["solves_per_unit"] / rep64["solves_per_unit"]
    per_solve = rep32.get("cell_steps_per_completed")
    if cpu_all and per_solve:
        mix = cpu_all["serve_mix"]
        cpu_all["serve_mix"]["solves_per_s_estimate"] = mix["value"] * 1e6 / per_solve
        cpu_all["serve_mix"]["solves_per_s_note"] = (
            "all-core oracle rate on the mix over the cell updates a completed request needed in the FP32 "
            "serving run (the oracle finishes no such solve within the benchmark: one takes minutes)")
    return out


def run_single(args, torch, lbfs, wl, cpu_all=None) -> dict:
    prob, mag_flops, mag_launches = single_problem(args, wl, args.workload)
    cells = prob["nx"] * prob["ny"]
    copy_calibration(torch, args.copy_calibration_mib)
    solver, tuned = make_solver(args, lbfs, prob)
    shapes = shape_names(lbfs, prob["precision"], solver.tile_shapes_in_use())
    host_io = None if args.no_host_io else host_boundary(solver, lbfs, cells, max(5, min(200, args.steps // 10)))
    kern, secs, nsettle = timed_steps(args, torch, solver)
    obs = solver.observe()
    out = line(args, cells * args.steps / secs / 1e6, "MLUPS", secs * 1e3 / args.steps,
               "f64" if prob["precision"] == "fp64" else "f32",
               {"workload": prob["name"], "nx": prob["nx"], "ny": prob["ny"], "precision": prob["precision"],
                "angle_deg": prob["angle_deg"], "bo_m": prob["bo_m"], "ste": prob["ste"],
                "mag_method": prob.get("mag_method", "sweeps"),
                "mag_max_iters": prob.get("mag_max_iters", 0), "mag_tol": prob.get("mag_tol", 0.0),
                "sweeps_per_step": prob["sweeps"], "reductions": "f64 (when observed)",
                "order_parameter_storage": "f64",
                "timed_step": "magnetic phase, three Runge-Kutta stages, Eq. 8 and the lagged dFs/dt; the FP64 "
                              "observables are reduced when read, outside the timed steps",
                "sample_every": args.sample_every, "settle_steps": nsettle,
                "tile_shapes": dict(shapes, chosen_by="autotuner" if tuned else
                                    ("given" if args.tile_shapes else "default"))})
    profile_key = args.workload + ("-mag-lbfs" if args.mag_method == "lbfs" else "")
    out["roofline"] = roofline(kern, cells, prob["precision"], profile_key, shapes, mag_flops, mag_launches,
                               exclude=("mag",) if args.mag_method == "multigrid" else ())
    out["whole_step"] = whole_step(cells, prob["precision"], out["ms_per_step"], profile_key)
    out.update(kernel_fields(kern))
    if tuned:
        out["autotune"] = tuned
    out["liquid_fraction_reached"] = obs["liquid_fraction"]
    out["mag_residual_after_last_step"] = obs["mag_residual"]
    if host_io is not None:
        out["host_boundary"] = host_io
    solvers = {prob["precision"]: solver}
    if args.workload == "droplet1024" and not args.no_fp64:
        # the FP64 path on the same workload, timed the same way
        p64, mf64, ml64 = single_problem(args, wl, "droplet1024-fp64")
        s64, _ = make_solver(args, lbfs, p64)
        sh64 = shape_names(lbfs, "fp64", s64.tile_shapes_in_use())
        k64, sec64, ns64 = timed_steps(args, torch, s64)
        v64 = cells * args.steps / sec64 / 1e6
        out["fp64"] = {"value": v64, "unit": "MLUPS", "ms_per_step": sec64 * 1e3 / args.steps,
                       "steps": args.steps, "warmup": args.warmup, "settle_steps": ns64, "workload": p64["name"],
                       "tile_shapes": sh64,
                       "roofline": roofline(k64, cells, "fp64", "droplet1024-fp64", sh64, mf64, ml64,
                                            exclude=("mag",) if args.mag_method == "multigrid" else ()),
                       **kernel_fields(k64)}
        out["fp32_over_fp64"] = out["value"] / v64
        solvers["fp64"] = s64
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds, solver)
        if cpu_all:
            out["cpu_baseline"]["all_cores"] = cpu_all
        if cells <= 1024 * 1024:
            out["error_vs_oracle"] = error_vs_oracle(solver, solvers, prob)
    if args.workload == "droplet1024" and not args.no_serve_leg:
        out["serving"] = serving_leg(args, lbfs, wl, cpu_all)
    if not args.no_cpu_baseline and not args.no_freeze_check and args.mag_method == "sweeps" and \
            args.workload in ("droplet256", "droplet1024"):
        # the freezing time of the 256^2 droplet (R = 64, seeded field) in FP32 and FP64 (about 10 s)
        p256 = wl.droplet256()
        fz = freezing_fp32_vs_fp64(lbfs, wl, p256)
        fz["workload"] = p256["name"]
        out["freezing_fp32_vs_fp64"] = fz
    if args.freeze_check and "freezing_fp32_vs_fp64" not in out:
        out["freezing_fp32_vs_fp64"] = freezing_fp32_vs_fp64(lbfs, wl, prob)
    return out


def run_batch(args, torch, lbfs, wl, cpu_all=None) -> dict:
    probs = wl.batch64()
    cells = sum(p["nx"] * p["ny"] for p in probs)
    budget = sum(lbfs.Batch.instance_bytes(p) for p in probs) + (64 << 20)
    copy_calibration(torch, args.copy_calibration_mib)
    batch = lbfs.Batch(len(probs), budget, precision="fp32", sweeps=probs[0]["sweeps"], omega=probs[0]["omega"])
    for p in probs:
        if batch.admit(p) is None:
            raise RuntimeError("the batch buffer is too small for the workload")
    nsettle = 0
    if args.tile_shapes:
        batch.set_tile_shapes(*(int(v) for v in args.tile_shapes.split(",")))
        tuned = None
    else:
        if args.autotune in ("auto", "on"):
            # (at the sustained clock: candidates timed while the clock still rises would
            # favour the later ones)
            nsettle += settle(args, torch, batch)
            tuned = batch.autotune(reps=10)
        else:
            tuned = None
    shapes = shape_names(lbfs, "fp32", batch.tile_shapes_in_use())
    batch.prepare()
    nsettle += settle(args, torch, batch)
    batch.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step_profiled_start(args.steps, args.sample_every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = batch.profile_result()
    obs = batch.observe()
    secs = t1 - t0
    fl = [o["liquid_fraction"] for o in obs.values()]
    out = line(args, cells * args.steps / secs / 1e6, "MLUPS", secs * 1e3 / args.steps, "f32",
               {"workload": f"batch of {len(probs)} droplets, edges 64-256 (seed 1), FP32", "instances": len(probs),
                "cells": cells, "edges": sorted({p["nx"] for p in probs}), "precision": "fp32",
                "sweeps_per_step": probs[0]["sweeps"], "reductions": "f64",
                "tile_shapes": dict(shapes, chosen_by="autotuner" if tuned else ("given" if args.tile_shapes else "default")),
                "launches_per_step": "one graph replay", "sample_every": args.sample_every,
                "settle_steps": nsettle})
    out["roofline"] = roofline(kern, cells, "fp32", args.workload, shapes)
    out["whole_step"] = whole_step(cells, "fp32", out["ms_per_step"], args.workload)
    out.update(kernel_fields(kern))
    if tuned:
        out["autotune"] = tuned
    out["liquid_fraction_range"] = [min(fl), max(fl)]
    if not args.no_cpu_baseline:
        # the oracle on one instance of the mix (the largest edge), per-cell rate
        big = max(probs, key=lambda p: p["nx"] * p["ny"])
        out["cpu_baseline"] = cpu_baseline(big, args.cpu_seconds)
        if cpu_all:
            out["cpu_baseline"]["all_cores"] = cpu_all
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
    from paper_2511_10257_amd import workloads as wl

    # the all-core oracle runs fork worker processes: before anything touches the GPU
    cpu_all = None
    if not args.no_cpu_baseline and args.workload in ("droplet1024", "batch64") and args.cpu_all_seconds > 0:
        cpu_all = all_cores_baseline(wl, args.cpu_all_seconds)
    import torch

    from paper_2511_10257_amd import lbfs

    if args.workload == "batch64":
        out = run_batch(args, torch, lbfs, wl, cpu_all)
    elif args.workload == "serve":
        out = run_serve(args, torch, lbfs, wl)
    else:
        out = run_single(args, torch, lbfs, wl, cpu_all)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
