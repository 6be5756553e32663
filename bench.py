"""Benchmark of the coupled LBFS time step on one MI355X.

Workload (default): the 256 x 256 freezing droplet (radius 64, Ste 0.1, field angle
0 or 90 deg and magnetic Bond number ~ U[0, 2] drawn with seed 0), FP32 fields with
FP64 reductions, 4 red-black sweeps per step. One "step" is the whole hot path: the
magnetic sweeps and residual, three fused Runge-Kutta stages with the Kelvin force,
the end-of-step Eq. 8 update and the FP64 reductions.

Prints one JSON line: throughput in MLUPS (cell updates per second / 1e6) with the
state resident in HBM, the roofline of the dominant kernel (its mean launch duration
from HIP events recorded on the solver's stream inside the timed region), and the
FP64 CPU oracle timed on a bounded sample of the same workload on the host.
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
# the resource that bounds each kernel: the sweeps stream fields with little arithmetic,
# the stages are far above the ridge point (68 FLOP/B against 19.7 FP32 / 9.8 FP64)
BOUND = {"mag": "hbm", "stage1": "alu", "stage2": "alu", "stage3": "alu", "reduce": "hbm"}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="config1", choices=["config0", "config1", "config2", "config2-fp64"])
    ap.add_argument("--sample-every", type=int, default=20,
                    help="bracket the kernels of every n-th timed step with HIP events")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run a plain device copy of this size (HBM counter calibration)")
    return ap.parse_args()


def kernel_sources_digest() -> str:
    h = hashlib.sha256()
    for name in ("lbfs_kernels.hip", "lbfs_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2511_10257_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_sources_sha256_16:\s*([0-9a-f]+)", text)
    if not m or m.group(1) != kernel_sources_digest():
        return None
    m = re.search(rf"^\|\s*{kernel}\s*\|[^|]*\|[^|]*\|\s*([0-9.eE+]+)\s*\|", text, re.M)
    return float(m.group(1)) if m else None


def cpu_baseline(prob: dict, budget_s: float) -> dict:
    from oracle import oracle as orc
    p64 = dict(prob, precision="fp64", init_tol=1e-9)
    o = orc.Oracle(p64)
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter()
    n = max(1, int(budget_s / max(t1 - t0, 1e-6)) - 1)
    t2 = time.perf_counter()
    o.step(n)
    t3 = time.perf_counter()
    steps = n + 1
    secs = (t1 - t0) + (t3 - t2)
    cells = prob["nx"] * prob["ny"]
    return {"value": cells * steps / secs / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of the {prob['nx']}x{prob['ny']} droplet from its initial state, "
                      f"FP64, single thread, {secs:.1f} s (init excluded)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (this build runs on a "
              f"single MI355X; see the multi-GPU design notes)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2511_10257_amd import lbfs, workloads as wl

    if args.workload == "config0":
        prob = wl.config0()
    elif args.workload == "config1":
        prob = wl.config1()
    elif args.workload == "config2":
        prob = wl.config2("fp32")
    else:
        prob = wl.config2("fp64")
    nx, ny = prob["nx"], prob["ny"]
    cells = nx * ny
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    solver = lbfs.Solver(prob, device="cuda:0")
    solver.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern = solver.step_profiled(args.steps, args.sample_every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    obs = solver.observe()
    secs = t1 - t0
    mlups = cells * args.steps / secs / 1e6

    share = {k: kern[k][0] for k in kern}
    dominant = max(share, key=share.get)
    esize = 8 if prob["precision"] == "fp64" else 4
    alg_bytes = FIELD_ACCESSES[dominant] * esize * cells
    alg_flops = ALG_FLOPS[dominant] * cells
    dur_s = kern[dominant][0] * 1e-3
    gbs = alg_bytes / dur_s / 1e9
    tflops = alg_flops / dur_s / 1e12
    traffic = measured_traffic(dominant, args.workload)
    hbm = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": gbs / HBM_PEAK_GBS, "traffic": traffic, "algorithmic_bytes_per_launch": alg_bytes}
    vpeak = VALU_PEAK_TFLOPS[prob["precision"]]
    alu = {"bound": "alu", "achieved": tflops, "peak": vpeak, "unit": "TFLOP/s", "frac": tflops / vpeak,
           "traffic": traffic, "algorithmic_flops_per_launch": alg_flops,
           "frac_of_nonpacked_peak": tflops / VALU_PEAK_NONPACKED_TFLOPS}
    roof = dict(alu if BOUND[dominant] == "alu" else hbm)
    roof.update({"kernel": dominant, "mean_launch_us": kern[dominant][0] * 1e3,
                 "timed_launches": kern[dominant][1],
                 "other_ceiling": hbm if BOUND[dominant] == "alu" else alu})

    line = {
        "metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": secs * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prob["precision"] == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": prob["name"], "nx": nx, "ny": ny, "precision": prob["precision"],
                   "angle_deg": prob["angle_deg"], "bo_m": prob["bo_m"], "ste": prob["ste"],
                   "sweeps_per_step": prob["sweeps"], "reductions": "f64"},
        "roofline": roof,
        "kernels_us": {k: round(v[0] * 1e3, 3) for k, v in kern.items()},
        "step_share": {k: round(v / sum(share.values()), 4) for k, v in share.items()},
        "liquid_fraction_reached": obs["liquid_fraction"],
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
