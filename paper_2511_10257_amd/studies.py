"""Sec. 5 studies: freezing droplets swept over Bo_m, field orientation and Ste.

Every case of a sweep is one instance of a single device batch (lbfs_batch_*), so the
whole sweep advances with the same launches. Between chunks of steps one FP64
reduction reads every live instance's observables; a case retires once its liquid
fraction has fallen below the threshold (frozen, R29), and its freezing time and final
height are recorded. From the time series and the summary come the quantities of the
paper's figures:

- H/R0 against Fo (Fig. 11), with H the droplet height along the centre column;
- Pe against Fo (Fig. 12, Eq. 50);
- the solid ratio Q_L of Eq. 51 against Fo (Fig. 16);
- the scaling of the final height with the freezing time, H_m/R0 against Ste Fo
  (Fig. 17), as the slope of a least-squares line in log-log axes;
- the dimensionless freezing time t* = (t(Bo_m) - t(0)) / t(0) per Ste and
  orientation (Fig. 18).

Inputs are the synthetic half droplets of workloads.droplet_problem; nothing here
reads a dataset.
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np

from . import lbfs
from . import workloads as wl

ORIENTATION = {"vertical": 90.0, "horizontal": 0.0}


def sweep_cases(edge: int, bo_list, ste_list, orientations=("vertical", "horizontal"),
                precision: str = "fp32", gas_lambda_ratio: float | None = None) -> list[dict]:
    """One case per (Ste, orientation, Bo_m > 0) plus one field-free case per Ste."""
    out = []
    for ste in ste_list:
        for bo in bo_list:
            for ori in (orientations if bo > 0 else ("none",)):
                angle = ORIENTATION.get(ori, 90.0)
                p = wl.droplet_problem(edge, edge / 4.0, ste=float(ste), bo_m=float(bo), angle_deg=angle,
                                       precision=precision, gas_lambda_ratio=gas_lambda_ratio)
                p["case"] = dict(ste=float(ste), bo_m=float(bo), orientation=ori)
                out.append(p)
    return out


def run(cases: list[dict], chunk: int = 50, max_steps: int = 200000, done_fl: float = 1e-3,
        progress=None) -> list[dict]:
    """Advance every case to freezing (or max_steps) in one batch; returns per case its
    time series (every chunk) and, when frozen, the freezing step, time, Fo and final
    height over R0."""
    budget = sum(lbfs.Batch.instance_bytes(p) for p in cases) + (16 << 20)
    batch = lbfs.Batch(len(cases), budget, precision=cases[0]["precision"])
    results = []
    live = {}
    for p in cases:
        slot = batch.admit(p)
        if slot is None:
            raise RuntimeError("the batch buffer does not hold every case")
        r0 = float(p["drop"][2])
        rec = dict(case=p["case"], r0=r0, series=dict(step=[], fo=[], h_r0=[], pe=[], q_l=[], fl=[], wall_heat=[]),
                   frozen=False)
        results.append(rec)
        live[slot] = rec
    steps = 0
    while live and steps < max_steps:
        n = min(chunk, max_steps - steps)
        batch.step(n)
        steps += n
        obs = batch.observe(allow_nonfinite=True)
        for slot, o in obs.items():
            rec = live[slot]
            s = rec["series"]
            s["step"].append(int(o["step"]))
            s["fo"].append(o["fourier"])
            s["h_r0"].append(o["height"] / rec["r0"])
            s["pe"].append(o["peclet"])
            s["q_l"].append(o["solid_ratio"])
            s["fl"].append(o["liquid_fraction"])
            s["wall_heat"].append(o["wall_heat"])
            if o["nonfinite"]:
                rec["nonfinite"] = True
            if o["liquid_fraction"] < done_fl or o["nonfinite"]:
                rec.update(frozen=not o["nonfinite"], freeze_step=int(o["step"]), freeze_t=o["t"],
                           freeze_fo=o["fourier"], hm_r0=o["height"] / rec["r0"])
                batch.retire(slot)
                del live[slot]
        if progress is not None:
            progress(steps, len(live))
    batch.close()
    return results


def t_star(results: list[dict]) -> list[dict]:
    """(t(Bo_m) - t(0)) / t(0) for every frozen case with a frozen field-free case of the
    same Ste (Fig. 18)."""
    base = {r["case"]["ste"]: r["freeze_t"] for r in results if r["case"]["bo_m"] == 0 and r.get("frozen")}
    out = []
    for r in results:
        c = r["case"]
        if c["bo_m"] > 0 and r.get("frozen") and c["ste"] in base:
            out.append(dict(c, t_star=(r["freeze_t"] - base[c["ste"]]) / base[c["ste"]]))
    return out


def scaling_slope(results: list[dict]) -> float:
    """Slope of log(H_m/R0) against log(Ste Fo_freeze) over the frozen cases (Fig. 17)."""
    pts = [(math.log(r["case"]["ste"] * r["freeze_fo"]), math.log(r["hm_r0"]))
           for r in results if r.get("frozen") and r["freeze_fo"] > 0 and r["hm_r0"] > 0]
    if len(pts) < 2:
        return float("nan")
    x, y = np.array(pts).T
    return float(np.polyfit(x, y, 1)[0])


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--edge", type=int, default=64)
    ap.add_argument("--bo", default="0,4,8,16", help="Bo_m values")
    ap.add_argument("--ste", default="0.1,0.2,0.3", help="Stefan numbers")
    ap.add_argument("--chunk", type=int, default=50)
    ap.add_argument("--max-steps", type=int, default=100000)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--gas-lambda-ratio", type=float, default=None,
                    help="gas conductivity over the liquid's at the default gas diffusivity (air: 0.036)")
    ap.add_argument("--out", default=None, help="write the results as JSON here")
    args = ap.parse_args(argv)
    cases = sweep_cases(args.edge, [float(b) for b in args.bo.split(",")],
                        [float(s) for s in args.ste.split(",")], precision=args.precision,
                        gas_lambda_ratio=args.gas_lambda_ratio)

    def progress(steps, nlive):
        if steps % (20 * args.chunk) == 0:
            print(f"studies: step {steps}, {nlive} cases still freezing", file=sys.stderr, flush=True)

    res = run(cases, chunk=args.chunk, max_steps=args.max_steps, progress=progress)
    summary = dict(edge=args.edge, gas_lambda_ratio=args.gas_lambda_ratio, cases=[dict(r["case"], frozen=r.get("frozen", False),
                                               freeze_step=r.get("freeze_step"), freeze_fo=r.get("freeze_fo"),
                                               hm_r0=r.get("hm_r0"),
                                               h_r0_max=max(r["series"]["h_r0"]) if r["series"]["h_r0"] else None,
                                               pe_max=max(r["series"]["pe"]) if r["series"]["pe"] else None)
                                          for r in res],
                   t_star=t_star(res), scaling_slope=scaling_slope(res))
    print(json.dumps(summary))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(dict(summary=summary, results=res), f)


if __name__ == "__main__":
    main()
