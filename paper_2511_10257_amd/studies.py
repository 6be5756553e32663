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
- the scaling of Fig. 17 in two readings, each as the slope of a least-squares line in
  log-log axes: the final height against the freezing time (one point per case, H_m/R0
  against Ste Fo at freezing), and the rise of the freezing front (the frozen height
  along the centre column, Hs/R0, against Ste Fo during freezing, every case pooled);
- the dimensionless freezing time t* = (t(Bo_m) - t(0)) / t(0) per Ste and
  orientation (Fig. 18);
- without freezing, the deformation ratio b/a of a suspended ferrofluid droplet in a
  vertical field against Bo_m (Sec. 4.3, Fig. 7): b and a from the moments of the order
  parameter along and across the field;
- and water droplets at different contact angles freezing on the cold wall (Sec. 4.2).

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
        rec = dict(case=p["case"], r0=r0, series=dict(step=[], fo=[], h_r0=[], hs_r0=[], pe=[], q_l=[], fl=[],
                                                      wall_heat=[]),
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
            s["hs_r0"].append(o["solid_height"] / rec["r0"])
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


def deformation(n: int, bo_list, steps: int, chunk: int = 500, precision: str = "fp32") -> list[dict]:
    """Suspended droplets (workloads.deformation_problem) for each Bo_m in one batch:
    the series of b/a = semi_axis_y / semi_axis_x every chunk, and its mean over the last
    third of the run (the shape oscillates about its equilibrium while viscosity damps
    it)."""
    cases = [wl.deformation_problem(n, float(bo), precision=precision) for bo in bo_list]
    budget = sum(lbfs.Batch.instance_bytes(p) for p in cases) + (16 << 20)
    batch = lbfs.Batch(len(cases), budget, precision=precision)
    slots = [batch.admit(p) for p in cases]
    if None in slots:
        raise RuntimeError("the batch buffer does not hold every case")
    series = {s: dict(step=[], b_over_a=[], umax=[]) for s in slots}
    bad = set()
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        batch.step(k)
        done += k
        obs = batch.observe(allow_nonfinite=True)
        for s, o in obs.items():
            series[s]["step"].append(int(o["step"]))
            series[s]["b_over_a"].append(o["semi_axis_y"] / o["semi_axis_x"] if o["semi_axis_x"] > 0 else float("nan"))
            series[s]["umax"].append(o["umax"])
            if o["nonfinite"]:
                bad.add(s)
    batch.close()
    out = []
    for p, s in zip(cases, slots):
        ba = np.array(series[s]["b_over_a"])
        tail = ba[len(ba) - max(1, len(ba) // 3):]
        out.append(dict(bo_m=p["bo_m"], radius=p["drop"][2], b_over_a=float(np.mean(tail)),
                        b_over_a_spread=float(np.max(tail) - np.min(tail)), nonfinite=s in bad,
                        series=series[s]))
    return out


def static_freezing(thetas, nx: int = 400, ny: int = 200, R0: float | None = None, chunk: int = 100,
                    max_steps: int = 400000, done_fl: float = 1e-3, precision: str = "fp32") -> list[dict]:
    """Sec. 4.2: water droplets at the given contact angles freezing on the cold wall
    (workloads.static_droplet_problem), one batch to freezing; per angle the freezing
    step, the final height and x semi-axis over R0, and the series of the liquid
    fraction and height."""
    cases = [wl.static_droplet_problem(float(t), nx, ny, R0, precision) for t in thetas]
    budget = sum(lbfs.Batch.instance_bytes(p) for p in cases) + (16 << 20)
    batch = lbfs.Batch(len(cases), budget, precision=precision)
    slots = [batch.admit(p) for p in cases]
    if None in slots:
        raise RuntimeError("the batch buffer does not hold every case")
    recs = {s: dict(theta=p["contact_angle"][2], r0=p["r0"], frozen=False,
                    series=dict(step=[], fl=[], h_r0=[], a_r0=[])) for s, p in zip(slots, cases)}
    live = set(slots)
    steps = 0
    while live and steps < max_steps:
        batch.step(chunk)
        steps += chunk
        obs = batch.observe(allow_nonfinite=True)
        for s, o in obs.items():
            if s not in live:
                continue
            r = recs[s]
            r["series"]["step"].append(int(o["step"]))
            r["series"]["fl"].append(o["liquid_fraction"])
            r["series"]["h_r0"].append(o["height"] / r["r0"])
            r["series"]["a_r0"].append(o["semi_axis_x"] / r["r0"])
            if o["liquid_fraction"] < done_fl or o["nonfinite"]:
                r.update(frozen=not o["nonfinite"], freeze_step=int(o["step"]), hm_r0=o["height"] / r["r0"],
                         am_r0=o["semi_axis_x"] / r["r0"])
                batch.retire(s)
                live.discard(s)
    batch.close()
    return [recs[s] for s in slots]


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


def front_scaling(results: list[dict], lo: float = 0.1, hi: float = 0.6) -> dict:
    """Slope of log(Hs/R0) against log(Ste Fo) while the freezing front rises through the
    centre column: over the observations of each frozen case whose frozen height lies
    between lo and hi of its final value (a first solid layer has formed, and the front
    is still below the apex, where the droplet narrows). The slope of all cases pooled,
    and of each case alone."""
    xs, ys, per = [], [], []
    for r in results:
        if not r.get("frozen"):
            continue
        s = r["series"]
        hs, fo = np.array(s["hs_r0"]), np.array(s["fo"])
        if hs.size == 0 or hs[-1] <= 0:
            continue
        keep = (hs >= lo * hs[-1]) & (hs <= hi * hs[-1]) & (fo > 0)
        if keep.sum() < 2:
            continue
        x = np.log(r["case"]["ste"] * fo[keep])
        y = np.log(hs[keep])
        per.append(dict(r["case"], slope=float(np.polyfit(x, y, 1)[0]), points=int(keep.sum())))
        xs.append(x)
        ys.append(y)
    if not xs:
        return dict(slope=float("nan"), cases=per)
    x, y = np.concatenate(xs), np.concatenate(ys)
    return dict(slope=float(np.polyfit(x, y, 1)[0]) if x.size >= 2 else float("nan"), cases=per)


def write_csv(results: list[dict], directory: str) -> list[str]:
    """One CSV per case: step, Fo, Ste Fo, H/R0, Hs/R0, Pe, Q_L, liquid fraction, wall heat."""
    import os
    os.makedirs(directory, exist_ok=True)
    paths = []
    for r in results:
        c = r["case"]
        path = os.path.join(directory, f"ste{c['ste']:g}_bo{c['bo_m']:g}_{c['orientation']}.csv")
        s = r["series"]
        with open(path, "w") as f:
            f.write("step,fo,ste_fo,h_r0,hs_r0,pe,q_l,liquid_fraction,wall_heat\n")
            for k in range(len(s["step"])):
                f.write(f"{s['step'][k]},{s['fo'][k]:.9g},{c['ste'] * s['fo'][k]:.9g},{s['h_r0'][k]:.9g},"
                        f"{s['hs_r0'][k]:.9g},{s['pe'][k]:.9g},{s['q_l'][k]:.9g},{s['fl'][k]:.9g},"
                        f"{s['wall_heat'][k]:.9g}\n")
        paths.append(path)
    return paths


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--deformation", action="store_true",
                    help="the Sec. 4.3 deformation sweep (suspended droplets, no freezing) instead")
    ap.add_argument("--steps", type=int, default=40000, help="steps of the deformation sweep")
    ap.add_argument("--static", default=None,
                    help="contact angles (e.g. 64,98) of the Sec. 4.2 static-droplet freezing instead")
    ap.add_argument("--edge", type=int, default=64)
    ap.add_argument("--bo", default="0,4,8,16", help="Bo_m values")
    ap.add_argument("--ste", default="0.1,0.2,0.3", help="Stefan numbers")
    ap.add_argument("--chunk", type=int, default=50)
    ap.add_argument("--max-steps", type=int, default=100000)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--gas-lambda-ratio", type=float, default=None,
                    help="gas conductivity over the liquid's at the default gas diffusivity (air: 0.036)")
    ap.add_argument("--out", default=None, help="write the results as JSON here")
    ap.add_argument("--csv", default=None, metavar="DIR",
                    help="also write each case's time series (Figs. 11, 12, 16, 17) as a CSV file in DIR")
    args = ap.parse_args(argv)
    if args.static:
        res = static_freezing([float(t) for t in args.static.split(",")], nx=2 * args.edge, ny=args.edge,
                              precision=args.precision)
        print(json.dumps([{k: v for k, v in r.items() if k != "series"} for r in res]))
        if args.out:
            with open(args.out, "w") as f:
                json.dump(res, f)
        return
    if args.deformation:
        res = deformation(args.edge, [float(b) for b in args.bo.split(",")], args.steps, precision=args.precision)
        print(json.dumps([{k: v for k, v in r.items() if k != "series"} for r in res]))
        if args.out:
            with open(args.out, "w") as f:
                json.dump(res, f)
        return
    cases = sweep_cases(args.edge, [float(b) for b in args.bo.split(",")],
                        [float(s) for s in args.ste.split(",")], precision=args.precision,
                        gas_lambda_ratio=args.gas_lambda_ratio)

    def progress(steps, nlive):
        if steps % (20 * args.chunk) == 0:
            print(f"studies: step {steps}, {nlive} cases still freezing", file=sys.stderr, flush=True)

    res = run(cases, chunk=args.chunk, max_steps=args.max_steps, progress=progress)
    if args.csv:
        write_csv(res, args.csv)
    per_case = [dict(r["case"], frozen=r.get("frozen", False), freeze_step=r.get("freeze_step"),
                     freeze_fo=r.get("freeze_fo"), hm_r0=r.get("hm_r0"),
                     h_r0_max=max(r["series"]["h_r0"]) if r["series"]["h_r0"] else None,
                     pe_max=max(r["series"]["pe"]) if r["series"]["pe"] else None)
                for r in res]
    summary = dict(edge=args.edge, gas_lambda_ratio=args.gas_lambda_ratio, cases=per_case,
                   t_star=t_star(res), scaling_slope=scaling_slope(res), front_scaling=front_scaling(res))
    print(json.dumps(summary))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(dict(summary=summary, results=res), f)


if __name__ == "__main__":
    main()
