"""Writes freeze_time.json: the freezing time of small droplets computed by the FP64 oracle.

The criterion is the one a freezing solve ends on: the liquid fraction of the droplet,
sum(C Fl) / sum(C) with C clamped to [0, 1] and Fl from Eq. 8, falls below 1e-3 (Sec. 5
follows the droplet until it has frozen completely; Eq. 51 measures the frozen part).
The recorded value is the first step, checked after every step, at which it holds; the
liquid fraction at a quarter, half and three quarters of that time is kept as well.

Calls only the oracle.   python3 tests/golden/make_freeze_golden.py [case ...]
(named cases only: they are recomputed and merged into the existing file; the 128 x 128
case takes about half an hour on one core)
"""
from __future__ import annotations

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as orc  # noqa: E402
from paper_2511_10257_amd import workloads as wl  # noqa: E402

CASES = {
    "droplet32": dict(n=32, radius=8.0, ste=0.1, bo_m=1.0, angle_deg=45.0),
    "droplet64": dict(n=64, radius=16.0, ste=0.1, bo_m=0.5, angle_deg=90.0),
    "droplet128": dict(n=128, radius=32.0, ste=0.1, bo_m=1.5, angle_deg=0.0),
}
THRESHOLD = 1e-3


def problem(case: dict, precision: str = "fp64") -> dict:
    return wl.droplet_problem(case["n"], case["radius"], ste=case["ste"], bo_m=case["bo_m"],
                              angle_deg=case["angle_deg"], precision=precision)


def freeze(case: dict) -> dict:
    o = orc.Oracle(problem(case))
    fl = [o.observe()["liquid_fraction"]]
    while fl[-1] >= THRESHOLD:
        o.step(1)
        fl.append(o.observe()["liquid_fraction"])
    n = len(fl) - 1
    return {"case": case, "threshold": THRESHOLD, "freeze_step": n,
            "fl_at": {str(q): fl[round(q * n / 4)] for q in (1, 2, 3)}}


def main():
    path = os.path.join(HERE, "freeze_time.json")
    names = sys.argv[1:] or list(CASES)
    out = json.load(open(path)) if sys.argv[1:] and os.path.exists(path) else {}
    for name in names:
        out[name] = freeze(CASES[name])
    out = {name: out[name] for name in CASES if name in out}
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
