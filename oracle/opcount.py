"""Algorithmic floating-point work of one time step, counted on the oracle itself.

TEST INFRASTRUCTURE. Compiles the oracle's C source as C++ with a counting number type
in place of double (opcount.cpp), runs one step of a workload and prints the operations
per cell: the whole step, the magnetic phase (permeability, sweeps, residual) and one
right-hand side R(W) with the Kelvin force, and the magnetic phase by the LBFS
pseudo-time solve (the literal m* construction of every face, same number of steps). Divisions, square roots and transcendental
calls count as one operation each, an add or a multiply as one (a fused multiply-add is
two), comparisons and selects are listed apart and not counted as FLOPs.

    python3 oracle/opcount.py [--workload droplet256] [--n 128]
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import oracle as orc  # noqa: E402

LIB = os.path.join(HERE, "libopcount.so")
KINDS = ("add", "mul", "div", "special", "cmp")


def build() -> str:
    src = os.path.join(HERE, "opcount.cpp")
    deps = [src, os.path.join(HERE, "lbfs_oracle.c"), os.path.join(HERE, "lbfs_oracle.h")]
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(d) for d in deps):
        subprocess.check_call(["g++", "-O1", "-std=c++17", "-Wall", "-fPIC", "-shared", "-o", LIB, src])
    return LIB


def _counts(L) -> dict:
    out = (C.c_longlong * 5)()
    L.opc_read(out)
    return dict(zip(KINDS, out))


def count(prob: dict) -> dict:
    L = orc.load(build())
    L.opc_reset.argtypes = []
    L.opc_read.argtypes = [C.POINTER(C.c_longlong)]
    o = orc.Oracle(dict(prob, precision="fp64"), library=L)
    o.step(2)                      # leave the initial state: S and velocities non-zero
    cells = o.n
    res = {}
    L.opc_reset()
    o.step(1)
    res["step"] = _counts(L)
    L.opc_reset()
    o.mag_sweeps(0, 1.0)
    res["mag_setup"] = _counts(L)           # permeability and residual only
    L.opc_reset()
    o.mag_sweeps(int(prob.get("sweeps", 4)), float(prob.get("omega", 1.0)))
    res["mag"] = _counts(L)
    L.opc_reset()
    o.mag_lbfs(0, 1.0, 0.0)
    res["mag_lbfs_setup"] = _counts(L)      # permeability and residual only
    L.opc_reset()
    o.mag_lbfs(int(prob.get("sweeps", 4)), 1.0, 0.0)
    res["mag_lbfs"] = _counts(L)
    L.opc_reset()
    o.rhs()
    res["rhs"] = _counts(L)
    per = {}
    for k, c in res.items():
        flops = c["add"] + c["mul"] + c["div"] + c["special"]
        per[k] = dict({n: c[n] / cells for n in KINDS}, flops=flops / cells)
    per["stage"] = {"flops": (per["step"]["flops"] - per["mag"]["flops"]) / 3.0}
    per["mag_sweep"] = {"flops": (per["mag"]["flops"] - per["mag_setup"]["flops"]) / max(1, int(prob.get("sweeps", 4)))}
    per["mag_lbfs_pseudo_step"] = {"flops": (per["mag_lbfs"]["flops"] - per["mag_lbfs_setup"]["flops"]) /
                                   max(1, int(prob.get("sweeps", 4)))}
    return {"workload": prob.get("name", f"droplet {o.nx}x{o.ny}"), "cells": cells, "per_cell": per}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", default="droplet256", choices=["droplet64", "droplet256", "droplet1024"])
    ap.add_argument("--n", type=int, default=128, help="grid edge of the counted run (droplet radius n/4)")
    args = ap.parse_args()
    from paper_2511_10257_amd import workloads as wl
    base = {"droplet64": wl.droplet64, "droplet256": wl.droplet256,
            "droplet1024": lambda: wl.droplet1024("fp64")}[args.workload]()
    prob = base
    if args.n != base["nx"]:
        prob = wl.droplet_problem(args.n, args.n / 4.0, base["ste"], base["bo_m"], base["angle_deg"],
                                  rho_ratio=round(base["rho"][1] / base["rho"][2]), precision="fp64")
    print(json.dumps(count(prob), indent=1))


if __name__ == "__main__":
    main()
