"""Continuous batching of freezing solves on one GPU (host scheduler over lbfs_batch_*).

Requests (a droplet problem each, with its own size, field direction and strength and
Stefan number) arrive over time. The server keeps one batch resident on the device:
between chunks of steps it admits waiting requests while the batch buffer (the HBM
budget) and the slots allow, advances every live solve by the same launches, reads
the FP64 observables of all of them with one reduction, and retires each solve once its
liquid fraction sum(C Fl)/sum(C) has fallen below the threshold (frozen). A solve that
is admitted while others run joins their launches at the next chunk; its fields evolve
exactly as they would alone.

Two clocks: "wall" (arrival times in seconds, latencies measured with the host clock
around device-synchronised observations) and "steps" (arrival times counted in batch
steps; deterministic, used by the tests).
"""
from __future__ import annotations

import dataclasses
import sys
import time
from collections import deque

import numpy as np

from . import lbfs


@dataclasses.dataclass
class Request:
    rid: int
    prob: dict
    arrival: float
    admitted: float | None = None
    finished: float | None = None
    slot: int | None = None
    steps: int = 0
    liquid_fraction: float = 1.0
    nonfinite: bool = False
    rejected: bool = False      # larger than the whole budget
    obs: dict | None = None

    @property
    def cells(self) -> int:
        return int(self.prob["nx"]) * int(self.prob["ny"])

    @property
    def latency(self) -> float | None:
        return None if self.finished is None else self.finished - self.arrival


class Server:
    """One resident batch plus a FIFO queue with backfill: the oldest waiting request
    that fits is admitted first, and smaller ones behind a request that does not fit
    yet may pass it."""

    def __init__(self, hbm_budget: int, max_slots: int = 256, precision: str = "fp32", chunk: int = 100,
                 done_fl: float = 1e-3, max_steps: int | None = None, device: str = "cuda:0",
                 on_finish=None, on_admit=None):
        self.batch = lbfs.Batch(max_slots, hbm_budget, precision=precision, device=device)
        self.precision = precision
        self.chunk = int(chunk)
        self.done_fl = float(done_fl)
        self.max_steps = max_steps
        self.on_finish = on_finish    # (request, slot view) before a solve retires
        self.on_admit = on_admit      # (request, slot view) after a solve is admitted
        self.live: dict[int, Request] = {}
        self.cell_steps = 0
        self.chunks = 0

    def close(self) -> None:
        self.batch.close()

    def _admit(self, waiting: deque, now: float) -> None:
        kept = deque()
        while waiting:
            req = waiting.popleft()
            prob = dict(req.prob, precision=self.precision)
            slot = self.batch.admit(prob)
            if slot is None:
                kept.append(req)
                continue
            req.slot, req.admitted = slot, now
            self.live[slot] = req
            if self.on_admit is not None:
                self.on_admit(req, self.batch.slot(slot))
        waiting.extend(kept)

    def run(self, arrivals, clock: str = "wall", horizon: float | None = None, cap: float | None = None,
            progress_every: float | None = None) -> dict:
        """Serve (arrival time, problem) pairs in arrival order. Arrivals after `horizon`
        are dropped; the run ends when everything admitted has finished or at `cap`
        (same unit as the clock), whichever is first. With progress_every (seconds of
        host time), a status line goes to stderr that often."""
        reqs = [Request(i, prob, float(t)) for i, (t, prob) in enumerate(arrivals)
                if horizon is None or t < horizon]
        waiting: deque = deque()
        nxt = 0
        t0 = time.perf_counter()
        vsteps = 0

        def now() -> float:
            return time.perf_counter() - t0 if clock == "wall" else float(vsteps)

        last_report = time.perf_counter()

        while True:
            t = now()
            while nxt < len(reqs) and reqs[nxt].arrival <= t:
                waiting.append(reqs[nxt])
                nxt += 1
            if cap is not None and t >= cap:
                break
            self._admit(waiting, t)
            if not self.live:
                # whatever still waits does not fit even into the empty batch
                while waiting:
                    waiting.popleft().rejected = True
                if nxt >= len(reqs):
                    break
                # idle until the next arrival
                if clock == "wall":
                    time.sleep(max(0.0, min(reqs[nxt].arrival - now(), 0.05)))
                else:
                    vsteps = max(vsteps, int(np.ceil(reqs[nxt].arrival)))
                continue
            if progress_every is not None and time.perf_counter() - last_report >= progress_every:
                last_report = time.perf_counter()
                done = sum(1 for r in reqs if r.finished is not None)
                print(f"serve: t={t:.1f} arrived={nxt} live={len(self.live)} waiting={len(waiting)} "
                      f"done={done} cell_steps={self.cell_steps:.3e}", file=sys.stderr, flush=True)
            n = self.chunk
            if self.max_steps is not None:
                n = min(n, max(1, min(self.max_steps - r.steps for r in self.live.values())))
            self.batch.step(n)
            obs = self.batch.observe(allow_nonfinite=True)    # synchronises the device
            vsteps += n
            self.chunks += 1
            t_done = now()
            for slot, o in obs.items():
                req = self.live[slot]
                req.steps += n
                self.cell_steps += n * req.cells
                req.liquid_fraction = o["liquid_fraction"]
                req.nonfinite = bool(o["nonfinite"])
                # (a non-finite state can read as frozen: the clamps of Eq. 8 map NaN to a bound)
                frozen = o["liquid_fraction"] < self.done_fl and not req.nonfinite
                over = self.max_steps is not None and req.steps >= self.max_steps
                if frozen or over or req.nonfinite:
                    req.obs = o
                    if frozen:
                        req.finished = t_done
                    if self.on_finish is not None:
                        self.on_finish(req, self.batch.slot(slot))
                    self.batch.retire(slot)
                    del self.live[slot]
        elapsed = now()
        return report(reqs, elapsed, self.cell_steps, clock, unfinished_live=len(self.live), waiting=len(waiting))


def report(reqs, elapsed: float, cell_steps: int, clock: str, unfinished_live: int = 0, waiting: int = 0) -> dict:
    lat = np.array([r.latency for r in reqs if r.latency is not None])
    done = len(lat)
    out = {
        "requests": len(reqs), "completed": done, "unfinished": len(reqs) - done,
        "unfinished_live": unfinished_live, "unfinished_waiting": waiting,
        "nonfinite": sum(1 for r in reqs if r.nonfinite),
        "rejected": sum(1 for r in reqs if r.rejected),
        "elapsed": elapsed, "clock": clock,
        "solves_per_unit": done / elapsed if elapsed > 0 else 0.0,
        "p50": float(np.percentile(lat, 50)) if done else None,
        "p99": float(np.percentile(lat, 99)) if done else None,
        "cell_steps": int(cell_steps),
        # cell updates one completed solve needed (its cells times its steps), on average
        "cell_steps_per_completed": (float(np.mean([r.cells * r.steps for r in reqs if r.latency is not None]))
                                     if done else None),
    }
    if clock == "wall" and elapsed > 0:
        out["mlups"] = cell_steps / elapsed / 1e6
    return out
