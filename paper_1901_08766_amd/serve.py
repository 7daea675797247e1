"""Serving loop over the native pool (``lbvp.Pool``): requests arrive on the wall
clock at their Poisson arrival times, are admitted first-in first-out while the
pool has a free slot and room under its memory cap, advance in epochs together
with every other resident solve, and are handed back (force and mass records,
optionally the final fields) as soon as they complete on the device, which
frees their slot and memory for the next arrivals. Latency = time the results
are on the host minus arrival time.

The scheduling itself (epochs, admission by footprint, the arena, completion
events) is native; this module only drives the clock and collects results.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from . import lbvp


@dataclass
class ServeReport:
    """Latencies and node updates count valid results only: a solve whose mass
    went non-finite (E_UNSTABLE) delivered no usable result, so its latency and
    its node updates are kept apart."""
    latencies: Dict[int, float] = field(default_factory=dict)   # request id -> seconds (valid results)
    node_updates: int = 0                                       # of valid results
    wall_s: float = 0.0
    epochs: int = 0
    max_resident: int = 0
    unstable: List[int] = field(default_factory=list)           # ids whose mass went non-finite
    unstable_latencies: Dict[int, float] = field(default_factory=dict)
    unstable_node_updates: int = 0

    def percentile(self, q: float) -> float:
        v = np.array(sorted(self.latencies.values()))
        return float(np.percentile(v, q)) if len(v) else float("nan")

    @property
    def mlups(self) -> float:
        return self.node_updates / max(self.wall_s, 1e-12) / 1e6

    def summary(self) -> dict:
        return {"requests": len(self.latencies), "p50_s": round(self.percentile(50), 4),
                "p99_s": round(self.percentile(99), 4), "mean_s": round(float(np.mean(list(self.latencies.values()))), 4)
                if self.latencies else None, "MLUPS": round(self.mlups, 1), "wall_s": round(self.wall_s, 3),
                "epochs": self.epochs, "max_resident": self.max_resident, "unstable": len(self.unstable),
                "unstable_node_updates": self.unstable_node_updates}


def serve(requests, pool, max_epoch_steps: int = 256, fields: bool = False,
          on_result: Optional[Callable] = None) -> ServeReport:
    """Run ``requests`` (``inputs.Request``: rid, arrival seconds, problem with
    .steps) through ``pool``. ``on_result(request, forces, mass, fields_or_None)``
    is called for each completed request before its slot is released."""
    arrivals = collections.deque(sorted(requests, key=lambda r: r.arrival))
    queued: collections.deque = collections.deque()
    resident: Dict[int, object] = {}
    rep = ServeReport()
    t0 = time.perf_counter()
    while arrivals or queued or resident:
        now = time.perf_counter() - t0
        while arrivals and arrivals[0].arrival <= now:
            queued.append(arrivals.popleft())
        while queued:
            r = queued[0]
            slot = pool.admit(r.problem, r.problem.steps)
            if slot is None:
                if not resident:
                    raise RuntimeError(f"request {r.rid} ({r.problem.nx}x{r.problem.ny}) can never fit the pool")
                break
            resident[slot] = r
            queued.popleft()
        rep.max_resident = max(rep.max_resident, len(resident))
        ran = pool.run_epoch(max_epoch_steps) if resident else 0
        done = pool.poll(wait=(ran == 0 and bool(resident)))
        for slot in done:
            r = resident.pop(slot)
            ok = True
            try:
                forces, mass, _ = pool.forces(slot)
            except lbvp.LbvpError as e:       # reported, not fatal: the solve itself diverged
                if e.status != lbvp.E_UNSTABLE:
                    raise
                forces, mass, _ = e.data
                rep.unstable.append(r.rid)
                ok = False
            flds = pool.fields(slot) if fields else None
            latency = time.perf_counter() - t0 - r.arrival
            work = r.problem.nx * r.problem.ny * r.problem.steps
            if ok:
                rep.latencies[r.rid] = latency
                rep.node_updates += work
            else:
                rep.unstable_latencies[r.rid] = latency
                rep.unstable_node_updates += work
            if on_result is not None:
                on_result(r, forces, mass, flds)
            pool.release(slot)
        if not resident and not queued and arrivals:
            time.sleep(max(0.0, arrivals[0].arrival - (time.perf_counter() - t0)))
    rep.wall_s = time.perf_counter() - t0
    rep.epochs = pool.stats()["epochs"]
    return rep


def sample_pool_shape(problems: List, storage: str, steps: int = 40):
    """Tune the launch shape and layout on a sample of request domains (run as
    one batch); returns the tuner's best row."""
    import torch

    stream = torch.cuda.Stream()
    solvers = [lbvp.Solver(p, storage=storage, force_every=1, force_capacity=8, stream=stream) for p in problems]
    try:
        _, best = lbvp.tune(solvers, steps=steps, layouts=True)
    finally:
        for s in solvers:
            s.close()
    return best
