"""Continuous-batching server for block-MPS Trotter evolutions.

Requests (grid, chi, J, h, theta0, number of steps) arrive over time. A
request is admitted when the device-memory budget (the library's
mps_footprint_bytes per instance) and the slot limit allow; admitted
instances stay resident on the GPU, each on its own HIP stream, and every
scheduler round enqueues one Trotter step for every active instance without
waiting in between, so independent instances overlap on the device. When an
instance finishes its steps it is measured and freed, and its memory admits
queued requests in the next round (continuous batching, not a FIFO).

Per-step latency is the device time between HIP events recorded on the
instance's stream before and after its step; queue wait (arrival to
admission) is reported separately.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import mpsim
from .workloads import Instance, Request


@dataclass
class Active:
    req: Request
    rid: int
    sim: mpsim.Simulation
    stream: torch.cuda.Stream
    bytes: int
    admitted_s: float
    steps_done: int = 0
    events: list = field(default_factory=list)   # (start, stop) per step


@dataclass
class Result:
    rid: int
    inst: Instance
    obs: dict
    queue_wait_s: float
    step_ms: list


class Server:
    def __init__(self, budget_bytes: int, max_active: int = 16, seed: int = 0):
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.seed = seed

    def _admit(self, req: Request, rid: int, now: float) -> Active:
        cfg = mpsim.config_from_instance(req.inst, seed=self.seed + rid)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            sim = mpsim.Simulation(cfg, stream=stream.cuda_stream)
        return Active(req, rid, sim, stream, mpsim.footprint_bytes(cfg), now)

    def run(self, trace: list[Request], time_limit_s: Optional[float] = None) -> dict:
        """Serve `trace` (arrival times relative to the start of the run)."""
        t0 = time.perf_counter()
        pending = sorted(enumerate(trace), key=lambda x: x[1].arrival_s)
        queue: list[tuple[int, Request]] = []
        active: list[Active] = []
        results: list[Result] = []
        used = 0
        peak = 0
        peak_active = 0
        total_steps = 0
        rounds = 0
        rejected = []
        while pending or queue or active:
            now = time.perf_counter() - t0
            if time_limit_s is not None and now > time_limit_s and not active:
                break
            while pending and pending[0][1].arrival_s <= now:
                queue.append(pending.pop(0))
            # admission by footprint (continuous: every round)
            still = []
            for rid, req in queue:
                need = mpsim.footprint_bytes(mpsim.config_from_instance(req.inst))
                if need > self.budget:
                    rejected.append(rid)
                    continue
                stop_admitting = time_limit_s is not None and now > time_limit_s
                if (not stop_admitting and len(active) < self.max_active
                        and used + need <= self.budget):
                    a = self._admit(req, rid, now)
                    active.append(a)
                    used += a.bytes
                    peak = max(peak, used)
                    peak_active = max(peak_active, len(active))
                else:
                    still.append((rid, req))
            queue = still
            if not active:
                if pending:
                    time.sleep(max(0.0, min(0.01, pending[0][1].arrival_s - now)))
                continue
            # one step for every active instance, all enqueued before any wait
            evs = []
            for a in active:
                ev0 = torch.cuda.Event(enable_timing=True)
                ev0.record(a.stream)
                evs.append(ev0)
            mpsim.apply_batched([a.sim for a in active], 1)
            for a, ev0 in zip(active, evs):
                ev1 = torch.cuda.Event(enable_timing=True)
                ev1.record(a.stream)
                a.events.append((ev0, ev1))
                a.steps_done += 1
            rounds += 1
            total_steps += len(active)
            # retire finished instances
            keep = []
            for a in active:
                if a.steps_done >= a.req.inst.steps:
                    a.stream.synchronize()
                    obs = a.sim.measure()
                    ms = [e0.elapsed_time(e1) for (e0, e1) in a.events]
                    results.append(Result(a.rid, a.req.inst, obs,
                                          a.admitted_s - a.req.arrival_s, ms))
                    a.sim.free()
                    used -= a.bytes
                else:
                    keep.append(a)
            active = keep
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat = np.array([m for r in results for m in r.step_ms]) if results else np.zeros(1)
        waits = np.array([r.queue_wait_s for r in results]) if results else np.zeros(1)
        return {
            "completed": len(results), "rejected": len(rejected), "rounds": rounds,
            "peak_bytes": peak, "peak_active": peak_active, "budget_bytes": self.budget,
            "total_steps": total_steps, "wall_s": wall,
            "steps_per_s": total_steps / wall if wall > 0 else 0.0,
            "step_latency_ms_p50": float(np.percentile(lat, 50)),
            "step_latency_ms_p99": float(np.percentile(lat, 99)),
            "queue_wait_s_p50": float(np.percentile(waits, 50)),
            "queue_wait_s_p99": float(np.percentile(waits, 99)),
            "results": results,
        }


def run_alone(inst: Instance, seed: int) -> dict:
    """Evolve one instance by itself (reference for the alone-vs-mix check)."""
    cfg = mpsim.config_from_instance(inst, seed=seed)
    sim = mpsim.Simulation(cfg)
    sim.step(inst.steps)
    obs = sim.measure()
    sim.free()
    return obs
