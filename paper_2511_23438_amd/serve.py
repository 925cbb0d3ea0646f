"""Continuous-batching server for block-MPS Trotter evolutions.

Requests (grid, chi, J, h, theta0, number of steps) arrive over time. A
request is admitted when the device-memory budget (the library's
mps_footprint_bytes per instance) and the slot limit allow. An admitted
instance stays resident on the GPU with its own HIP stream and its own
worker thread, which enqueues its Trotter steps one after another and keeps
at most `depth` steps in flight on the device (it waits on the event of the
step `depth` back, which blocks only that worker). Independent instances
therefore overlap on the device, and the scheduler thread never waits on a
device: it admits arrivals as memory and slots free up (continuous
batching, not a FIFO), and retires instances whose workers report back.

Per-step latency is the device time between HIP events recorded on the
instance's stream before and after its step (the time the step took while
sharing the GPU with the other instances); queue wait (arrival to
admission) is reported separately. With an admission window, requests not
admitted by its end are left unserved; with a hard stop, workers stop
after their current step, and steps completed until then still count.
A request the library rejects (an invalid configuration, or a footprint
above the whole budget) is counted as rejected; one whose instance cannot
be created (device allocation failed) is reported with its error, and the
others are served.
"""
from __future__ import annotations

import queue as _queue
import threading
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
    events: list = field(default_factory=list)   # (start, stop) per enqueued step
    thread: Optional[threading.Thread] = None


@dataclass
class Result:
    rid: int
    inst: Instance
    obs: Optional[dict]          # None when the instance was stopped early
    queue_wait_s: float
    step_ms: list
    finished: bool
    error: str = ""


class Server:
    def __init__(self, budget_bytes: int, max_active: int = 16, seed: int = 0,
                 depth: int = 2):
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.seed = seed
        self.depth = max(1, int(depth))

    def _admit(self, req: Request, rid: int, now: float, nbytes: int) -> Active:
        cfg = mpsim.config_from_instance(req.inst, seed=self.seed + rid)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            sim = mpsim.Simulation(cfg, stream=stream.cuda_stream)
        return Active(req, rid, sim, stream, nbytes, now)

    def _worker(self, a: Active, stop: threading.Event, done: "_queue.Queue") -> None:
        err = ""
        obs = None
        finished = False
        ms: list = []
        try:
            for _ in range(a.req.inst.steps):
                if stop.is_set():
                    break
                ev0 = torch.cuda.Event(enable_timing=True)
                ev0.record(a.stream)
                a.sim.step(1)
                ev1 = torch.cuda.Event(enable_timing=True)
                ev1.record(a.stream)
                a.events.append((ev0, ev1))
                if len(a.events) > self.depth:
                    a.events[-1 - self.depth][1].synchronize()
            a.stream.synchronize()
            finished = len(a.events) == a.req.inst.steps
            if finished:
                obs = a.sim.measure()
            ms = [e0.elapsed_time(e1) for (e0, e1) in a.events]
        except Exception as e:  # reported with the result; the instance is dropped
            err = repr(e)
        finally:
            try:
                a.sim.free()
            finally:
                done.put((a, obs, finished, ms, err))

    def run(self, trace: list[Request], time_limit_s: Optional[float] = None,
            hard_stop_s: Optional[float] = None) -> dict:
        """Serve `trace` (arrival times relative to the start of the run).
        `time_limit_s`: admission window (None: until the trace is served);
        `hard_stop_s`: stop every instance after its current step."""
        t0 = time.perf_counter()
        pending = sorted(enumerate(trace), key=lambda x: x[1].arrival_s)
        need = {}
        for rid, req in pending:
            try:
                need[rid] = mpsim.footprint_bytes(mpsim.config_from_instance(req.inst))
            except mpsim.MpsError:
                need[rid] = None             # invalid configuration: rejected on arrival
        queue: list[tuple[int, Request]] = []
        active: dict[int, Active] = {}
        results: list[Result] = []
        done: "_queue.Queue" = _queue.Queue()
        stop = threading.Event()
        used = peak = peak_active = 0
        rejected: list[int] = []
        unserved: list[int] = []
        while True:
            now = time.perf_counter() - t0
            admitting = time_limit_s is None or now <= time_limit_s
            if hard_stop_s is not None and now > hard_stop_s and not stop.is_set():
                stop.set()
            while pending and pending[0][1].arrival_s <= now:
                queue.append(pending.pop(0))
            # retire instances whose workers have reported back
            while True:
                try:
                    a, obs, finished, ms, err = done.get_nowait()
                except _queue.Empty:
                    break
                a.thread.join()
                del active[a.rid]
                used -= a.bytes
                results.append(Result(a.rid, a.req.inst, obs, a.admitted_s - a.req.arrival_s,
                                      ms, finished, err))
            # admission by footprint, every round
            still = []
            for rid, req in queue:
                if need[rid] is None or need[rid] > self.budget:
                    rejected.append(rid)
                elif (admitting and not stop.is_set() and len(active) < self.max_active
                      and used + need[rid] <= self.budget):
                    try:
                        a = self._admit(req, rid, now, need[rid])
                    except mpsim.MpsError as e:
                        results.append(Result(rid, req.inst, None, now - req.arrival_s, [],
                                              False, repr(e)))
                        continue
                    a.thread = threading.Thread(target=self._worker, args=(a, stop, done),
                                                daemon=True)
                    active[rid] = a
                    used += a.bytes
                    peak = max(peak, used)
                    peak_active = max(peak_active, len(active))
                    a.thread.start()
                else:
                    still.append((rid, req))
            queue = still
            if not active:
                if stop.is_set() or not admitting or not (pending or queue):
                    break
            time.sleep(0.002)
        unserved = [rid for rid, _ in queue] + [rid for rid, _ in pending]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat = np.array([m for r in results for m in r.step_ms]) if results else np.zeros(0)
        waits = np.array([r.queue_wait_s for r in results]) if results else np.zeros(0)
        total_steps = int(sum(len(r.step_ms) for r in results))

        def pct(x, q):
            return float(np.percentile(x, q)) if len(x) else float("nan")
        return {
            "completed": int(sum(1 for r in results if r.finished)),
            "stopped": int(sum(1 for r in results if not r.finished and not r.error)),
            "errors": [r.error for r in results if r.error],
            "admitted": len(results), "rejected": len(rejected), "unserved": len(unserved),
            "peak_bytes": peak, "peak_active": peak_active, "budget_bytes": self.budget,
            "total_steps": total_steps, "wall_s": wall,
            "steps_per_s": total_steps / wall if wall > 0 else 0.0,
            "step_latency_ms_p50": pct(lat, 50),
            "step_latency_ms_p99": pct(lat, 99),
            "queue_wait_s_p50": pct(waits, 50),
            "queue_wait_s_p99": pct(waits, 99),
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
