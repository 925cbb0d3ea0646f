#!/usr/bin/env python3
"""Trotter steps per second of the block-MPS evolution of the periodic 6x8
transverse-field Ising grid (two half-row blocks of 4 qubits per row: d = 16,
12 sites) at bond dimension chi = 1024, on one MI355X.

One step = one whole Trotter step of the hot path: every two-site update of
the step schedule (contraction with the gate, Gram matrix, top-chi
eigenspace, truncation, fidelity), the single-site layer, and one
measurement of <Z_tot>, <Z_tot^2> and F_MPS, with the paper's couplings
(J = -1, h = 2, dt = 0.25). `--schedule 2` (default) is the rotating-row
schedule (34 two-site updates per step at 6x8), `--schedule 1` the
block-pair schedule with routed wrap pairs (54); both apply every coupling
once per step. `--schedule 4` is the paper's own gate-by-gate path: every
ZZ bond between two blocks is a rank-2 operator that doubles the bonds
between them, followed by bond-by-bond truncation (60 gates and 172 bond
truncations per step at 6x8); its finite-chi results differ from the
block-pair schedules.

The roofline line times one launch class on the library's stream (HIP
events, `mps_profile`): `gram` (default) is the float64 Gram-matrix GEMM,
`gemm` every float64 GEMM, `theta` the theta contraction, `trd_hemv` the
mat-vec of the one-stage tridiagonalisation (only used below a Gram side of
2048). Achieved = algorithmic work of the timed launches / their summed
duration; peak = the published MI355X figure.

Start state (`--start`): `random` (default) is a seeded random MPS in mixed
canonical form at the saturated bond dimensions of the workload
([1, 16, 256, 1024 x 7, 256, 16, 1]), so every timed step has steady-state
shapes; `product` is the paper's product state (theta0 = pi/18), whose first
steps are cheaper while the bonds grow (use --warmup to skip them).

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

T_PROC0 = time.perf_counter()   # the wall budget counts from here

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Trotter steps/sec at 6x8 χ=1024 (MFMA %); p50/p99 step latency served"
PEAK = {"hbm": (8000.0, "GB/s"), "fp64": (78.6, "TFLOP/s")}
# kernel class timed for the roofline line and its bound
DOMINANT = {"trd_hemv": "hbm", "gram": "fp64", "gemm": "fp64", "theta": "fp64"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("linalg.hip", "gemm.hip", "band.hip"):
        with open(os.path.join(ROOT, "paper_2511_23438_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kind: str, workload: str):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary, valid
    only while the kernel sources still hash to the value it records."""
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.md" % (kind, workload))
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("traffic_") and "=" in line:
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("traffic_source_hash") != kernel_source_hash():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline_gate_by_gate(rows: int, cols: int, chi: int, budget_s: float) -> dict:
    """Oracle timed on one gate of the gate-by-gate path at a reduced bond
    dimension (a rank-2 operator between neighbouring bulk sites: one LQ
    step and one bond SVD), extrapolated to chi by the cubic cost and
    multiplied by the bond truncations of one step."""
    from oracle import mps as omps
    from oracle.lattice import Grid
    from oracle.schedule import step_ops
    from paper_2511_23438_amd import workloads
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    g = Grid(rows, cols)
    ops = [o for o in step_ops(g, g.snake(), 1, 4) if o[0] == "ZZ"]
    ntrunc = sum(o[2] - o[1] for o in ops)
    gate = [o for o in ops if o[2] == o[1] + 1 and o[1] == rows - 1][0]
    chi_s = 64
    while True:
        sites, centre = workloads.random_mps(rows, cols, chi_s, 99, centre=gate[1])
        m = omps.BlockMPS.from_sites(g, chi_s, sites, centre, -1.0, 2.0, 0.25, schedule=4)
        t0 = time.perf_counter()
        m.apply_zz_mpo(*gate[1:])
        t_s = time.perf_counter() - t0
        log("cpu baseline sample: chi_s=%d one gate %.2fs" % (chi_s, t_s))
        if t_s * 8 > budget_s or chi_s * 2 > chi:
            break
        chi_s *= 2
    step_s = t_s * (chi / chi_s) ** 3 * ntrunc
    return {"value": 1.0 / step_s, "unit": "steps/s", "cores": int(cores), "kind": "oracle",
            "sample": ("one gate between neighbouring bulk sites (LQ step + bond SVD) of the "
                       "%dx%d grid at chi=%d took %.2fs; scaled by (chi/%d)^3 over the %d bond "
                       "truncations of a saturated chi=%d step" % (rows, cols, chi_s, t_s, chi_s,
                                                                  ntrunc, chi))}


def cpu_baseline(rows: int, cols: int, chi: int, budget_s: float, schedule: int = 1) -> dict:
    """Oracle (numpy, float64) timed on a bounded sample of the workload: one
    bulk two-site update of the same grid at a reduced bond dimension,
    extrapolated to chi by the cubic cost of its SVD and summed over the
    updates of one steady-state step."""
    if schedule == 4:
        return cpu_baseline_gate_by_gate(rows, cols, chi, budget_s)
    import numpy as np
    from oracle import mps as omps
    from oracle.lattice import Grid
    from oracle.schedule import step_ops
    from paper_2511_23438_amd import workloads
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    d = 2 ** ((cols + 1) // 2)
    g = Grid(rows, cols)
    timed = None
    chi_s = 64
    while True:
        sites, centre = workloads.random_mps(rows, cols, chi_s, 99)
        m = omps.BlockMPS.from_sites(g, chi_s, sites, centre, -1.0, 2.0, 0.25)
        i = rows - 1  # a bulk site pair
        m.move_centre(i)
        t0 = time.perf_counter()
        m.apply_u2(i, False, True)
        dt = time.perf_counter() - t0
        kg = min(sites[i].shape[0] * d, d * sites[i + 1].shape[2])
        timed = (chi_s, kg, dt)
        log("cpu baseline sample: chi_s=%d kg=%d update %.2fs" % (chi_s, kg, dt))
        if dt * 8 > budget_s or chi_s * 2 > chi:
            break
        chi_s *= 2
    chi_s, kg_s, t_s = timed
    # steady-state kg of every update in one step at the target chi
    N = 2 * rows
    caps = [1] + [int(min(chi, d ** b, d ** (N - b))) for b in range(1, N)] + [1]
    step_s = 0.0
    nup = 0
    for op in step_ops(g, g.snake(), 1, schedule):
        if op[0] != "U2":
            continue
        i = op[1]
        kg = min(caps[i] * d, d * caps[i + 2])
        step_s += t_s * (kg / kg_s) ** 3
        nup += 1
    return {"value": 1.0 / step_s, "unit": "steps/s", "cores": int(cores), "kind": "oracle",
            "sample": ("one bulk two-site update (numpy SVD) of the %dx%d grid at chi=%d "
                       "(Gram side %d) took %.2fs; scaled by (kg/%d)^3 over the %d updates "
                       "of a saturated chi=%d step" % (rows, cols, chi_s, kg_s, t_s, kg_s, nup,
                                                       chi))}


def served(time_limit: float, chi_cap: int, n_req: int, hard_stop_s: float,
           seed: int = 2511) -> dict:
    """Continuous-batching run over the first `n_req` requests of the seeded
    Poisson trace of the served workload (50 requests/s, grids 4x4..7x8, chi
    log-uniform in [64, chi_cap], 10-40 steps each, complex64 contractions):
    admission closes after `time_limit` seconds and every instance stops
    after its current step at `hard_stop_s`; the steps completed by then
    give the per-step latency distribution and the aggregate rate."""
    import torch
    from paper_2511_23438_amd import serve, workloads
    trace = workloads.serving_trace(n_req, seed=seed, chi_max=chi_cap)
    free, total = torch.cuda.mem_get_info()
    srv = serve.Server(budget_bytes=int(0.8 * free), max_active=16, seed=seed, depth=1)
    out = srv.run(trace, time_limit_s=time_limit, hard_stop_s=hard_stop_s)
    res = out.pop("results")
    out["requests"] = [{"grid": "%dx%d" % (r.inst.rows, r.inst.cols), "chi": r.inst.chi,
                        "steps": r.inst.steps, "steps_done": len(r.step_ms),
                        "finished": r.finished} for r in sorted(res, key=lambda r: r.rid)]
    out.update({"requests_in_trace": n_req, "chi_cap": chi_cap, "precision": "c64",
                "arrival_rate_per_s": 50.0})
    return out


def concurrent_from(sites, centre, rows: int, cols: int, chi: int, precision: str,
                    schedule: int, count: int) -> dict:
    """`count` independent instances of the workload, each loaded with the
    given start state and on its own stream, stepped together through the
    batched entry point; one step and one measurement per instance in the
    timed region."""
    import torch
    from paper_2511_23438_amd import mpsim
    sims, streams = [], []
    try:
        for k in range(count):
            st = torch.cuda.Stream()
            cfg = mpsim.make_config(rows, cols, chi, precision=precision, schedule=schedule,
                                    seed=k)
            with torch.cuda.stream(st):
                sim = mpsim.Simulation(cfg, stream=st.cuda_stream)
            sims.append(sim)
            if sites is not None:
                sim.set_state(sites, centre)
            streams.append(st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mpsim.apply_batched(sims, 1)
        obs = [s.measure() for s in sims]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    finally:
        for s in sims:
            s.free()
    return {"instances": count, "precision": precision, "seconds": el,
            "steps_per_s": count / el, "per_instance_steps_per_s": 1.0 / el,
            "z": [o["z"] for o in obs], "fidelity": [o["fidelity"] for o in obs]}


def batched_set(count: int, steps: int, seed: int = 2511, alone_sample: int = 0,
                alone_only: bool = False) -> dict:
    """The batched workload: `count` independent instances (grids 4x5, 5x5,
    5x6, 6x6 with d 4 and 8, chi in {32, 64, 128, 256}, random J, h, theta0,
    complex64 contractions), each evolved `steps` Trotter steps from its
    product state. Batched: every instance on its own stream, all stepped
    through mps_apply_trotter_step_batched one step at a time (all instances
    enqueued, then one synchronisation per step). One at a time: the first
    `alone_sample` instances (all if 0) evolved alone, one after another; the
    aggregate rates are compared per instance-step. Results of those
    instances are compared bit for bit between the two runs."""
    import torch
    from paper_2511_23438_amd import mpsim, workloads
    insts = workloads.batched(count, seed=seed)
    if alone_only:
        t0 = time.perf_counter()
        per = []
        for k in range(count):
            t1 = time.perf_counter()
            sim = mpsim.Simulation(mpsim.config_from_instance(insts[k], seed=k))
            sim.step(steps)
            sim.measure()
            sim.free()
            per.append(time.perf_counter() - t1)
            log("batched set: instance %d alone done, %.1fs" % (k, time.perf_counter() - t0))
        t_alone = time.perf_counter() - t0
        return {"instances": count, "steps_each": steps,
                "alone_seconds": t_alone, "alone_steps_per_s": count * steps / t_alone,
                "alone_seconds_each": per}
    sims, streams = [], []
    for k, inst in enumerate(insts):
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            sims.append(mpsim.Simulation(mpsim.config_from_instance(inst, seed=k),
                                         stream=st.cuda_stream))
        streams.append(st)
    torch.cuda.synchronize()
    log("batched set: %d instances created" % count)
    t0 = time.perf_counter()
    for k in range(steps):
        mpsim.apply_batched(sims, 1)
        torch.cuda.synchronize()
        log("batched set: step %d done, %.1fs" % (k + 1, time.perf_counter() - t0))
    obs = [s.measure() for s in sims]
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    for s in sims:
        s.free()
    log("batched set: %d x %d steps in %.1fs (%.3f steps/s)" % (
        count, steps, t_batched, count * steps / t_batched))
    nalone = count if alone_sample <= 0 else min(alone_sample, count)
    t0 = time.perf_counter()
    same = 0
    for k in range(nalone):
        sim = mpsim.Simulation(mpsim.config_from_instance(insts[k], seed=k))
        sim.step(steps)
        o = sim.measure()
        sim.free()
        same += int(all(o[key] == obs[k][key] for key in ("z", "z2", "log_fidelity")))
        log("batched set: instance %d alone done, %.1fs" % (k, time.perf_counter() - t0))
    torch.cuda.synchronize()
    t_alone = time.perf_counter() - t0
    rate_b = count * steps / t_batched
    rate_a = nalone * steps / t_alone
    grids = sorted({"%dx%d" % (i.rows, i.cols) for i in insts})
    return {"instances": count, "steps_each": steps, "grids": grids,
            "chis": sorted({i.chi for i in insts}), "precision": "c64",
            "batched_seconds": t_batched, "batched_steps_per_s": rate_b,
            "alone_instances": nalone, "alone_seconds": t_alone, "alone_steps_per_s": rate_a,
            "speedup": rate_b / rate_a, "bitwise_equal_alone_and_batched": same,
            "min_fidelity": min(o["fidelity"] for o in obs)}


def cube_rate(shape: tuple[int, int, int], chi: int, precision: str, steps: int,
              seed: int) -> dict:
    """Trotter steps/s of the cubic lattice with one qubit per site (open
    boundaries, route-and-return schedule) from a seeded random MPS at
    saturated bonds; each step includes one measurement."""
    import torch
    from paper_2511_23438_amd import mpsim, workloads
    lx, ly, lz = shape
    n = lx * ly * lz
    cfg = mpsim.make_config(lx, ly, chi, precision=precision, schedule=3, layers=lz,
                            periodic=False)
    sim = mpsim.Simulation(cfg)
    sites, centre = workloads.random_mps(lx, ly, chi, seed, dims=[2] * n)
    sim.set_state(sites, centre)
    del sites
    ops = mpsim.schedule_dump(cfg, 1)
    nu2 = int(sum(1 for r in ops if r[0] == 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sim.step(1)
        obs = sim.measure()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sim.free()
    return {"workload": "tfim_cube_%dx%dx%d_chi%d" % (lx, ly, lz, chi), "qubits": n,
            "two_site_updates_per_step": nu2, "steps": steps, "seconds": el,
            "steps_per_s": steps / el, "z": obs["z"], "fidelity": obs["fidelity"]}


def xy_rate(shape: tuple[int, int], chi: int, precision: str, steps: int, seed: int) -> dict:
    """Trotter steps/s of the XY-model quench (one qubit per site, open
    boundaries, depth-7 second-order steps with every bond routed and
    returned) from a seeded random MPS at saturated bonds; each step includes
    one measurement of the X^2 signal and the charge."""
    import torch
    from paper_2511_23438_amd import mpsim, workloads
    lx, ly = shape
    n = lx * ly
    # no preparation at init: the random start state replaces it
    cfg = mpsim.make_xy_config(lx, ly, chi, precision=precision, tau=0.0)
    sim = mpsim.Simulation(cfg)
    sites, centre = workloads.random_mps(lx, ly, chi, seed, dims=[2] * n)
    sim.set_state(sites, centre)
    del sites
    ops = mpsim.schedule_dump(cfg, 1)
    nu2 = int(sum(1 for r in ops if r[0] == 1))
    ngate = int(sum(1 for r in ops if r[0] == 1 and r[3] != 0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sim.step(1)
        obs = sim.measure()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sim.free()
    return {"workload": "xy_%dx%d_chi%d" % (lx, ly, chi), "qubits": n,
            "two_site_updates_per_step": nu2, "gated_updates_per_step": ngate, "steps": steps,
            "seconds": el, "steps_per_s": steps / el, "x2": obs["z2"], "z": obs["z"],
            "fidelity": obs["fidelity"]}


def state_rate(sites, centre, rows: int, cols: int, chi: int, precision: str, schedule: int,
               theta0: float, warmup: int, max_steps: int, deadline: float, prof: str,
               min_work: float, reserve_fn=None) -> dict:
    """Timed Trotter steps of one instance loaded with the given start state:
    `warmup` untimed steps, then up to `max_steps` timed steps (each a whole
    step plus one measurement), stopping before a step that would end after
    `deadline` (perf_counter seconds; the first timed step always runs).
    `reserve_fn(step_seconds)` may move the deadline earlier once the step
    time is known. The launch class `prof` is timed with HIP events on the
    library's stream over the timed steps."""
    import torch
    from paper_2511_23438_amd import mpsim
    cfg = mpsim.make_config(rows, cols, chi, theta0=theta0, precision=precision,
                            schedule=schedule)
    sim = mpsim.Simulation(cfg)
    try:
        if sites is not None:       # None: the product state of the config
            sim.set_state(sites, centre)
        est = None
        done_w = 0
        for w in range(warmup):
            if est is not None and time.perf_counter() + 2 * est > deadline:
                break
            t0 = time.perf_counter()
            sim.step(1)
            sim.measure()
            est = time.perf_counter() - t0
            done_w += 1
            log("[%s] warmup step %d: %.2fs" % (precision, w + 1, est))
            if reserve_fn is not None:
                deadline = min(deadline, reserve_fn(est))
        t_start = [time.perf_counter()]

        def progress(step, upd, n):
            if upd % 6 == 0 or upd == n:
                log("  [%s] update %d/%d enqueued, %.1fs" % (precision, upd, n,
                                                            time.perf_counter() - t_start[0]))
        sim.set_progress(progress)
        sim.profile(prof, min_work=min_work)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_start[0] = t0
        k = 0
        obs = None
        while k < max_steps:
            if k > 0:
                per = (time.perf_counter() - t0) / k
                if time.perf_counter() + per > deadline:
                    break
            sim.step(1)
            obs = sim.measure()          # part of the step: one measurement per step
            k += 1
            log("[%s] step %d: %.2fs since start, <Z>=%.6f <Z^2>=%.6f F=%.4e" % (
                precision, k, time.perf_counter() - t0, obs["z"], obs["z2"], obs["fidelity"]))
            if k == 1 and reserve_fn is not None:
                deadline = min(deadline, reserve_fn(time.perf_counter() - t0))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        ms_k, launches, work = sim.profile_read()
        sim.profile("off")
        sim.set_progress(None)
        return {"precision": precision, "steps": k, "warmup": done_w, "seconds": elapsed,
                "steps_per_s": k / elapsed, "ms_per_step": 1e3 * elapsed / k,
                "prof": {"kernel": prof, "ms": ms_k, "launches": launches, "work": work},
                "observables": {"z": obs["z"], "z2": obs["z2"], "fidelity": obs["fidelity"],
                                "norm": obs["norm"], "eig_suspect": obs["eig_suspect"]}}
    finally:
        sim.free()


def step_model_flops(rows: int, cols: int, chi: int, schedule: int, order: int = 1):
    """Algorithmic work of one step at saturated bonds, in flops of the
    standard two-site update (8 flops per complex multiply-add): per update
    the theta contraction 8 m n b1, the Gram matrix on the smaller side
    (lower half) 4 kg (kg + 1) o, the reduction of that Hermitian matrix
    (16/3) kg^3, the back-transformation of the q kept vectors 8 kg^2 q and
    C = U^H theta 8 q kg o (m x n the theta shape, kg x o its sides after a
    SWAP, q = min(chi, kg)); plus the measurement sweep (three environments,
    two products per site). The factored Gram matrix of updates without
    SWAP does less than this. None for the gate-by-gate schedule."""
    if schedule not in (1, 2, 3):
        return None
    from paper_2511_23438_amd import mpsim
    cfg = mpsim.make_config(rows, cols, chi, schedule=schedule, order=order)
    ops = mpsim.schedule_dump(cfg, 1)
    wl, wr = (cols + 1) // 2, cols // 2
    n_sites = 2 * rows

    def dim(b: int) -> int:
        return 2 ** (wl if b % 2 == 0 else wr)

    pos = []
    for r in range(rows):
        pos += [2 * r, 2 * r + 1] if r % 2 == 0 else [2 * r + 1, 2 * r]

    def caps() -> list:
        dims = [dim(b) for b in pos]
        out = []
        for p in range(n_sites + 1):
            left = math.prod(dims[:p])
            right = math.prod(dims[p:])
            out.append(min(chi, left, right))
        return out

    total = 0.0
    for kind, site, swap, _gate, _ba, _bb in ops.tolist():
        if kind != 1:
            continue
        c = caps()
        b0, b1, b2 = c[site], c[site + 1], c[site + 2]
        d1, d2 = dim(pos[site]), dim(pos[site + 1])
        m, n = b0 * d1, d2 * b2
        mo, no = (b0 * d2, d1 * b2) if swap else (m, n)
        kg, o = min(mo, no), max(mo, no)
        q = min(chi, kg)
        total += (8.0 * m * n * b1 + 4.0 * kg * (kg + 1) * o + 16.0 / 3.0 * kg ** 3
                  + 8.0 * kg * kg * q + 8.0 * q * kg * o)
        if swap:
            pos[site], pos[site + 1] = pos[site + 1], pos[site]
    c = caps()
    for p in range(n_sites):
        b, d, b2 = c[p], dim(pos[p]), c[p + 1]
        total += 3 * (8.0 * b * b * d * b2 + 8.0 * b2 * b2 * b * d)
    return total


def roofline(prof: dict, elapsed: float) -> dict:
    bound = DOMINANT[prof["kernel"]]
    peak, unit = PEAK[bound]
    launches = max(prof["launches"], 1)
    avg_s = (prof["ms"] / 1e3) / launches
    per_launch = prof["work"] / launches
    scale = 1e9 if bound == "hbm" else 1e12
    achieved = per_launch / avg_s / scale if avg_s > 0 else 0.0
    return {"bound": "hbm" if bound == "hbm" else "mfma", "achieved": achieved, "peak": peak,
            "unit": unit, "frac": achieved / peak, "traffic": None,
            "kernel": prof["kernel"], "launches": prof["launches"],
            "avg_launch_us": avg_s * 1e6, "work_per_launch": per_launch,
            "kernel_time_share": (prof["ms"] / 1e3) / elapsed if elapsed > 0 else 0.0}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed steps requested (fewer are timed if the wall budget ends first)")
    ap.add_argument("--warmup", type=int, default=1,
                    help="untimed steps requested; at most one is run from the saturated "
                         "random start state, whose steps already have steady-state shapes")
    ap.add_argument("--budget", type=float, default=500.0,
                    help="wall-clock seconds from process start to the JSON line; the timed "
                         "loop and the later legs are cut to fit")
    ap.add_argument("--start", default="random", choices=["random", "product"])
    ap.add_argument("--seed", type=int, default=1234)
    ap.add_argument("--pmc-sample", action="store_true",
                    help="counter sample: a 1 GiB elementwise kernel, then one bulk two-site "
                         "update with SWAP (direct Gram matrix)")
    ap.add_argument("--pmc-eig-path", type=int, default=0, choices=[0, 1, 2],
                    help="eigensolver of the counter sample (0 automatic, 1 one-stage, "
                         "2 two-stage)")
    ap.add_argument("--rows", type=int, default=6)
    ap.add_argument("--cols", type=int, default=8)
    ap.add_argument("--chi", type=int, default=1024)
    ap.add_argument("--precision", default="bf16x3", choices=["fp64", "c64", "bf16x3"])
    ap.add_argument("--compare", default="fp64",
                    help="precision of the one-step comparison leg on the same start state "
                         "('none' disables it)")
    ap.add_argument("--theta0", type=float, default=math.pi / 18)
    ap.add_argument("--schedule", type=int, default=2, choices=[1, 2, 4],
                    help="1: wrap pairs routed by SWAPs and back; 2: rotating rows; "
                         "4: gate by gate (rank-2 operators, bond truncations)")
    ap.add_argument("--prof", default="gram", choices=sorted(DOMINANT))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=30.0)
    ap.add_argument("--serve-seconds", type=float, default=40.0,
                    help="admission window of the served run (0 disables it)")
    ap.add_argument("--serve-chi-cap", type=int, default=1024)
    ap.add_argument("--serve-requests", type=int, default=16)
    ap.add_argument("--cube", default="",
                    help="also time the cubic lattice LX,LY,LZ (one qubit per site)")
    ap.add_argument("--cube-chi", type=int, default=64)
    ap.add_argument("--cube-steps", type=int, default=2)
    ap.add_argument("--xy", default="",
                    help="also time the XY-model quench on the LX,LY grid")
    ap.add_argument("--xy-chi", type=int, default=256)
    ap.add_argument("--xy-steps", type=int, default=1)
    ap.add_argument("--batched-set", type=int, default=0,
                    help="also run the batched workload with this many instances (64 in the "
                         "workload definition)")
    ap.add_argument("--batched-steps", type=int, default=20)
    ap.add_argument("--batched-alone-only", action="store_true",
                    help="with --batched-only: run every instance of the set one at a time only")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched workload and print its result")
    ap.add_argument("--batched-alone", type=int, default=0,
                    help="instances of the batched set also run one at a time (0: all)")
    ap.add_argument("--instances", type=int, default=4,
                    help="concurrent instances of the workload in the batched leg (one step "
                         "each, headline precision; 0 disables it)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: runs on several GPUs are not supported "
              "(--gpus must be 1; independent instances shard by placing whole "
              "instances on each GPU)", file=sys.stderr)
        return 2
    deadline = T_PROC0 + args.budget

    def left() -> float:
        return deadline - time.perf_counter()

    cpu = None
    if not args.no_cpu_baseline and not args.pmc_sample and not args.batched_only:
        t0 = time.perf_counter()
        cpu = cpu_baseline(args.rows, args.cols, args.chi, args.cpu_budget, args.schedule)
        log("cpu baseline: %.3e steps/s (%.1fs)" % (cpu["value"], time.perf_counter() - t0))

    import torch
    from paper_2511_23438_amd import mpsim
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.batched_only:
        res = batched_set(args.batched_set or 64, args.batched_steps,
                          alone_sample=args.batched_alone, alone_only=args.batched_alone_only)
        print(json.dumps({"batched_set": res, "wall_s": time.perf_counter() - T_PROC0}),
              flush=True)
        return 0

    if args.pmc_sample:
        from paper_2511_23438_amd import workloads
        cfg = mpsim.make_config(args.rows, args.cols, args.chi, theta0=args.theta0,
                                precision="fp64", schedule=args.schedule,
                                eig_path=args.pmc_eig_path)
        sim = mpsim.Simulation(cfg)
        sites, centre = workloads.random_mps(args.rows, args.cols, args.chi, args.seed,
                                             centre=args.rows - 1)
        sim.set_state(sites, centre)
        del sites
        # calibration: an elementwise kernel that reads 1 GiB and writes 1 GiB
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.mul(x, 2.0, out=y)
        torch.cuda.synchronize()
        del x, y
        log("calibration kernel (1 GiB read, 1 GiB written) done")
        t0 = time.perf_counter()
        sim.apply_two_site(args.rows - 1, 1, 1)
        sim.sync()
        log("bulk update done in %.2fs" % (time.perf_counter() - t0))
        sim.free()
        torch.cuda.synchronize()
        print(json.dumps({"pmc_sample": True, "workload": "tfim_%dx%d_chi%d" % (
            args.rows, args.cols, args.chi), "eig_path": args.pmc_eig_path}), flush=True)
        return 0

    from paper_2511_23438_amd import workloads
    t0 = time.perf_counter()
    if args.start == "random":
        sites, centre = workloads.random_mps(args.rows, args.cols, args.chi, args.seed,
                                             centre=args.rows - 1)
    else:
        sites, centre = None, 0
    log("start state generated in %.1fs" % (time.perf_counter() - t0))

    # the roofline kernel at the workload's dominant shape: the Gram GEMMs of
    # the widest updates (side n = chi*d, K = n: 4 n^3 flops; the next widest
    # carry less than a tenth of that); other launch classes: every launch
    dblk = 2 ** ((args.cols + 1) // 2)
    nwide = min(args.chi * dblk, dblk ** args.rows)
    if args.schedule == 4:
        gram_max = 4.0 * float(min(2 * args.chi, nwide)) ** 2 * float(nwide)
    else:
        gram_max = 4.0 * float(nwide) ** 3
    min_work = 0.5 * gram_max if args.prof == "gram" else 0.0

    do_cmp = args.compare != "none" and args.compare != args.precision
    do_conc = args.instances > 0
    do_serve = args.serve_seconds > 0

    def reserve(step_s: float) -> float:
        # deadline of the headline loop: leave room for the later legs
        r = 10.0
        if do_cmp:
            r += 1.3 * step_s + 10.0
        if do_conc:
            r += 1.25 * args.instances * step_s + 20.0
        if do_serve:
            r += args.serve_seconds + 30.0
        return deadline - r

    # a saturated random start needs at most one untimed step; from the
    # product state the warmup steps grow the bonds and all of them run
    warm = min(args.warmup, 1) if sites is not None else args.warmup
    head = state_rate(sites, centre, args.rows, args.cols, args.chi, args.precision,
                      args.schedule, args.theta0, warm, args.steps, reserve(0.0), args.prof,
                      min_work, reserve_fn=reserve)
    log("headline: %.4f steps/s over %d steps" % (head["steps_per_s"], head["steps"]))
    workload = "tfim_%dx%d_chi%d" % (args.rows, args.cols, args.chi)
    roof = roofline(head["prof"], head["seconds"])
    roof["traffic"] = read_traffic(args.prof, workload)
    # the whole step against the float64 matrix peak (the standard method's
    # algorithmic flops at saturated bonds; the contractions of the reduced
    # modes are counted at that peak too)
    try:
        model = step_model_flops(args.rows, args.cols, args.chi, args.schedule)
    except Exception as e:  # a reporting extra: never lose the line for it
        log("step model skipped: %r" % (e,))
        model = None
    if model is not None and head["ms_per_step"] > 0:
        roof["step_model_flops"] = model
        roof["step_frac_fp64_peak"] = model / (head["ms_per_step"] / 1e3) / (PEAK["fp64"][0] * 1e12)
    dtype = {"fp64": "f64", "c64": "c64+f64", "bf16x3": "bf16x3+f64"}[args.precision]
    out = {
        "metric": METRIC, "value": head["steps_per_s"], "unit": "steps/s", "n_gpus": 1,
        "steps": head["steps"], "steps_requested": args.steps,
        "warmup": head["warmup"], "warmup_requested": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": workload, "rows": args.rows, "cols": args.cols,
                   "d": dblk, "sites": 2 * args.rows, "chi": args.chi,
                   "precision": args.precision, "contractions": args.precision,
                   "truncation": "f64 Gram + eigensolver, f64 fidelity",
                   "theta0": args.theta0, "J": -1.0, "h": 2.0,
                   "dt": 0.25, "trotter_order": 1,
                   "schedule": {1: "block-pair", 2: "rotating-rows",
                                4: "gate-by-gate"}[args.schedule],
                   "start": ("seeded random MPS at saturated bonds (seed %d)" % args.seed
                             if args.start == "random" else
                             "product state + %d untimed steps" % warm)},
        "roofline": roof,
        "observables": head["observables"],
        "budget_s": args.budget,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    if do_cmp and left() > 1.3 * head["ms_per_step"] / 1e3 + 10.0:
        cmp_ = state_rate(sites, centre, args.rows, args.cols, args.chi, args.compare,
                          args.schedule, args.theta0, 0, 1, time.perf_counter(), args.prof,
                          min_work)
        croof = roofline(cmp_["prof"], cmp_["seconds"])
        out["compare"] = {"precision": args.compare, "steps": cmp_["steps"],
                          "steps_per_s": cmp_["steps_per_s"], "ms_per_step": cmp_["ms_per_step"],
                          "headline_over_compare": head["steps_per_s"] / cmp_["steps_per_s"],
                          "roofline_frac": croof["frac"],
                          "observables": cmp_["observables"]}
        log("compare (%s): %.4f steps/s" % (args.compare, cmp_["steps_per_s"]))
    elif do_cmp:
        out["compare"] = {"skipped": "wall budget"}
    if do_conc and left() > 1.25 * args.instances * head["ms_per_step"] / 1e3 + 20.0:
        log("concurrent run: %d instances" % args.instances)
        out["concurrent"] = concurrent_from(sites, centre, args.rows, args.cols, args.chi,
                                           args.precision, args.schedule, args.instances)
        ref = out.get("compare", {}).get("steps_per_s") if args.compare == "fp64" else None
        if args.precision == "fp64":
            ref = head["steps_per_s"]
        if ref:
            out["concurrent"]["aggregate_over_fp64_single"] = out["concurrent"]["steps_per_s"] / ref
        log("concurrent: %.4f steps/s aggregate" % out["concurrent"]["steps_per_s"])
    elif do_conc:
        out["concurrent"] = {"skipped": "wall budget"}
    del sites
    if do_serve and left() > args.serve_seconds + 20.0:
        log("served run: %d requests, chi <= %d, admission window %.0fs" % (
            args.serve_requests, args.serve_chi_cap, args.serve_seconds))
        out["served"] = served(args.serve_seconds, args.serve_chi_cap, args.serve_requests,
                               hard_stop_s=max(5.0, min(args.serve_seconds + 5.0, left() - 40.0)))
        log("served: %s" % {k: out["served"][k] for k in ("completed", "steps_per_s",
                                                         "step_latency_ms_p50",
                                                         "step_latency_ms_p99")})
    elif do_serve:
        out["served"] = {"skipped": "wall budget"}
    if args.batched_set > 0:
        log("batched set: %d instances x %d steps" % (args.batched_set, args.batched_steps))
        out["batched_set"] = batched_set(args.batched_set, args.batched_steps,
                                         alone_sample=args.batched_alone)
        log("batched set: %s" % {k: out["batched_set"][k] for k in (
            "batched_steps_per_s", "alone_steps_per_s", "speedup",
            "bitwise_equal_alone_and_batched")})
    if args.cube:
        shape = tuple(int(v) for v in args.cube.split(","))
        log("cube run: %s chi %d" % (shape, args.cube_chi))
        out["cube"] = cube_rate(shape, args.cube_chi, args.precision, args.cube_steps, args.seed)
        log("cube: %.3f steps/s" % out["cube"]["steps_per_s"])
    if args.xy:
        shape = tuple(int(v) for v in args.xy.split(","))
        log("XY run: %s chi %d" % (shape, args.xy_chi))
        out["xy"] = xy_rate(shape, args.xy_chi, args.precision, args.xy_steps, args.seed)
        log("xy: %.3f steps/s" % out["xy"]["steps_per_s"])
    out["wall_s"] = time.perf_counter() - T_PROC0
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
