"""Serving and batching: continuous admission by device footprint, device
overlap of independent instances, and results identical alone and in a mix."""
import math

import numpy as np
import pytest

from paper_2511_23438_amd import mpsim, serve, workloads

pytestmark = pytest.mark.gpu


def _small_trace(n=8, seed=7):
    g = workloads.rng(seed)
    out, t = [], 0.0
    for k in range(n):
        t += float(g.exponential(1 / 50.0))
        r, c = int(g.integers(3, 5)), int(g.integers(3, 6))
        inst = workloads.Instance(r, c, int(g.choice([8, 16, 32])), J=float(g.uniform(-1.5, -0.5)),
                                  h=float(g.uniform(0.5, 3)), theta0=float(g.uniform(0, math.pi / 2)),
                                  steps=int(g.integers(2, 5)), precision="fp64", name="t%d" % k)
        out.append(workloads.Request(t, inst))
    return out


def test_served_results_equal_alone_and_admission_respects_budget():
    trace = _small_trace()
    sizes = [mpsim.footprint_bytes(mpsim.config_from_instance(r.inst)) for r in trace]
    budget = int(2.5 * max(sizes))          # forces queueing
    srv = serve.Server(budget, max_active=4, seed=100)
    out = srv.run(trace)
    assert out["completed"] == len(trace)
    assert out["peak_bytes"] <= budget
    assert out["peak_active"] >= 2          # instances overlapped on the device
    for res in out["results"]:
        alone = serve.run_alone(res.inst, seed=100 + res.rid)
        for k in ("z", "z2", "log_fidelity"):
            assert res.obs[k] == alone[k], (k, res.obs[k], alone[k])
        assert len(res.step_ms) == res.inst.steps
    assert out["step_latency_ms_p99"] >= out["step_latency_ms_p50"] > 0


def test_batched_call_equals_sequential():
    insts = workloads.batched(6, seed=3)
    for i in insts:
        i.precision = "fp64"
        i.chi = min(i.chi, 32)
    sims = [mpsim.Simulation(mpsim.config_from_instance(i, seed=k)) for k, i in enumerate(insts)]
    mpsim.apply_batched(sims, 2)
    got = [s.measure() for s in sims]
    for k, (i, o) in enumerate(zip(insts, got)):
        s2 = mpsim.Simulation(mpsim.config_from_instance(i, seed=k))
        s2.step(2)
        ref = s2.measure()
        assert o["z"] == ref["z"] and o["z2"] == ref["z2"]
        assert o["log_fidelity"] == ref["log_fidelity"]
