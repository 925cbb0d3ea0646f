"""Serving and batching: continuous admission by device footprint, device
overlap of independent instances, and results identical alone and in a mix."""
import math

import numpy as np
import pytest

from paper_2511_23438_amd import mpsim, serve, workloads

pytestmark = pytest.mark.gpu


def _small_trace(n=8, seed=7, chis=(8, 16, 32), rows=(3, 5), cols=(3, 6)):
    g = workloads.rng(seed)
    out, t = [], 0.0
    for k in range(n):
        t += float(g.exponential(1 / 50.0))
        r, c = int(g.integers(*rows)), int(g.integers(*cols))
        inst = workloads.Instance(r, c, int(g.choice(chis)), J=float(g.uniform(-1.5, -0.5)),
                                  h=float(g.uniform(0.5, 3)), theta0=float(g.uniform(0, math.pi / 2)),
                                  steps=int(g.integers(2, 5)), precision="fp64", name="t%d" % k)
        out.append(workloads.Request(t, inst))
    return out


@pytest.mark.parametrize("chis,rows,cols", [((8, 16, 32), (3, 5), (3, 6)),
                                             ((64, 128), (4, 6), (4, 7))])
def test_served_results_equal_alone_and_admission_respects_budget(chis, rows, cols):
    trace = _small_trace(chis=chis, rows=rows, cols=cols)
    sizes = [mpsim.footprint_bytes(mpsim.config_from_instance(r.inst)) for r in trace]
    budget = int(2.5 * max(sizes))          # forces queueing
    srv = serve.Server(budget, max_active=4, seed=100)
    out = srv.run(trace)
    assert out["completed"] == len(trace), out["errors"]
    assert out["peak_bytes"] <= budget
    assert out["peak_active"] >= 2          # instances overlapped on the device
    print("served: %d requests, chi %s, peak %d active, p50 %.1f ms p99 %.1f ms" % (
        len(trace), sorted({r.inst.chi for r in trace}), out["peak_active"],
        out["step_latency_ms_p50"], out["step_latency_ms_p99"]))
    for res in out["results"]:
        alone = serve.run_alone(res.inst, seed=100 + res.rid)
        for k in ("z", "z2", "log_fidelity"):
            assert res.obs[k] == alone[k], (k, res.obs[k], alone[k])
        assert len(res.step_ms) == res.inst.steps
    assert out["step_latency_ms_p99"] >= out["step_latency_ms_p50"] > 0


def test_served_hard_stop_counts_completed_steps():
    """A hard stop ends every instance after its current step; the steps it
    completed are reported and nothing is left running."""
    trace = _small_trace(n=4, seed=11, chis=(64,), rows=(4, 5), cols=(4, 6))
    for r in trace:
        r.inst.steps = 400
    srv = serve.Server(1 << 40, max_active=4, seed=5)
    out = srv.run(trace, time_limit_s=0.5, hard_stop_s=2.0)
    assert out["completed"] == 0 and out["stopped"] == out["admitted"] > 0
    assert 0 < out["total_steps"] < 400 * out["admitted"]
    assert not out["errors"]


def test_served_invalid_request_is_rejected_and_the_rest_served():
    """A request with an invalid configuration (chi = 0) is rejected on
    arrival; the requests around it are served and match their runs alone."""
    trace = _small_trace(n=4, seed=13)
    trace[1].inst.chi = 0
    srv = serve.Server(1 << 40, max_active=4, seed=200)
    out = srv.run(trace)
    assert out["rejected"] == 1 and out["completed"] == 3 and not out["errors"]
    for res in out["results"]:
        alone = serve.run_alone(res.inst, seed=200 + res.rid)
        assert res.obs["z"] == alone["z"]


@pytest.mark.parametrize("chi_cap,precision", [(32, "fp64"), (256, "c64")])
def test_batched_call_equals_sequential(chi_cap, precision):
    """The batched entry point on the batched workload set (grids 4x5..6x6,
    d 4 and 8, ragged for odd widths, chi up to the cap) gives every
    instance bit for bit the result it has alone."""
    insts = workloads.batched(6, seed=3)
    for i in insts:
        i.precision = precision
        i.chi = min(i.chi, chi_cap)
    sims = [mpsim.Simulation(mpsim.config_from_instance(i, seed=k)) for k, i in enumerate(insts)]
    mpsim.apply_batched(sims, 2)
    got = [s.measure() for s in sims]
    for k, (i, o) in enumerate(zip(insts, got)):
        s2 = mpsim.Simulation(mpsim.config_from_instance(i, seed=k))
        s2.step(2)
        ref = s2.measure()
        assert o["z"] == ref["z"] and o["z2"] == ref["z2"]
        assert o["log_fidelity"] == ref["log_fidelity"]
