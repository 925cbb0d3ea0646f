"""Steps captured as HIP graphs (config field graphs = 1) against the same
steps launched directly, through the C-ABI: bit for bit equal after every
step, with the program's own eager work (measurements, which synchronise)
between the replays; graphs are captured once per shape signature and
replayed; ineligible configurations run directly; and a symmetry-free
truncating run in graph mode matches the oracle."""
import numpy as np
import pytest

from oracle import mps as omps
from oracle.lattice import Grid
from paper_2511_23438_amd import mpsim, workloads

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _stream():
    import torch
    return torch.cuda.Stream()


def _sim(cfg):
    import torch
    st = _stream()
    with torch.cuda.stream(st):
        return mpsim.Simulation(cfg, stream=st.cuda_stream), st


@pytest.mark.parametrize("R,C,chi,prec,order,schedule", [
    (4, 5, 32, "c64", 1, 1), (5, 6, 64, "fp64", 1, 1), (4, 4, 16, "fp64", 2, 2),
    (3, 5, 24, "bf16x3", 1, 3)])
def test_graph_steps_equal_direct_steps(R, C, chi, prec, order, schedule):
    steps = 8
    a, sa = _sim(mpsim.make_config(R, C, chi, theta0=0.7, precision=prec, order=order,
                                   schedule=schedule, graphs=1))
    b, sb = _sim(mpsim.make_config(R, C, chi, theta0=0.7, precision=prec, order=order,
                                   schedule=schedule, graphs=0))
    for s_ in range(steps):
        a.step(1)
        b.step(1)
        oa, ob = a.measure(), b.measure()
        for k in ("z", "z2", "log_fidelity", "norm"):
            assert oa[k] == ob[k], (s_, k, oa[k], ob[k])
        assert a.bond_dims() == b.bond_dims() and a.site_blocks() == b.site_blocks()
    fa, ga = a.truncation_log()
    fb, gb = b.truncation_log()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    cap, rep = a.graph_stats()
    print(R, C, chi, prec, "captured", cap, "replayed", rep)
    assert cap + rep == steps and rep > 0
    assert b.graph_stats() == (0, 0)
    a.free()
    b.free()


def test_graph_replays_after_set_state_and_two_site_calls():
    """Loading a new state and single updates outside steps leave the
    captured graphs valid: later replays still equal direct launches."""
    R, C, chi = 4, 4, 12
    sites, centre = workloads.random_mps(R, C, chi, 61)
    a, _ = _sim(mpsim.make_config(R, C, chi, graphs=1))
    b, _ = _sim(mpsim.make_config(R, C, chi, graphs=0))
    for sim in (a, b):
        sim.set_state(sites, centre)
        sim.step(3)
    c1, r1 = a.graph_stats()
    assert c1 >= 2 and c1 + r1 == 3
    for sim in (a, b):
        sim.set_state(sites, centre)      # the same signatures again: replays
        sim.step(3)
    assert a.graph_stats() == (c1, r1 + 3)
    for sim in (a, b):
        sim.apply_two_site(2, 1, 1)       # blocks moved: new signatures
        sim.step(2)
    oa, ob = a.measure(), b.measure()
    for k in ("z", "z2", "log_fidelity"):
        assert oa[k] == ob[k]
    assert a.bond_dims() == b.bond_dims() and a.site_blocks() == b.site_blocks()
    assert a.graph_stats()[0] > c1
    a.free()
    b.free()


def test_graph_mode_truncating_parity_with_oracle():
    R, C, chi, seed = 4, 4, 16, 62
    sites, centre = workloads.random_mps(R, C, chi, seed)
    sim, _ = _sim(mpsim.make_config(R, C, chi, graphs=1))
    sim.set_state(sites, centre)
    ora = omps.BlockMPS.from_sites(Grid(R, C), chi, sites, centre, -1.0, 2.0, 0.25)
    for _ in range(4):
        sim.step(1)
        ora.step()
        a, r = sim.measure(), ora.measure()
        for k in ("z", "z2", "log_fidelity"):
            assert abs(a[k] - r[k]) < TOL
    f_gpu, _ = sim.truncation_log()
    f_ora = np.array([u["f"] for u in ora.update_log])
    assert np.max(np.abs(f_gpu - f_ora)) < TOL
    assert sim.graph_stats()[1] > 0
    sim.free()


def test_ineligible_configurations_run_directly():
    """The two-stage eigensolver (forced here) replays a graph of its own, so
    such handles launch their steps directly; so does a handle on the null
    stream and one timing a launch class."""
    a, _ = _sim(mpsim.make_config(3, 4, 16, graphs=1, eig_path=2))
    a.step(2)
    assert a.graph_stats() == (0, 0)
    a.free()
    b = mpsim.Simulation(mpsim.make_config(3, 4, 16, graphs=1), stream=0)
    b.step(2)
    assert b.graph_stats() == (0, 0)
    b.free()
    c, _ = _sim(mpsim.make_config(3, 4, 16, graphs=1))
    c.profile("gemm")
    c.step(2)
    c.profile("off")
    assert c.graph_stats() == (0, 0)
    c.step(2)
    assert c.graph_stats()[0] > 0
    c.free()
