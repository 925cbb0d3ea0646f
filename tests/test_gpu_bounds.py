"""Operand extent checks (mps_debug_check_bounds) switched on over every
launch path of the library: before each complex GEMM, reflector extraction,
QR and eigensolver launch the host checks that every operand's first and
last accessed element lie inside the one library buffer that holds its
base address. A failing check launches nothing and fails the call, so each
run below passing means no operand of its launches reaches outside its
buffer: one- and two-stage eigensolvers, both Gram paths, the three
arithmetic modes, the gate-by-gate schedule, the XY model, the measurement,
bond spectra, the allocation-free measurement, and the 16384-wide updates
of the 6x8, chi = 1024 workload with and without SWAP.
"""
import numpy as np
import pytest

from paper_2511_23438_amd import mpsim, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture
def checks_on():
    mpsim.debug_check_bounds(True)
    try:
        yield
    finally:
        mpsim.debug_check_bounds(False)


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("case", [
    dict(rows=4, cols=4, chi=16),
    dict(rows=4, cols=4, chi=16, schedule=4, theta0=0.6),
    dict(rows=4, cols=4, chi=16, schedule=2, order=2),
    dict(rows=5, cols=6, chi=64, precision="c64"),
    dict(rows=5, cols=6, chi=64, precision="bf16x3"),
    dict(rows=6, cols=8, chi=128, eig_path=2, eig_batch=7),
    dict(rows=6, cols=8, chi=128, eig_path=2, precision="bf16x3", schedule=2),
    dict(rows=3, cols=5, chi=24, eig_path=2),
])
def test_checked_steps_from_random_states(checks_on, case):
    case = dict(case)
    R, C, chi = case.pop("rows"), case.pop("cols"), case.pop("chi")
    say("checked step", R, C, chi, case)
    sites, centre = workloads.random_mps(R, C, chi, 61)
    case.setdefault("theta0", 0.0)
    sim = mpsim.Simulation(mpsim.make_config(R, C, chi, **case))
    if case.get("schedule", 1) != 4:
        sim.set_state(sites, centre)
    sim.step(2)
    o = sim.measure()
    assert np.isfinite(o["z"]) and o["eig_suspect"] == 0
    sim.bond_spectrum(R)
    sim.free()


def test_checked_xy_and_product_start(checks_on):
    sim = mpsim.Simulation(mpsim.make_xy_config(3, 4, 8))
    sim.step(1)
    assert np.isfinite(sim.measure()["z"])
    sim.free()
    sim = mpsim.Simulation(mpsim.make_config(3, 4, 8, eig_path=1))
    sim.step(2)
    assert np.isfinite(sim.measure()["z"])
    sim.free()


def test_checked_static_measurement(checks_on):
    import torch
    sites, centre = workloads.random_mps(3, 4, 8, 62)
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in sites]
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    mpsim.measure_static([1] + [a.shape[2] for a in sites], [a.shape[1] for a in sites],
                         [t.data_ptr() for t in dev], stream.cuda_stream, out.data_ptr())
    torch.cuda.synchronize()
    assert abs(out[0].item() - 1.0) < 1e-12


def test_checked_wide_updates_6x8_chi1024(checks_on):
    i = 5
    sites, centre = workloads.random_mps(6, 8, 1024, 2031, centre=i)
    say("random state built")
    sim = mpsim.Simulation(mpsim.make_config(6, 8, 1024, theta0=0.0, precision="bf16x3"))
    sim.set_state(sites, centre)
    sim.apply_two_site(i, 1, 1)        # SWAP: direct Gram matrix, side 16384
    say("update with SWAP done")
    sim.apply_two_site(i, 0, 1)        # no SWAP: factored Gram matrix
    say("update without SWAP done")
    o = sim.measure()
    assert np.isfinite(o["z"]) and o["eig_suspect"] == 0
    sim.free()
