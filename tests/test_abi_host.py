"""Host-side checks of the C-ABI library (no GPU needed): every symbol the
header declares is exported, the step schedule equals the oracle's own,
invalid configurations are rejected, and the admission footprint is sane."""
import math
import os
import re

import numpy as np
import pytest

from oracle.lattice import Grid
from oracle.schedule import schedule as oracle_schedule
from paper_2511_23438_amd import mpsim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in sorted(os.listdir(inc)):
        if f.endswith(".h"):
            txt = re.sub(r"/\*.*?\*/", "", open(os.path.join(inc, f)).read(), flags=re.S)
            names |= set(re.findall(r"\b(mps_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


def test_header_symbols_exported():
    names = _declared()
    assert len(names) >= 18 and "mps_measure_static" in names
    for n in names:
        assert hasattr(mpsim._lib, n), n
        assert n in mpsim.EXPORTED, n


@pytest.mark.parametrize("R,C", [(4, 4), (5, 6), (6, 8), (7, 8), (3, 3), (4, 5), (1, 4),
                                 (2, 3), (5, 5)])
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("sched", [1, 2, 3, 4])
def test_schedule_equals_oracle(R, C, order, sched):
    cfg = mpsim.make_config(R, C, 16, order=order, schedule=sched)
    got = mpsim.schedule_dump(cfg, 3)
    ref = oracle_schedule(Grid(R, C), 3, order, sched)
    _same_ops(got, ref)


def _same_ops(got, ref):
    assert len(got) == len(ref)
    for row, op in zip(got, ref):
        if op[0] == "U2":
            assert tuple(row) == (1, op[1], op[2], op[3], op[4], op[5])
        elif op[0] == "ZZ":
            assert tuple(row) == (3, op[1], op[2], op[3], op[4], 0)
        else:
            assert tuple(row[:4]) == (2, op[1], op[2], op[3])


@pytest.mark.parametrize("shape", [(2, 2, 3), (3, 3, 3), (2, 3, 4), (1, 2, 5), (4, 4, 4)])
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("sched", [3, 4])
def test_cube_schedule_equals_oracle(shape, order, sched):
    """Cube with one qubit per site: the C++ planner's route-and-return and
    gate-by-gate lists equal the oracle's."""
    from oracle.lattice import Cube
    lx, ly, lz = shape
    cfg = mpsim.make_config(lx, ly, 8, order=order, schedule=sched, layers=lz, periodic=False)
    got = mpsim.schedule_dump(cfg, 2)
    ref = oracle_schedule(Cube(lx, ly, lz), 2, order, sched)
    _same_ops(got, ref)


@pytest.mark.parametrize("kw,status", [
    (dict(cols=1), mpsim.MPS_E_INVAL), (dict(rows=0), mpsim.MPS_E_INVAL),
    (dict(cols=9), mpsim.MPS_E_UNSUPPORTED), (dict(chi=0), mpsim.MPS_E_INVAL),
    (dict(order=3), mpsim.MPS_E_INVAL), (dict(schedule=5), mpsim.MPS_E_INVAL),
    (dict(layers=2, schedule=1), mpsim.MPS_E_INVAL),
    (dict(rows=8, cols=8, layers=8, schedule=3), mpsim.MPS_E_UNSUPPORTED)])
def test_invalid_config_rejected(kw, status):
    args = dict(rows=4, cols=4, chi=16)
    args.update(kw)
    cfg = mpsim.make_config(**args)
    with pytest.raises(mpsim.MpsError) as e:
        mpsim.footprint_bytes(cfg)
    assert e.value.status == status
    with pytest.raises(mpsim.MpsError):
        mpsim.schedule_dump(cfg, 1)


def test_footprint_monotone_and_fits():
    fp = [mpsim.footprint_bytes(mpsim.make_config(6, 8, chi)) for chi in (256, 512, 1024)]
    assert fp[0] < fp[1] < fp[2]
    # sites alone: 7 bulk sites of chi*16*chi complex128
    assert fp[2] > 7 * 1024 * 16 * 1024 * 16
    assert fp[2] < 288 * 2 ** 30


def test_eig_batch_bounds_the_inverse_iteration_workspace():
    """6x8, chi = 1024 (Gram side 16384, two-stage): 256 vectors per band
    inverse-iteration launch instead of 1024 saves the LU rows (99 complex
    per Gram row) of 768 vectors; out-of-range values are rejected."""
    fp = {b: mpsim.footprint_bytes(mpsim.make_config(6, 8, 1024, schedule=2, eig_batch=b))
          for b in (0, 1024, 256)}
    assert fp[0] == fp[1024]
    assert fp[1024] - fp[256] == 768 * 16384 * 99 * 16
    for bad in (-1, 1025):
        with pytest.raises(mpsim.MpsError) as e:
            mpsim.footprint_bytes(mpsim.make_config(6, 8, 1024, eig_batch=bad))
        assert e.value.status == mpsim.MPS_E_INVAL


@pytest.mark.parametrize("shape", [(2, 3), (3, 3), (4, 4), (1, 5), (6, 6), (5, 4)])
def test_xy_schedule_equals_oracle(shape):
    """XY model: the C++ planner's sublayer / route-and-return list equals the
    oracle's for two steps."""
    from oracle.xy import XYGrid, xy_step_ops
    g = XYGrid(*shape)
    cfg = mpsim.make_xy_config(shape[0], shape[1], 16)
    got = mpsim.schedule_dump(cfg, 2)
    pos = g.snake()
    ref = xy_step_ops(g, pos) + xy_step_ops(g, pos)
    assert pos == g.snake()
    _same_ops(got, ref)


@pytest.mark.parametrize("field,value", [("periodic", 1), ("trotter_order", 1), ("layers", 2),
                                         ("schedule", 1), ("model", 2)])
def test_xy_invalid_configs(field, value):
    cfg = mpsim.make_xy_config(3, 3, 8)
    setattr(cfg, field, value)
    with pytest.raises(mpsim.MpsError) as e:
        mpsim.schedule_dump(cfg, 1)
    assert e.value.status == mpsim.MPS_E_INVAL


def test_xy_footprint():
    fp = mpsim.footprint_bytes(mpsim.make_xy_config(6, 6, 256))
    assert 0 < fp < 8 * 2 ** 30


def test_eigh_top_rejects_bad_arguments():
    """mps_eigh_top validates its arguments on the host before any device
    work: q outside 1..n or an unknown eigensolver path."""
    G = np.eye(4, dtype=np.complex128)
    for q, path in ((0, 1), (5, 1), (2, 3)):
        with pytest.raises(mpsim.MpsError) as e:
            mpsim.eigh_top(G, q, eig_path=path)
        assert e.value.status == mpsim.MPS_E_INVAL


def test_step_flop_model():
    """The whole-step work model of bench.py (standard two-site updates at
    saturated bonds, from the planner's own schedule): the largest term is
    the Gram matrix and reduction of the 16384-wide updates, so halving chi
    at 6x8 divides the model by about 8; the gate-by-gate schedule has no
    model. Block-pair schedule at 6x8, chi = 1024: 1.37e15 flops."""
    import bench
    f = {chi: bench.step_model_flops(6, 8, chi, 1) for chi in (512, 1024)}
    assert abs(f[1024] / 1.367e15 - 1) < 0.01
    assert 6.0 < f[1024] / f[512] < 10.0
    f2 = bench.step_model_flops(6, 8, 1024, 2)
    assert 0.5 * f[1024] < f2 < f[1024]        # rotating rows: fewer, narrower updates
    assert bench.step_model_flops(6, 8, 1024, 4) is None
