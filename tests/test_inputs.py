"""Seeded input generators: shapes, determinism and canonical form of the
random start states used as symmetry-free parity inputs."""
import numpy as np
import pytest

from oracle import mps as omps
from oracle.lattice import Grid
from paper_2511_23438_amd import workloads


@pytest.mark.parametrize("R,C,chi,centre", [(3, 4, 16, None), (4, 4, 8, 3), (3, 5, 24, 0)])
def test_random_mps_is_mixed_canonical_and_normalised(R, C, chi, centre):
    sites, c = workloads.random_mps(R, C, chi, 5, centre=centre)
    assert len(sites) == 2 * R
    assert [a.shape[1] for a in sites] == workloads.snake_dims(R, C)
    for p, A in enumerate(sites):
        b0, d, b1 = A.shape
        if p < c:
            M = A.reshape(b0 * d, b1)
            assert np.allclose(M.conj().T @ M, np.eye(b1), atol=1e-12)
        elif p > c:
            M = A.reshape(b0, d * b1)
            assert np.allclose(M @ M.conj().T, np.eye(b0), atol=1e-12)
    m = omps.BlockMPS.from_sites(Grid(R, C), chi, sites, c, -1.0, 2.0, 0.25)
    assert abs(m.measure()["norm"] - 1) < 1e-12
    s2, _ = workloads.random_mps(R, C, chi, 5, centre=centre)
    assert all(np.array_equal(a, b) for a, b in zip(sites, s2))


def test_traces_are_seeded():
    a = workloads.serving_trace(20, seed=3)
    b = workloads.serving_trace(20, seed=3)
    assert [(r.arrival_s, r.inst.rows, r.inst.cols, r.inst.chi) for r in a] == \
           [(r.arrival_s, r.inst.rows, r.inst.cols, r.inst.chi) for r in b]
    assert all(64 <= r.inst.chi <= 1024 and 4 <= r.inst.rows <= 7 for r in a)
    insts = workloads.batched(64)
    assert {(i.rows, i.cols) for i in insts} <= {(4, 5), (5, 5), (5, 6), (6, 6)}
