"""Full-size checks at the benchmark's configuration (6x8 grid, d = 16,
chi = 1024), through the C-ABI.

* The two chain-end updates (theta 256 x 16384 and 16384 x 256, so both
  Gram sides) are compared with the oracle's numpy-SVD update on the same
  seeded input: truncation fidelity, and sampled rows of the new two-site
  block A_i' A_{i+1}' (gauge invariant).
* A bulk update (Gram side 16384) is checked through properties that hold
  at any size: the new left site U is an isometry, the new centre has unit
  norm, and U spans an invariant subspace of G = theta theta^H: the
  residual G U_S - U (U^H G U_S) of sampled columns S is at rounding level
  (G applied in factored form, never formed). The oracle's own results for
  updates of this size are compared in test_gpu_bulk_goldens.py.
"""
import numpy as np
import pytest

from oracle import mps as omps
from oracle.lattice import Grid, pair_phase
from paper_2511_23438_amd import mpsim, workloads

pytestmark = pytest.mark.gpu
J, H, DT = -1.0, 2.0, 0.25


def say(*a):
    print(*a, flush=True)


def _theta(sites, pos, i, gate, grid):
    A, B = sites[i], sites[i + 1]
    b0, d1, b1 = A.shape
    _, d2, b2 = B.shape
    M = (A.reshape(b0 * d1, b1) @ B.reshape(b1, d2 * b2)).reshape(b0, d1, d2, b2)
    if gate:
        M = M * pair_phase(grid, pos[i], pos[i + 1], J, DT)[None, :, :, None]
    return M.reshape(b0 * d1, d2 * b2)


@pytest.mark.parametrize("i", [1, 9])
def test_chain_end_updates_match_oracle(i):
    sites, centre = workloads.random_mps(6, 8, 1024, 2024 + i, centre=i)
    say("random state built, update at site", i)
    grid = Grid(6, 8)
    sim = mpsim.Simulation(mpsim.make_config(6, 8, 1024, theta0=0.0))
    sim.set_state(sites, centre)
    sim.apply_two_site(i, 0, 1)
    f_gpu = sim.truncation_log()[0][-1]
    Ai, Aj = sim.get_site(i), sim.get_site(i + 1)
    sim.free()
    say("gpu update done", f_gpu)
    ora = omps.BlockMPS.from_sites(grid, 1024, sites, centre, J, H, DT)
    f_ora = ora.apply_u2(i, False, True)
    say("oracle update done", f_ora, "gap", ora.update_log[-1]["gap"])
    assert abs(f_gpu - f_ora) < 1e-10
    rng = np.random.default_rng(5)
    b0, d1, q = Ai.shape
    rows = rng.choice(b0 * d1, 48, replace=False)
    Bi, Bj = ora.sites[i], ora.sites[i + 1]
    got = Ai.reshape(b0 * d1, q)[rows] @ Aj.reshape(q, -1)
    ref = Bi.reshape(b0 * d1, -1)[rows] @ Bj.reshape(Bj.shape[0], -1)
    err = np.max(np.abs(got - ref))
    say("max sampled block error", err)
    assert err < 1e-10


def test_bulk_update_gram16384_spans_an_invariant_subspace():
    i = 5
    sites, centre = workloads.random_mps(6, 8, 1024, 2030, centre=i)
    say("random state built")
    grid = Grid(6, 8)
    ora = omps.BlockMPS.from_sites(grid, 1024, sites, centre, J, H, DT)
    pos = grid.snake()
    sim = mpsim.Simulation(mpsim.make_config(6, 8, 1024, theta0=0.0))
    sim.set_state(sites, centre)
    sim.apply_two_site(i, 0, 1)
    f_gpu = sim.truncation_log()[0][-1]
    dims = sim.bond_dims()
    Ai, Aj = sim.get_site(i), sim.get_site(i + 1)
    sim.free()
    assert dims[i + 1] == 1024
    b0, d1, q = Ai.shape
    U = Ai.reshape(b0 * d1, q)
    rng = np.random.default_rng(6)
    cols = rng.choice(q, 64, replace=False)
    G = U[:, cols].conj().T @ U[:, cols]
    assert np.max(np.abs(G - np.eye(64))) < 1e-12
    Cn = Aj.reshape(q, -1)
    assert abs(np.linalg.norm(Cn) - 1.0) < 1e-12
    # theta before the update, in factored form (centre on site i)
    A = ora.sites[i].reshape(b0 * d1, -1)
    B = ora.sites[i + 1]
    ph = pair_phase(grid, pos[i], pos[i + 1], J, DT)
    b1, d2, b2 = B.shape

    def M_mul(x):
        # theta[(a,s1),(s2,g)] = sum_b A[(a,s1),b] B[b,s2,g] ph[s1,s2]
        xx = x.reshape(d2, b2, -1)
        BX = np.einsum('bsg,sgk->bsk', B, xx)
        AB = np.einsum('xb,bsk->xsk', A, BX).reshape(b0, d1, d2, -1)
        return (AB * ph[None, :, :, None]).sum(axis=2).reshape(b0 * d1, -1)

    def MH_mul(y):
        Y = (y.reshape(b0, d1, 1, -1) * np.conj(ph)[None, :, :, None]).reshape(b0 * d1, d2, -1)
        AY = np.einsum('xb,xsk->bsk', A.conj(), Y)
        return np.einsum('bsg,bsk->sgk', B.conj(), AY).reshape(d2 * b2, -1)

    # invariant subspace: G U_S - U (U^H G U_S) for 64 sampled columns S of U,
    # with G = theta theta^H applied as theta (theta^H x)
    say("invariant-subspace residual")
    US = U[:, cols]
    GUS = M_mul(MH_mul(US))
    res = GUS - U @ (U.conj().T @ GUS)
    rel = np.linalg.norm(res) / np.linalg.norm(GUS)
    say("relative residual %.2e" % rel)
    assert rel < 1e-10
