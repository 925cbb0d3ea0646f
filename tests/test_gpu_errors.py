"""Error paths of the C-ABI on the GPU, each forced from the host so that
every kernel still runs to its normal end:

* a non-finite value in a loaded state flows through the (bounded) kernels
  of the next update; the truncation bookkeeping sees a non-finite norm and
  the next synchronising call returns MPS_E_NUMERIC, after which the handle
  is failed and every call returns MPS_E_STATE;
* an allocator that refuses a request makes mps_init_product return
  MPS_E_NOMEM, leave no handle, and hand every buffer it had obtained back
  to the allocator;
* argument errors return MPS_E_INVAL and leave the handle usable and its
  state unchanged.

Plus a planted rank-deficient state (bonds larger than the Schmidt rank, so
exact zeros are kept): the evolution matches the oracle.
"""
import ctypes as C
import math

import numpy as np
import pytest

from oracle import mps as omps
from oracle.lattice import Grid
from paper_2511_23438_amd import mpsim, workloads

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _status(fn):
    try:
        fn()
    except mpsim.MpsError as e:
        return e.status
    return mpsim.MPS_OK


def test_non_finite_state_fails_the_handle():
    R, Cc, chi = 3, 4, 8
    sites, centre = workloads.random_mps(R, Cc, chi, 51)
    sites[2] = sites[2].copy()
    sites[2][0, 1, 0] = np.nan
    sim = mpsim.Simulation(mpsim.make_config(R, Cc, chi))
    sim.set_state(sites, centre)
    sim.step(1)                                       # enqueued; no error yet
    assert _status(sim.sync) == mpsim.MPS_E_NUMERIC
    assert b"non-finite" in mpsim._lib.mps_last_error(sim.h)
    for call in (lambda: sim.step(1), sim.measure, sim.fidelity, sim.sync,
                 lambda: sim.apply_two_site(0, 0, 1), sim.bond_dims,
                 lambda: sim.get_site(0), sim.truncation_log):
        assert _status(call) == mpsim.MPS_E_STATE
    sim.free()
    sim.free()                                        # idempotent


def test_allocator_refusal_returns_nomem_and_releases_everything():
    import torch
    dev = torch.cuda.current_device()
    cfg = mpsim.make_config(4, 4, 16)
    for fail_at in (1, 5, 20):
        live, count = {}, [0]

        def _alloc(ctx, nbytes, stream):
            count[0] += 1
            if count[0] == fail_at:
                return None
            p = int(torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0)))
            live[p] = nbytes
            return p

        def _free(ctx, ptr, stream):
            assert ptr in live, "freed a pointer it did not allocate"
            del live[ptr]
            torch.cuda.caching_allocator_delete(int(ptr))

        a = mpsim.ALLOC_FN(_alloc)
        f = mpsim.FREE_FN(_free)
        alloc = mpsim.MpsAllocator(None, a, f)
        h = mpsim.H()
        st = mpsim._lib.mps_init_product(C.byref(cfg), C.byref(alloc), None, C.byref(h))
        assert st == mpsim.MPS_E_NOMEM
        assert not h.value
        assert count[0] == fail_at and not live      # everything handed back
        assert b"allocation" in mpsim._lib.mps_last_error(None)


def test_argument_errors_change_nothing():
    R, Cc, chi = 3, 4, 8
    sites, centre = workloads.random_mps(R, Cc, chi, 52)
    sim = mpsim.Simulation(mpsim.make_config(R, Cc, chi))
    sim.set_state(sites, centre)
    sim.step(1)
    before = sim.measure()
    dims = sim.bond_dims()
    bad_sites = list(sites)
    bad_sites[3] = np.zeros((64, 4, 64), dtype=np.complex128)   # bond above its cap
    assert _status(lambda: sim.set_state(bad_sites, 3)) == mpsim.MPS_E_INVAL
    assert _status(lambda: sim.set_state(sites, 99)) == mpsim.MPS_E_INVAL
    assert _status(lambda: sim.apply_two_site(2 * R - 1, 0, 1)) == mpsim.MPS_E_INVAL
    assert _status(lambda: sim.apply_single_site(0, 7)) == mpsim.MPS_E_INVAL
    assert _status(lambda: sim.step(-1)) == mpsim.MPS_E_INVAL
    assert _status(lambda: sim.bond_spectrum(0)) == mpsim.MPS_E_INVAL
    after = sim.measure()
    assert sim.bond_dims() == dims
    for k in ("z", "z2", "log_fidelity", "norm"):
        assert after[k] == before[k]
    sim.step(1)                                       # still usable
    assert math.isfinite(sim.measure()["z"])
    sim.free()


def test_rank_deficient_state_keeps_exact_zeros():
    """The norm site's left index is confined to half of its bond, so the
    Schmidt rank at that bond is half the bond dimension: truncations there
    keep exact zeros (q above the rank). The run matches the oracle."""
    R, Cc, chi = 3, 4, 16
    c = 3
    sites, centre = workloads.random_mps(R, Cc, chi, 53, centre=c)
    b = sites[c].shape[0]
    A = sites[c].copy()
    A[b // 2:] = 0.0
    sites[c] = A / np.linalg.norm(A)
    sim = mpsim.Simulation(mpsim.make_config(R, Cc, chi))
    sim.set_state(sites, c)
    ora = omps.BlockMPS.from_sites(Grid(R, Cc), chi, sites, c, -1.0, 2.0, 0.25)
    assert abs(sim.measure()["z"] - ora.measure()["z"]) < TOL
    for _ in range(2):
        sim.step(1)
        ora.step()
        a, r = sim.measure(), ora.measure()
        for k in ("z", "z2", "log_fidelity"):
            assert abs(a[k] - r[k]) < TOL, (k, a[k], r[k])
    f_gpu, _ = sim.truncation_log()
    f_ora = np.array([u["f"] for u in ora.update_log])
    assert np.max(np.abs(f_gpu - f_ora)) < TOL
    assert sim.bond_dims() == ora.bond_dims()
    sim.free()


def test_batched_step_isolates_a_failing_instance():
    """One instance of a batched call holds a NaN: its handle fails at the
    next synchronising call, while the other instances of the same call keep
    exactly the results they have alone."""
    R, Cc, chi = 3, 4, 8
    good = [workloads.random_mps(R, Cc, chi, 60 + k) for k in range(3)]
    bad_sites, bad_centre = workloads.random_mps(R, Cc, chi, 64)
    bad_sites[1] = bad_sites[1].copy()
    bad_sites[1][0, 0, 0] = np.nan
    sims = []
    for sites, centre in good[:1] + [(bad_sites, bad_centre)] + good[1:]:
        s = mpsim.Simulation(mpsim.make_config(R, Cc, chi))
        s.set_state(sites, centre)
        sims.append(s)
    mpsim.apply_batched(sims, 2)
    assert _status(sims[1].sync) == mpsim.MPS_E_NUMERIC
    for k, s in enumerate([sims[0], sims[2], sims[3]]):
        sites, centre = good[k]
        ref = mpsim.Simulation(mpsim.make_config(R, Cc, chi))
        ref.set_state(sites, centre)
        ref.step(2)
        a, b = s.measure(), ref.measure()
        for key in ("z", "z2", "log_fidelity"):
            assert a[key] == b[key]
        ref.free()
    for s in sims:
        s.free()
