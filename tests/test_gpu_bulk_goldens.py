"""Parity at the metric workload's own shapes: single bulk two-site updates
of the 6x8 grid (d = 16) at Gram sides 4096 (chi = 256, one-stage
eigensolver), 8192 (chi = 512) and 16384 (chi = 1024, both two-stage), with
SWAP (direct Gram matrix of theta) and without (factored Gram matrix),
through the C-ABI, against the oracle's results stored by
tests/golden/make_bulk_goldens.py (which calls only the oracle): the
truncation fidelity f, sampled entries of the new two-site block (gauge
invariant) and the kept singular values of the new bond.

Tolerances: float64 path, 1e-10 on f and on the block entries (the block
has unit Frobenius norm); squared singular values within 1e-12 of the
largest (the library takes singular values as square roots of Gram
eigenvalues, so a singular value s carries an error of about that bound
over 2s), singular values above 1e-3 within 1e-10.
"""
import glob
import json
import os

import numpy as np
import pytest

from paper_2511_23438_amd import mpsim, workloads

pytestmark = pytest.mark.gpu
GOLDEN = sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden",
                                       "bulk_update_*.json")))


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("path", GOLDEN, ids=[os.path.basename(p)[:-5] for p in GOLDEN])
def test_bulk_update_matches_oracle(path):
    gold = json.load(open(path))
    R, C = gold["grid"]
    chi, site = gold["chi"], gold["site"]
    say("case", os.path.basename(path), "gram side", gold["gram_side"],
        "relative gap at the cut %.2e" % gold["relative_gap"])
    assert gold["relative_gap"] > 1e-6          # a unique truncation
    sites, centre = workloads.random_mps(R, C, chi, gold["seed"], centre=gold["centre"])
    say("start state generated")
    sim = mpsim.Simulation(mpsim.make_config(R, C, chi, J=gold["J"], h=gold["h"],
                                             dt=gold["dt"], theta0=0.0))
    try:
        sim.set_state(sites, centre)
        del sites
        assert sim.site_blocks()[site:site + 2] == gold["blocks"]
        sim.apply_two_site(site, bool(gold["swap"]), bool(gold["gate"]))
        sim.sync()
        f = sim.truncation_log()[0][-1]
        say("f gpu %.17g oracle %.17g" % (f, gold["f"]))
        assert abs(f - gold["f"]) < 1e-10
        assert sim.bond_dims()[site + 1] == gold["q"]
        A, B = sim.get_site(site), sim.get_site(site + 1)
        q = A.shape[2]
        Am, Bm = A.reshape(-1, q), B.reshape(q, -1)
        assert list(Am.shape[:1]) + list(Bm.shape[1:]) == gold["theta_shape"]
        smp = np.array(gold["samples"])
        r, c = smp[:, 0].astype(np.int64), smp[:, 1].astype(np.int64)
        got = np.einsum('kq,qk->k', Am[r], Bm[:, c])
        want = smp[:, 2] + 1j * smp[:, 3]
        err = np.max(np.abs(got - want))
        say("sampled block entries: max error %.2e (largest entry %.2e)" % (
            err, np.max(np.abs(want))))
        assert err < 1e-10
        del A, B, Am, Bm
        sv = sim.bond_spectrum(site + 1)
        gsv = np.array(gold["sv_kept"])
        assert len(sv) == len(gsv) == gold["q"]
        e2 = np.max(np.abs(sv ** 2 - gsv ** 2))
        big = gsv > 1e-3
        e1 = np.max(np.abs(sv[big] - gsv[big]))
        say("kept singular values: squared error %.2e, error above 1e-3 %.2e" % (e2, e1))
        assert e2 < 1e-12 and e1 < 1e-10
        assert sim.measure()["eig_suspect"] == 0
    finally:
        sim.free()


def _reduced_cases():
    out = []
    for p in GOLDEN:
        name = os.path.basename(p)
        if name.startswith("bulk_update_5x6_"):
            out.append((p, "c64"))
        elif name.startswith("bulk_update_6x8_chi256") or name.startswith("bulk_update_6x8_chi512"):
            out.append((p, "bf16x3"))
    return out


RED = _reduced_cases()


@pytest.mark.parametrize("path,prec", RED,
                         ids=["%s-%s" % (os.path.basename(p)[12:-5], q) for p, q in RED])
def test_bulk_update_reduced_precision(path, prec):
    """The same updates with the contractions in complex64 (the 5x6
    workload) or the three-term bf16 split (the 6x8 workload), FP32
    accumulation, and the float64 truncation: f, the sampled block entries
    (relative to the largest) and the kept singular values within 1e-5
    relative of the float64 oracle, each error printed."""
    gold = json.load(open(path))
    R, C = gold["grid"]
    chi, site = gold["chi"], gold["site"]
    sites, centre = workloads.random_mps(R, C, chi, gold["seed"], centre=gold["centre"])
    sim = mpsim.Simulation(mpsim.make_config(R, C, chi, J=gold["J"], h=gold["h"],
                                             dt=gold["dt"], theta0=0.0, precision=prec))
    try:
        sim.set_state(sites, centre)
        del sites
        sim.apply_two_site(site, bool(gold["swap"]), bool(gold["gate"]))
        f = sim.truncation_log()[0][-1]
        ef = abs(f - gold["f"]) / gold["f"]
        A, B = sim.get_site(site), sim.get_site(site + 1)
        q = A.shape[2]
        Am, Bm = A.reshape(-1, q), B.reshape(q, -1)
        smp = np.array(gold["samples"])
        r, c = smp[:, 0].astype(np.int64), smp[:, 1].astype(np.int64)
        got = np.einsum('kq,qk->k', Am[r], Bm[:, c])
        want = smp[:, 2] + 1j * smp[:, 3]
        et = np.max(np.abs(got - want)) / np.max(np.abs(want))
        del A, B, Am, Bm
        sv = sim.bond_spectrum(site + 1)
        gsv = np.array(gold["sv_kept"])
        es = np.max(np.abs(sv - gsv)) / gsv[0]
        say("%s %s: f rel err %.2e, block entries rel err %.2e, singular values rel err %.2e"
            % (os.path.basename(path), prec, ef, et, es))
        assert ef < 1e-5 and et < 1e-5 and es < 1e-5
        assert sim.measure()["eig_suspect"] == 0
    finally:
        sim.free()
