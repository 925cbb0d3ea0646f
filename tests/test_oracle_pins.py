"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these checks re-runs the oracle's own formula: each compares it with
an independent construction (dense Hamiltonian and matrix exponentials), a
closed form (single-qubit precession at J = 0, conservation at h = 0, the
product state at s = 0), exact state-vector evolution (full bond dimension),
or a property the paper states (the kept/discarded decomposition of a
truncation, unit norm, monotone fidelity).
"""
import copy
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import estimators, mps, statevector
from oracle.lattice import Grid, pair_coupled
from oracle.schedule import step_ops

J, H, DT = -1.0, 2.0, 0.25


# --------------------------------------------------------------------------
# independent dense construction of H_ZZ and H_X (Kronecker products)
def _dense_h(R, C):
    n = R * C
    I2 = np.eye(2)
    Zm = np.diag([1.0, -1.0])
    Xm = np.array([[0.0, 1.0], [1.0, 0.0]])

    def op(single, q):
        out = np.ones((1, 1))
        for k in range(n):
            out = np.kron(out, single if k == q else I2)
        return out

    pairs = set()
    for r in range(R):
        for c in range(C):
            for (r2, c2) in (((r + 1) % R, c), (r, (c + 1) % C)):
                a, b = r * C + c, r2 * C + c2
                if a != b:
                    pairs.add((min(a, b), max(a, b)))
    hzz = sum(op(Zm, a) @ op(Zm, b) for (a, b) in pairs)
    hx = sum(op(Xm, q) for q in range(n))
    return hzz, hx, len(pairs)


@pytest.mark.parametrize("R,C", [(2, 2), (2, 3), (3, 3), (1, 4)])
@pytest.mark.parametrize("order", [1, 2])
def test_statevector_matches_dense_expm(R, C, order):
    hzz, hx, npairs = _dense_h(R, C)
    g = Grid(R, C)
    assert len(g.zz_bonds()) == npairs
    th = 0.37
    if order == 1:
        U = scipy.linalg.expm(-1j * DT * H * hx) @ scipy.linalg.expm(-1j * DT * J * hzz)
    else:
        half = scipy.linalg.expm(-0.5j * DT * H * hx)
        U = half @ scipy.linalg.expm(-1j * DT * J * hzz) @ half
    psi = np.ones(1)
    for _ in range(R * C):
        psi = np.kron(psi, [math.cos(th / 2), math.sin(th / 2)])
    sv = statevector.StateVector(g, th, J, H, DT, order)
    for _ in range(3):
        psi = U @ psi
        sv.step()
    assert np.max(np.abs(sv.psi - psi)) < 1e-12


def test_bond_counts_periodic():
    # 2n nearest-neighbour bonds on a periodic grid with R, C >= 3
    for (R, C) in [(4, 4), (5, 6), (6, 8), (7, 8), (3, 3)]:
        assert len(Grid(R, C).zz_bonds()) == 2 * R * C


# --------------------------------------------------------------------------
@pytest.mark.parametrize("R,C", [(3, 3), (4, 4), (2, 5)])
@pytest.mark.parametrize("th", [0.0, 0.3, math.pi / 18, 2.0])
def test_t1_initial_state(R, C, th):
    g = Grid(R, C)
    n = g.n
    m = mps.BlockMPS(g, 8, th, J, H, DT).measure()
    s = statevector.StateVector(g, th, J, H, DT).measure()
    for o in (m, s):
        assert abs(o["z"] - math.cos(th)) < 1e-14
        assert abs(o["z2"] - (1 / n + (1 - 1 / n) * math.cos(th) ** 2)) < 1e-14
    assert m["fidelity"] == 1.0


@pytest.mark.parametrize("R,C,chi", [(3, 3, 4), (4, 4, 2), (3, 4, 16)])
def test_t2_no_coupling_precession(R, C, chi):
    g = Grid(R, C)
    n = g.n
    th = 0.41
    m = mps.BlockMPS(g, chi, th, 0.0, H, DT)
    sv = statevector.StateVector(g, th, 0.0, H, DT)
    for s in range(1, 6):
        m.step()
        sv.step()
        zc = math.cos(th) * math.cos(2 * H * DT * s)
        z2c = 1 / n + (1 - 1 / n) * (math.cos(th) * math.cos(2 * H * DT * s)) ** 2
        for o in (m.measure(), sv.measure()):
            assert abs(o["z"] - zc) < 1e-12
            assert abs(o["z2"] - z2c) < 1e-12
        assert abs(m.log_fidelity) < 1e-12
    for b in range(1, len(m.sites)):
        sv_b = m.bond_spectrum(b)
        assert np.sum(sv_b > 1e-10) == 1      # product state: Schmidt rank 1


@pytest.mark.parametrize("th", [0.0, 0.7])
def test_t3_no_field_conserves(th):
    g = Grid(3, 4)
    m = mps.BlockMPS(g, 64, th, J, 0.0, DT)
    z0 = m.measure()
    for _ in range(3):
        m.step()
        o = m.measure()
        assert abs(o["z"] - z0["z"]) < 1e-10
        assert abs(o["z2"] - z0["z2"]) < 1e-10
    if th == 0.0:
        assert abs(o["z"] - 1) < 1e-12 and abs(o["z2"] - 1) < 1e-12
        assert abs(o["fidelity"] - 1) < 1e-12


def _perm_statevector(g, pos, psi):
    """Reshape a dense state into chain order (blocks of pos, in-block MSB first)."""
    n = g.n
    order = [q for b in pos for q in g.block_qubits(b)]
    t = psi.reshape([2] * n).transpose(order)
    return t.reshape(-1)


@pytest.mark.parametrize("R,C,chi,steps,order", [
    (3, 3, 64, 4, 1), (2, 4, 16, 4, 1), (4, 4, 256, 3, 1), (3, 4, 64, 3, 2),
    (2, 3, 8, 5, 2)])
def test_t4_full_bond_dimension_is_exact(R, C, chi, steps, order):
    g = Grid(R, C)
    th = 0.6
    m = mps.BlockMPS(g, chi, th, J, H, DT, order)
    sv = statevector.StateVector(g, th, J, H, DT, order)
    for _ in range(steps):
        m.step()
        sv.step()
        a, b = m.measure(), sv.measure()
        assert abs(a["z"] - b["z"]) < 1e-10
        assert abs(a["z2"] - b["z2"]) < 1e-10
        assert abs(a["log_fidelity"]) < 1e-12
        psi = m.to_statevector()
        assert abs(abs(np.vdot(sv.psi, psi)) ** 2 - 1) < 1e-10
    # bond spectra equal the Schmidt values of the exact state in chain order
    chain = _perm_statevector(g, m.pos, sv.psi)
    dims = [g.block_dim(b) for b in m.pos]
    for bond in range(1, len(dims)):
        left = int(np.prod(dims[:bond]))
        ref = np.linalg.svd(chain.reshape(left, -1), compute_uv=False)
        got = m.bond_spectrum(bond)
        k = min(len(ref), len(got))
        assert np.max(np.abs(ref[:k] - got[:k])) < 1e-10
        assert np.all(ref[k:] < 1e-10) and np.all(got[k:] < 1e-10)


@pytest.mark.parametrize("R,C,chi,steps,order", [(3, 3, 64, 4, 1), (4, 4, 256, 3, 1),
                                                  (3, 4, 64, 3, 2), (5, 2, 32, 4, 1)])
def test_t4_rotating_schedule_full_chi_is_exact(R, C, chi, steps, order):
    """The rotating-row schedule applies every coupling once per step: at full
    bond dimension it reproduces the exact Trotterised state."""
    g = Grid(R, C)
    m = mps.BlockMPS(g, chi, 0.6, J, H, DT, order, schedule=2)
    sv = statevector.StateVector(g, 0.6, J, H, DT, order)
    for _ in range(steps):
        m.step()
        sv.step()
        a, b = m.measure(), sv.measure()
        assert abs(a["z"] - b["z"]) < 1e-10 and abs(a["z2"] - b["z2"]) < 1e-10
    assert abs(abs(np.vdot(sv.psi, m.to_statevector())) ** 2 - 1) < 1e-10


@pytest.mark.parametrize("R,C", [(3, 3), (4, 4), (5, 6), (6, 8), (7, 8), (5, 5), (3, 2)])
def test_rotating_schedule_gates_each_pair_once(R, C):
    g = Grid(R, C)
    pos = g.snake()
    coupled = {frozenset((a, b)) for a in range(g.n_blocks)
               for b in range(a + 1, g.n_blocks) if pair_coupled(g, a, b)}
    for _ in range(2 * R):
        ops = step_ops(g, pos, 1, 2)
        gated = [frozenset((o[4], o[5])) for o in ops if o[0] == "U2" and o[3]]
        assert len(gated) == len(set(gated)) and set(gated) == coupled
    nu2 = sum(1 for o in ops if o[0] == "U2")
    assert nu2 == (7 * R - 8 if R % 2 == 0 else 7 * R - 7)


def test_t4_translation_invariance_full_chi():
    g = Grid(3, 4)
    m = mps.BlockMPS(g, 64, 0.5, J, H, DT)
    for _ in range(3):
        m.step()
    psi = m.to_statevector()
    p = np.abs(psi) ** 2
    z = statevector.z_table(g.n).astype(np.float64) @ p
    assert np.max(z) - np.min(z) < 1e-10


def test_t5_truncation_fidelity_is_overlap():
    """A truncation splits the state into kept and discarded orthogonal parts
    with weights f and 1-f: |<exact|truncated>|^2 = f."""
    g = Grid(4, 4)
    m = mps.BlockMPS(g, 6, 0.5, J, H, DT)
    ops = step_ops(g, list(m.pos))
    found = False
    for op in ops:
        if op[0] != "U2":
            m.apply_u1(op[1], m._single_site_gate(op[3], op[2]))
            continue
        exact = copy.deepcopy(m)
        exact.chi = 10 ** 6
        exact.apply_u2(op[1], bool(op[2]), bool(op[3]))
        f = m.apply_u2(op[1], bool(op[2]), bool(op[3]))
        if f < 1 - 1e-9:
            pe, pt = exact.to_statevector(), m.to_statevector()
            assert abs(np.vdot(pt, pt) - 1) < 1e-12
            assert abs(abs(np.vdot(pe, pt)) ** 2 - f) < 1e-12
            found = True
            break
    assert found


def test_t6_norm_and_monotone_fidelity():
    g = Grid(4, 4)
    m = mps.BlockMPS(g, 12, 0.5, J, H, DT)
    last = 0.0
    for _ in range(4):
        m.step()
        assert m.log_fidelity <= last + 1e-15
        last = m.log_fidelity
    assert all(abs(u["norm2"] - 1) < 1e-12 for u in m.update_log)
    assert 0 < math.exp(m.log_fidelity) <= 1


def test_t7_bounds_and_measure_matches_dense():
    g = Grid(4, 4)
    m = mps.BlockMPS(g, 8, 1.1, J, H, DT)
    zt = statevector.z_table(g.n).sum(axis=0).astype(np.float64)
    for _ in range(4):
        m.step()
        o = m.measure()
        assert abs(o["z"]) <= 1 and o["z"] ** 2 <= o["z2"] + 1e-15 and o["z2"] <= 1
        p = np.abs(m.to_statevector()) ** 2
        assert abs(o["z"] - p @ zt / (g.n * p.sum())) < 1e-12
        assert abs(o["z2"] - p @ (zt * zt) / (g.n ** 2 * p.sum())) < 1e-12


@pytest.mark.parametrize("R,C", [(4, 4), (4, 5), (5, 5), (5, 6), (6, 6), (6, 8), (7, 8),
                                 (3, 3), (2, 4), (1, 4), (3, 2)])
def test_schedule_gates_each_coupled_pair_once(R, C):
    g = Grid(R, C)
    pos = g.snake()
    for _ in range(2):
        ops = step_ops(g, pos)
        gated = [frozenset((o[4], o[5])) for o in ops if o[0] == "U2" and o[3]]
        coupled = {frozenset((a, b)) for a in range(g.n_blocks)
                   for b in range(a + 1, g.n_blocks) if pair_coupled(g, a, b)}
        assert len(gated) == len(set(gated))
        assert set(gated) == coupled
    nu2 = sum(1 for o in step_ops(g, g.snake()) if o[0] == "U2")
    if R >= 3:
        assert nu2 == 11 * R - 12


@pytest.mark.parametrize("line", [l for l in open(
    __file__.replace("test_oracle_pins.py", "golden/gamma_fit.txt")) if l.strip()
    and not l.startswith("#")])
def test_t9_gamma_fit_golden(line):
    label, dth, x, expected, tol = line.split()
    n = 16
    chi = 2 ** (float(x) * n)
    got = estimators.gamma_fit(float(dth), int(round(chi)), n)
    assert abs(got - float(expected)) <= float(tol)


# --------------------------------------------------------------------------
# planted mistakes: each must make at least one pin above fail
def _t4_error():
    g = Grid(3, 4)       # equal block widths: a missing transpose stays shape-valid
    m = mps.BlockMPS(g, 64, 0.6, J, H, DT)
    sv = statevector.StateVector(g, 0.6, J, H, DT)
    err = 0.0
    for _ in range(2):
        m.step()
        sv.step()
        a, b = m.measure(), sv.measure()
        err = max(err, abs(a["z"] - b["z"]), abs(a["z2"] - b["z2"]))
    return err


def test_planted_sign_error_is_caught(monkeypatch):
    from oracle import lattice
    orig = lattice.pair_phase
    monkeypatch.setattr(mps, "pair_phase",
                        lambda g, a, b, Jx, dt: orig(g, a, b, -Jx, dt))
    assert _t4_error() > 1e-6


def test_planted_missing_swap_is_caught(monkeypatch):
    orig = mps.BlockMPS.apply_u2

    def bad(self, i, swap, gate):
        f = orig(self, i, False, gate)
        if swap:
            self.pos[i], self.pos[i + 1] = self.pos[i + 1], self.pos[i]
        return f
    monkeypatch.setattr(mps.BlockMPS, "apply_u2", bad)
    assert _t4_error() > 1e-6


# --------------------------------------------------------------------------
# cubic lattice, one qubit per site (open boundaries), route-and-return schedule
def _dense_h_cube(lx, ly, lz):
    """Independent Kronecker construction on the cube: neighbours differ by
    one in exactly one coordinate (no wrap)."""
    n = lx * ly * lz
    I2 = np.eye(2)
    Zm = np.diag([1.0, -1.0])
    Xm = np.array([[0.0, 1.0], [1.0, 0.0]])

    def op(single, q):
        out = np.ones((1, 1))
        for k in range(n):
            out = np.kron(out, single if k == q else I2)
        return out

    coords = [(x, y, z) for x in range(lx) for y in range(ly) for z in range(lz)]
    idx = {c: (c[0] * ly + c[1]) * lz + c[2] for c in coords}
    pairs = set()
    for c1 in coords:
        for c2 in coords:
            if sum(abs(u - v) for u, v in zip(c1, c2)) == 1:
                a, b = idx[c1], idx[c2]
                pairs.add((min(a, b), max(a, b)))
    hzz = sum(op(Zm, a) @ op(Zm, b) for (a, b) in pairs)
    hx = sum(op(Xm, q) for q in range(n))
    return hzz, hx, len(pairs)


@pytest.mark.parametrize("shape", [(2, 2, 2), (2, 2, 3), (1, 3, 3)])
@pytest.mark.parametrize("order", [1, 2])
def test_cube_statevector_matches_dense_expm(shape, order):
    from oracle.lattice import Cube
    hzz, hx, npairs = _dense_h_cube(*shape)
    g = Cube(*shape)
    assert len(g.zz_bonds()) == npairs
    th = 0.41
    if order == 1:
        U = scipy.linalg.expm(-1j * DT * H * hx) @ scipy.linalg.expm(-1j * DT * J * hzz)
    else:
        half = scipy.linalg.expm(-0.5j * DT * H * hx)
        U = half @ scipy.linalg.expm(-1j * DT * J * hzz) @ half
    psi = np.ones(1)
    for _ in range(g.n):
        psi = np.kron(psi, [math.cos(th / 2), math.sin(th / 2)])
    sv = statevector.StateVector(g, th, J, H, DT, order)
    for _ in range(3):
        psi = U @ psi
        sv.step()
    assert np.max(np.abs(sv.psi - psi)) < 1e-12


@pytest.mark.parametrize("shape", [(2, 2, 2), (3, 3, 3), (2, 3, 4), (4, 4, 4), (1, 1, 5)])
def test_cube_bonds_and_snake(shape):
    from oracle.lattice import Cube
    lx, ly, lz = shape
    g = Cube(*shape)
    bonds = set(g.zz_bonds())
    assert len(bonds) == (lx - 1) * ly * lz + lx * (ly - 1) * lz + lx * ly * (lz - 1)
    sn = g.snake()
    assert sorted(sn) == list(range(g.n))
    # consecutive sites of the snake are nearest neighbours
    assert all((min(a, b), max(a, b)) in bonds for a, b in zip(sn, sn[1:]))


@pytest.mark.parametrize("lattice", ["cube223", "cube222", "grid44", "grid35"])
def test_route_return_schedule_gates_each_pair_once(lattice):
    from oracle.lattice import Cube
    from oracle.schedule import coupled_pairs
    g = {"cube223": Cube(2, 2, 3), "cube222": Cube(2, 2, 2), "grid44": Grid(4, 4),
         "grid35": Grid(3, 5)}[lattice]
    pos = g.snake()
    start = list(pos)
    for _ in range(2):
        ops = step_ops(g, pos, 1, 3)
        gated = [frozenset((o[4], o[5])) for o in ops if o[0] == "U2" and o[3]]
        assert len(gated) == len(set(gated))
        assert set(gated) == {frozenset(p) for p in coupled_pairs(g)}
        assert pos == start            # every routed block returns
        # a gated update always acts on the two blocks of a coupled pair
        assert all(frozenset((o[4], o[5])) in set(gated) for o in ops if o[0] == "U2" and o[3])


@pytest.mark.parametrize("lattice,chi,steps,order", [("cube223", 64, 3, 1), ("cube222", 16, 3, 2),
                                                     ("grid34", 64, 2, 1)])
def test_t4_route_return_full_chi_is_exact(lattice, chi, steps, order):
    """Route-and-return schedule at full bond dimension == exact state vector
    (cube: one qubit per site, open boundaries)."""
    from oracle.lattice import Cube
    g = {"cube223": Cube(2, 2, 3), "cube222": Cube(2, 2, 2), "grid34": Grid(3, 4)}[lattice]
    m = mps.BlockMPS(g, chi, 0.6, J, H, DT, order, schedule=3)
    sv = statevector.StateVector(g, 0.6, J, H, DT, order)
    for _ in range(steps):
        m.step()
        sv.step()
        a, b = m.measure(), sv.measure()
        assert abs(a["z"] - b["z"]) < 1e-10 and abs(a["z2"] - b["z2"]) < 1e-10
    assert abs(m.log_fidelity) < 1e-12
    assert abs(abs(np.vdot(sv.psi, m.to_statevector())) ** 2 - 1) < 1e-10


# ---- gate-by-gate path (schedule 4): each inter-block ZZ as a rank-2 MPO ----

@pytest.mark.parametrize("R,C,chi,steps,order", [(3, 3, 64, 3, 1), (2, 4, 16, 3, 1),
                                                  (3, 4, 64, 2, 2), (4, 2, 16, 3, 1)])
def test_gate_by_gate_full_chi_is_exact(R, C, chi, steps, order):
    """At full bond dimension the MPO route reproduces the exact Trotterised
    state: a wrong MPO weight, sign or bond ordering breaks the overlap."""
    g = Grid(R, C)
    m = mps.BlockMPS(g, chi, 0.6, J, H, DT, order, schedule=4)
    sv = statevector.StateVector(g, 0.6, J, H, DT, order)
    for _ in range(steps):
        m.step()
        sv.step()
        a, b = m.measure(), sv.measure()
        assert abs(a["z"] - b["z"]) < 1e-10 and abs(a["z2"] - b["z2"]) < 1e-10
        assert abs(a["log_fidelity"]) < 1e-11
    assert abs(abs(np.vdot(sv.psi, m.to_statevector())) ** 2 - 1) < 1e-10
    # every bond is back within its cap
    dims = [g.block_dim(b) for b in m.pos]
    for bond, b in enumerate(m.bond_dims()):
        assert b <= min(int(np.prod(dims[:bond])), int(np.prod(dims[bond:])))


@pytest.mark.parametrize("shape,order", [((2, 2, 2), 1), ((1, 3, 3), 2)])
def test_gate_by_gate_cube_full_chi_is_exact(shape, order):
    from oracle.lattice import Cube
    g = Cube(*shape)
    m = mps.BlockMPS(g, 64, 0.5, J, H, DT, order, schedule=4)
    sv = statevector.StateVector(g, 0.5, J, H, DT, order)
    for _ in range(2):
        m.step()
        sv.step()
    assert abs(abs(np.vdot(sv.psi, m.to_statevector())) ** 2 - 1) < 1e-10


@pytest.mark.parametrize("R,C,gates,truncations", [(4, 4, 24, 56), (5, 6, 40, 106),
                                                    (6, 8, 60, 172), (7, 8, 70, 206)])
def test_gate_by_gate_counts(R, C, gates, truncations):
    """One gate per ZZ bond between different blocks (2n bonds minus those
    inside a block); bond truncations per step = sum of chain distances."""
    g = Grid(R, C)
    blk = g.block_of_qubit()
    inter = sum(1 for (a, b) in g.zz_bonds() if blk[a] != blk[b])
    assert len(g.zz_bonds()) == 2 * g.n
    ops = step_ops(g, g.snake(), 1, 4)
    zz = [o for o in ops if o[0] == "ZZ"]
    assert len(zz) == inter == gates
    assert sum(o[2] - o[1] for o in zz) == truncations
    assert all(o[1] < o[2] for o in zz)


def test_gate_by_gate_single_truncation_is_orthogonal_projection():
    """T5 for the MPO route: from an exact MPS, one gate between neighbouring
    sites truncated to chi gives |<psi_exact|psi_MPS>|^2 = f, the kept weight."""
    g = Grid(3, 4)
    m = mps.BlockMPS(g, 64, 0.7, J, H, DT, 1, schedule=4)
    m.step()                                     # exact (full chi)
    psi0 = m.to_statevector()
    ops = [o for o in step_ops(g, list(m.pos), 1, 4) if o[0] == "ZZ" and o[2] == o[1] + 1]
    _, sa, sb, ja, jb = [o for o in ops if o[1] == 2][0]     # the middle bond (cap 64)
    qa = g.block_qubits(m.pos[sa])[ja]
    qb = g.block_qubits(m.pos[sb])[jb]
    n = g.n
    x = np.arange(2 ** n)
    za = 1 - 2 * ((x >> (n - 1 - qa)) & 1)
    zb = 1 - 2 * ((x >> (n - 1 - qb)) & 1)
    exact = np.exp(-1j * J * DT * za * zb) * psi0
    m.chi = 6
    fs = m.apply_zz_mpo(sa, sb, ja, jb)
    assert len(fs) == 1 and fs[0] < 1 - 1e-6
    psi = m.to_statevector()
    assert abs(np.linalg.norm(psi) - 1) < 1e-12
    assert abs(abs(np.vdot(exact, psi)) ** 2 - fs[0]) < 1e-12


def test_gate_by_gate_zero_coupling_closed_form():
    """J = 0: the MPO's second term vanishes; T2's closed form holds and F = 1."""
    g = Grid(3, 3)
    th = 0.45
    m = mps.BlockMPS(g, 4, th, 0.0, H, DT, 1, schedule=4)
    for s in range(1, 4):
        m.step()
        o = m.measure()
        c = math.cos(2 * H * DT * s)
        assert abs(o["z"] - math.cos(th) * c) < 1e-12
        assert abs(o["z2"] - (1 / g.n + (1 - 1 / g.n) * math.cos(th) ** 2 * c ** 2)) < 1e-12
        assert abs(o["fidelity"] - 1) < 1e-12


# --------------------------------------------------------------------------
# theta_min / theta_from_delta (model section) and the rescaled estimators
# (eqs. "Z_tot_via_F" and "z2_tot_rescaled")
def _product_vector(n, th):
    psi = np.ones(1)
    for _ in range(n):
        psi = np.kron(psi, [math.cos(th / 2), math.sin(th / 2)])
    return psi


@pytest.mark.parametrize("J_,h_", [(-1.0, 2.0), (-1.0, 1.0), (-2.0, -3.0), (-0.7, 0.4)])
def test_theta_min_minimises_product_state_energy(J_, h_):
    """theta_min is where the energy of the product state of eq.
    "initial_state" is lowest (the model section's mean-field minimum, four
    neighbours per qubit): minimise <Psi(theta)|H|Psi(theta)> with the dense
    Hamiltonian of the periodic 3x3 grid, where every qubit has 4 distinct
    neighbours, over theta in [-pi/2, pi/2] (ferromagnetic J < 0)."""
    import scipy.optimize
    from oracle.lattice import theta_min
    hzz, hx, _ = _dense_h(3, 3)
    Hd = J_ * hzz + h_ * hx

    def energy(th):
        psi = _product_vector(9, th)
        return float(psi @ Hd @ psi)
    res = scipy.optimize.minimize_scalar(energy, bounds=(-math.pi / 2, math.pi / 2),
                                         method="bounded", options={"xatol": 1e-11})
    assert abs(theta_min(J_, h_) - res.x) < 1e-6
    # and it is a minimum of the energy on the whole circle
    grid_th = np.linspace(-math.pi, math.pi, 721)
    assert energy(theta_min(J_, h_)) <= min(energy(t) for t in grid_th) + 1e-12


def test_theta_values_of_the_paper_temperatures():
    """J = -1, h = 2: theta_min = asin(2 / (4 * -1)) = -pi/6, and the paper's
    temperatures delta_theta = 0, 2pi/9, 3pi/9 give theta = -pi/6, pi/18,
    pi/6 (the mid temperature pi/18 is the start angle of the workloads)."""
    from oracle.lattice import theta_from_delta, theta_min
    assert abs(theta_min(-1.0, 2.0) + math.pi / 6) < 1e-15
    for dth, th in [(0.0, -math.pi / 6), (2 * math.pi / 9, math.pi / 18),
                    (3 * math.pi / 9, math.pi / 6)]:
        assert abs(theta_from_delta(dth, -1.0, 2.0) - th) < 1e-15


def _z_tot_diag(n):
    x = np.arange(2 ** n)
    return sum(1.0 - 2.0 * ((x >> (n - 1 - q)) & 1) for q in range(n))


@pytest.mark.parametrize("R,C,chi,site", [(3, 3, 6, 2), (2, 4, 3, 1), (3, 4, 5, 3)])
def test_z_rescaled_single_truncation_identity(R, C, chi, site):
    """One truncation of an exact state splits it as sqrt(f) psi_MPS +
    sqrt(1 - f) psi_perp with orthogonal parts (results section). Z_tot is a
    sum of one-qubit operators, each acting on one side of the cut, so the
    cross terms vanish and <Z>_exact = F <Z>_MPS + (1 - F) <Z>_perp exactly:
    the rescaled estimator of eq. "Z_tot_via_F" is the exact value less the
    discarded part's contribution. Every quantity but F <Z>_MPS comes from
    dense state vectors."""
    g = Grid(R, C)
    n = R * C
    m = mps.BlockMPS(g, 4 ** n, 0.9, J, H, DT)
    m.step()
    m.step()                                      # exact (full bond dimension)
    m.move_centre(site)
    exact = copy.deepcopy(m)
    exact.apply_u2(site, False, True)             # no truncation
    assert abs(exact.log_fidelity) < 1e-12
    m.chi = chi
    f = m.apply_u2(site, False, True)             # truncating the same update
    assert f < 1 - 1e-6
    psi_e = exact.to_statevector()
    psi_m = m.to_statevector()
    perp = (psi_e - math.sqrt(f) * psi_m) / math.sqrt(1 - f)
    assert abs(np.vdot(psi_m, perp)) < 1e-12 and abs(np.linalg.norm(perp) - 1) < 1e-10
    zd = _z_tot_diag(n)
    z_exact = float(np.real(np.vdot(psi_e, zd * psi_e))) / n
    z_perp = float(np.real(np.vdot(perp, zd * perp))) / n
    z_mps = m.measure()["z"]
    assert abs(estimators.z_rescaled(z_mps, f) + (1 - f) * z_perp - z_exact) < 1e-12


def test_rescaled_estimators_at_full_bond_dimension_are_exact():
    """Full bond dimension: F = 1, so both rescaled estimators equal the exact
    Trotterised values (state vector) for any gamma (the limit the results
    section states for chi -> infinity)."""
    g = Grid(3, 3)
    m = mps.BlockMPS(g, 4 ** 9, 0.7, J, H, DT)
    sv = statevector.StateVector(g, 0.7, J, H, DT, 1)
    for _ in range(3):
        m.step()
        sv.step()
    a, b = m.measure(), sv.measure()
    assert abs(a["fidelity"] - 1) < 1e-12
    assert abs(estimators.z_rescaled(a["z"], a["fidelity"]) - b["z"]) < 1e-10
    for gamma in (0.0, 0.2804, 0.4563, 0.647, 1.0, 2.5):
        assert abs(estimators.z2_rescaled(a["z2"], a["fidelity"], gamma) - b["z2"]) < 1e-10


@pytest.mark.parametrize("F1,F2", [(0.9, 0.5), (0.31, 0.999), (1e-3, 0.2)])
def test_z2_rescaled_no_exponent_and_step_products(F1, F2):
    """gamma = 0 leaves <Z^2>_MPS unchanged whatever F; and since F_MPS is a
    product of step fidelities (results section), rescaling by the factors
    of two stretches in turn equals rescaling by their product."""
    z2 = 0.37
    for F in (F1, F2, F1 * F2):
        assert estimators.z2_rescaled(z2, F, 0.0) == z2
    for gamma in (0.2804, 0.647, 1.7):
        once = estimators.z2_rescaled(z2, F1 * F2, gamma)
        twice = estimators.z2_rescaled(estimators.z2_rescaled(z2, F1, gamma), F2, gamma)
        assert abs(once - twice) < 1e-15 * max(1.0, abs(once))
        assert once < z2                       # F < 1, gamma > 0: a smaller estimate
