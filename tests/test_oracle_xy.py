"""Pins of the XY-model oracle (supplement, section "XY Model") against
mathematics that does not run through it: dense matrix exponentials of the
sublayer Hamiltonians built from Pauli Kronecker products, a two-qubit closed
form, the conserved U(1) charge, the Neel value of the signal, bond coverage
of the four sublayers, exactness at full bond dimension and the projection
identity of a single truncation."""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle.xy import STEP_LAYERS, XYGrid, XYMPS, XYStateVector, prep_steps, xy_gate, xy_step_ops

G_, DT_ = 1.0, 0.05 * math.pi
PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.diag([1.0, -1.0]).astype(complex)


def _op(n, q, P):
    out = np.ones((1, 1), dtype=complex)
    for k in range(n):
        out = np.kron(out, P if k == q else np.eye(2))
    return out


def _dense_sublayer_h(grid, name):
    n = grid.n
    H = np.zeros((2 ** n, 2 ** n), dtype=complex)
    for (a, b) in grid.sublayer(name):
        H += 0.5 * G_ * (_op(n, a, PX) @ _op(n, b, PX) + _op(n, a, PY) @ _op(n, b, PY))
    return H


@pytest.mark.parametrize("shape", [(2, 3), (3, 3), (1, 4)])
def test_state_vector_matches_dense_trotter_product(shape):
    """eq. xy_trotter_step with H_XY of eq. XY_hamiltonian, from dense expm;
    initial state of eq. xy_init with tau = 0.06 pi / g."""
    g = XYGrid(*shape)
    n = g.n
    U = np.eye(2 ** n, dtype=complex)
    for (name, variant) in STEP_LAYERS:
        f = 0.5 if variant == 1 else 1.0
        U = scipy.linalg.expm(-1j * f * DT_ * _dense_sublayer_h(g, name)) @ U
    tau = 0.06 * math.pi
    k, dtau = prep_steps(G_, tau)
    assert k == 3
    Up = np.eye(2 ** n, dtype=complex)
    for (name, variant) in STEP_LAYERS:
        f = 0.5 if variant == 1 else 1.0
        Up = scipy.linalg.expm(-1j * f * dtau * _dense_sublayer_h(g, name)) @ Up
    HZ = sum(g.sign(q) * _op(n, q, PZ) for q in range(n))
    neel = np.zeros(2 ** n, dtype=complex)
    # ground state of H_Z
    neel[int(np.argmin(np.diag(HZ).real))] = 1.0
    psi = scipy.linalg.expm(-1j * math.pi / 8 * HZ) @ np.linalg.matrix_power(Up, k) @ neel
    sv = XYStateVector(g, G_, DT_, tau)
    assert np.max(np.abs(sv.psi - psi)) < 1e-12
    M = sum(g.sign(q) * _op(n, q, PX) for q in range(n))
    for _ in range(3):
        psi = U @ psi
        sv.step()
    assert np.max(np.abs(sv.psi - psi)) < 1e-12
    assert abs(sv.measure()["x2"] - np.vdot(M @ psi, M @ psi).real / n ** 2) < 1e-12


def test_two_qubit_closed_form():
    """1 x 2 grid: one bond (sublayer A, half angle twice per step), so the
    state stays in span{|10>, |01>} and rotates by g dt per step."""
    g = XYGrid(1, 2)
    tau = 0.1 * math.pi
    m = XYMPS(g, 2, G_, DT_, tau)
    for s in range(5):
        # the preparation rotates |10> by g tau inside span{|10>, |01>}, the
        # staggered phase multiplies |10> by e^{i pi/4} and |01> by e^{-i pi/4},
        # then s steps rotate by g dt s
        v = np.array([math.cos(G_ * tau), -1j * math.sin(G_ * tau)])   # (|10>, |01>)
        v = v * np.array([np.exp(1j * math.pi / 4), np.exp(-1j * math.pi / 4)])
        R = np.array([[math.cos(G_ * DT_ * s), -1j * math.sin(G_ * DT_ * s)],
                      [-1j * math.sin(G_ * DT_ * s), math.cos(G_ * DT_ * s)]])
        v = R @ v
        # M = X0 - X1: <M^2> = 2 - 2 <X0 X1> = 2 - 4 Re(conj(v0) v1)
        x2 = (2 - 4 * (np.conj(v[0]) * v[1]).real) / 4
        o = m.measure()
        assert abs(o["x2"] - x2) < 1e-12 and abs(o["z"]) < 1e-14
        m.step()


def test_neel_signal_and_charge():
    """tau = 0: the Neel state (with the staggered phase) has <X_j X_k> = 0
    for j != k, so X2_tot = 1/n, and <Z_tot> = (#(-1) sites - #(+1) sites)/n."""
    for shape in [(2, 3), (3, 3), (4, 4)]:
        g = XYGrid(*shape)
        o = XYMPS(g, 4, G_, DT_, 0.0).measure()
        n = g.n
        plus = sum(1 for q in range(n) if g.sign(q) == 1)
        assert abs(o["x2"] - 1 / n) < 1e-14
        assert abs(o["z"] - (n - 2 * plus) / n) < 1e-14


@pytest.mark.parametrize("shape", [(2, 3), (3, 4), (5, 5), (6, 6), (1, 7)])
def test_sublayers_cover_bonds_once(shape):
    g = XYGrid(*shape)
    R, C = shape
    allb = []
    for name in "ABCD":
        bs = g.sublayer(name)
        qs = [q for b in bs for q in b]
        assert len(qs) == len(set(qs))               # disjoint inside a sublayer
        allb += bs
    assert len(allb) == len(set(allb)) == R * (C - 1) + (R - 1) * C
    for (a, b) in allb:
        (ra, ca), (rb, cb) = g.coords(a), g.coords(b)
        assert abs(ra - rb) + abs(ca - cb) == 1


def test_gate_is_unitary_and_conserves_charge():
    G = xy_gate(0.37)
    assert np.max(np.abs(G.conj().T @ G - np.eye(4))) < 1e-15
    zz = np.diag([2.0, 0.0, 0.0, -2.0])               # Z x I + I x Z
    assert np.max(np.abs(G @ zz - zz @ G)) < 1e-15


@pytest.mark.parametrize("shape,chi,steps", [((2, 3), 8, 3), ((3, 3), 32, 2), ((2, 4), 16, 2)])
def test_full_chi_mps_is_exact_and_conserves_charge(shape, chi, steps):
    g = XYGrid(*shape)
    tau = 0.06 * math.pi
    m = XYMPS(g, chi, G_, DT_, tau)
    sv = XYStateVector(g, G_, DT_, tau)
    z0 = m.measure()["z"]
    for _ in range(steps):
        m.step()
        sv.step()
        a, b = m.measure(), sv.measure()
        assert abs(a["x2"] - b["x2"]) < 1e-10 and abs(a["z"] - z0) < 1e-12
        assert abs(a["log_fidelity"]) < 1e-11
    assert abs(abs(np.vdot(sv.psi, m.to_statevector())) ** 2 - 1) < 1e-10


def test_single_truncation_is_orthogonal_projection():
    g = XYGrid(3, 3)
    m = XYMPS(g, 64, G_, DT_, 0.1 * math.pi)
    m.step()
    psi0 = m.to_statevector()
    ops = xy_step_ops(g, list(m.pos))
    _, site, swap, gate, a, b = [o for o in ops if o[3] and o[1] == 4][0]
    assert not swap
    n = g.n
    t = psi0.reshape([2] * n)
    t = np.moveaxis(t, (a, b), (0, 1))
    sh = t.shape
    t = (xy_gate(G_ * DT_ / (4 if gate == 1 else 2)) @ t.reshape(4, -1)).reshape(sh)
    exact = np.moveaxis(t, (0, 1), (a, b)).reshape(-1)
    m.chi = 3
    f = m.apply_u2(site, False, gate)
    assert f < 1 - 1e-6
    psi = m.to_statevector()
    assert abs(np.linalg.norm(psi) - 1) < 1e-12
    assert abs(abs(np.vdot(exact, psi)) ** 2 - f) < 1e-12
