"""Quench of the two-dimensional XY model (supplement, section "XY Model").

  * H_XY = (g/2) sum over nearest-neighbour pairs of (X_i X_j + Y_i Y_j) on
    an Lx x Ly grid with open boundaries (eq. "XY_hamiltonian");
  * one qubit per MPS site (that section maps qubits one to one to sites),
    on a row snake: even rows left to right, odd rows right to left;
  * initial state exp(-i pi/8 H_Z) exp(-i tau H_XY) |Neel> with
    H_Z = sum_j (-1)^j Z_j (eq. "xy_init"): (-1)^j is the checkerboard sign
    (-1)^(r + c), |Neel> the ground state of H_Z (qubit j in |1> where the sign
    is +1, |0> where it is -1), and exp(-i tau H_XY) applied as Trotter steps
    of size dtau (the section quotes g dtau = 0.02 pi: 1, 3 or 5 steps);
  * Trotter step of depth 7, second order (eq. "xy_trotter_step"):
    A/2 B/2 C/2 D C/2 B/2 A/2 with A / B the horizontal bonds starting on an
    even / odd column and C / D the vertical bonds starting on an even / odd
    row; every bond of a sublayer gets exp(-i phi (XX + YY)) with
    phi = g dt / 4 (half) or g dt / 2 (full);
  * signal X2_tot = n^-2 sum_jk (-1)^(j-k) <X_j X_k> (eq. "xy_signal"), the
    second moment of the staggered magnetisation M = sum_j (-1)^j X_j; the
    conserved charge <Z_tot> is reported beside it. The rescaled signal is
    X2_tot * F_MPS^gamma.

Bonds of one sublayer act on disjoint qubits, so they commute; in the MPS each
is applied like the route-and-return schedule: the far qubit is swapped next
to its partner, the gate is applied, and it is swapped back.

Test infrastructure: see the package docstring.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .mps import BlockMPS


@dataclass(frozen=True)
class XYGrid:
    rows: int
    cols: int
    periodic: bool = False

    @property
    def n(self) -> int:
        return self.rows * self.cols

    @property
    def n_blocks(self) -> int:
        return self.n

    def qubit(self, r: int, c: int) -> int:
        return r * self.cols + c

    def coords(self, q: int) -> tuple[int, int]:
        return divmod(q, self.cols)

    def sign(self, q: int) -> int:
        r, c = self.coords(q)
        return 1 if (r + c) % 2 == 0 else -1

    def block_qubits(self, block: int) -> list[int]:
        return [block]

    def block_width(self, block: int) -> int:
        return 1

    def block_dim(self, block: int) -> int:
        return 2

    def block_of_qubit(self) -> dict[int, int]:
        return {q: q for q in range(self.n)}

    def snake(self) -> list[int]:
        out = []
        for r in range(self.rows):
            cs = range(self.cols) if r % 2 == 0 else range(self.cols - 1, -1, -1)
            out += [self.qubit(r, c) for c in cs]
        return out

    def sublayer(self, name: str) -> list[tuple[int, int]]:
        """Bonds of sublayer A, B (horizontal, first column even / odd) or
        C, D (vertical, first row even / odd), as (q, q') pairs."""
        out = []
        for r in range(self.rows):
            for c in range(self.cols):
                if name in "AB" and c + 1 < self.cols and c % 2 == "AB".index(name):
                    out.append((self.qubit(r, c), self.qubit(r, c + 1)))
                if name in "CD" and r + 1 < self.rows and r % 2 == "CD".index(name):
                    out.append((self.qubit(r, c), self.qubit(r + 1, c)))
        return out

    def bonds(self) -> list[tuple[int, int]]:
        return sorted(b for name in "ABCD" for b in self.sublayer(name))


# sublayer order of one step (eq. "xy_trotter_step"); gate variant 1 = half
# step, 2 = full step
STEP_LAYERS = (("A", 1), ("B", 1), ("C", 1), ("D", 2), ("C", 1), ("B", 1), ("A", 1))


def xy_gate(phi: float) -> np.ndarray:
    """exp(-i phi (XX + YY)) on two qubits, basis |q q'> with q the most
    significant bit: XX + YY = 2 (|01><10| + |10><01|), identity on |00>, |11>."""
    c, s = math.cos(2 * phi), math.sin(2 * phi)
    G = np.eye(4, dtype=np.complex128)
    G[1, 1] = G[2, 2] = c
    G[1, 2] = G[2, 1] = -1j * s
    return G


def xy_step_ops(grid: XYGrid, pos: list[int], prep: bool = False) -> list[tuple]:
    """Ops of one step: ("U2", site, swap, gate, a, b) with gate 0 for a pure
    SWAP, 1 / 2 for the half / full sublayer gate (3 / 4 in a preparation
    step, whose angles use dtau)."""
    ops: list[tuple] = []
    off = 2 if prep else 0

    def u2(site: int, swap: bool, gate: int):
        a, b = pos[site], pos[site + 1]
        ops.append(("U2", site, int(swap), int(gate), a, b))
        if swap:
            pos[site], pos[site + 1] = pos[site + 1], pos[site]

    for (name, variant) in STEP_LAYERS:
        where = {b: i for i, b in enumerate(pos)}
        pairs = sorted((min(where[a], where[b]), max(where[a], where[b]))
                       for (a, b) in grid.sublayer(name))
        for (pa, pb) in pairs:
            for p in range(pb - 1, pa, -1):
                u2(p, True, 0)
            u2(pa, False, variant + off)
            for p in range(pa + 1, pb):
                u2(p, True, 0)
    return ops


def prep_steps(g: float, tau: float, dtau_target: float = 0.02 * math.pi) -> tuple[int, float]:
    """Number of preparation steps and their size: g tau / (g dtau) rounded,
    at least one when tau > 0 (g dtau = 0.02 pi gives 1, 3, 5 steps for
    g tau = 0.02 pi, 0.06 pi, 0.10 pi)."""
    if tau == 0.0:
        return 0, 0.0
    k = max(1, int(round(abs(g * tau) / dtau_target)))
    return k, tau / k


class XYMPS(BlockMPS):
    """One qubit per site; steps of eq. "xy_trotter_step"."""

    def __init__(self, grid: XYGrid, chi: int, g: float, dt: float, tau: float = 0.0):
        super().__init__(grid, chi, 0.0, g, 0.0, dt, 2, schedule=3)
        self.g = float(g)
        self.tau = float(tau)
        self.sites = []
        for q in self.pos:
            v = np.zeros(2, dtype=np.complex128)
            v[1 if grid.sign(q) == 1 else 0] = 1.0
            self.sites.append(v.reshape(1, 2, 1))
        self.centre = 0
        self.nprep, self.dtau = prep_steps(self.g, self.tau)
        self._gates = {1: xy_gate(self.g * dt / 4), 2: xy_gate(self.g * dt / 2),
                       3: xy_gate(self.g * self.dtau / 4), 4: xy_gate(self.g * self.dtau / 2)}
        for _ in range(self.nprep):
            self._run(xy_step_ops(grid, list(self.pos), prep=True))
        # exp(-i pi/8 H_Z): phase exp(-i pi/8 sign z) on every qubit
        for p, q in enumerate(self.pos):
            ph = np.array([np.exp(-1j * math.pi / 8 * grid.sign(q)),
                           np.exp(1j * math.pi / 8 * grid.sign(q))])
            self.apply_u1(p, np.diag(ph))

    def _gate_theta(self, theta: np.ndarray, i: int, gate: int) -> np.ndarray:
        b, d1, d2, c = theta.shape
        G = self._gates[gate]
        t = np.einsum('uv,avc->auc', G, theta.reshape(b, d1 * d2, c))
        return t.reshape(b, d1, d2, c)

    def _run(self, ops) -> None:
        for op in ops:
            _, site, swap, gate, a, b = op
            assert (self.pos[site], self.pos[site + 1]) == (a, b)
            self.apply_u2(site, bool(swap), gate)

    def step(self) -> None:
        self._run(xy_step_ops(self.grid, list(self.pos)))
        self.step_count += 1

    def measure(self) -> dict:
        """<Z_tot>/n and X2_tot = <M^2>/n^2, M = sum_j (-1)^j X_j, by left
        sweeps of transfer matrices (full environments)."""
        X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
        Z = np.diag([1.0, -1.0]).astype(np.complex128)
        I2 = np.eye(2, dtype=np.complex128)

        def T(E, A, O):
            # sum_{s,t} O[s,t] A_s^H E A_t
            X_ = np.tensordot(E, A, axes=([1], [0]))            # (a', t, c')
            Y = np.einsum('st,atc->asc', O, X_)
            return np.tensordot(A.conj(), Y, axes=([0, 1], [0, 1]))

        E0 = np.ones((1, 1), dtype=np.complex128)
        E1 = np.zeros((1, 1), dtype=np.complex128)
        E2 = np.zeros((1, 1), dtype=np.complex128)
        Ez = np.zeros((1, 1), dtype=np.complex128)
        for p, A in enumerate(self.sites):
            O = self.grid.sign(self.pos[p]) * X
            n0 = T(E0, A, I2)
            n1 = T(E1, A, I2) + T(E0, A, O)
            n2 = T(E2, A, I2) + 2 * T(E1, A, O) + T(E0, A, O @ O)
            nz = T(Ez, A, I2) + T(E0, A, Z)
            E0, E1, E2, Ez = n0, n1, n2, nz
        n = self.grid.n
        norm = E0[0, 0].real
        return dict(step=self.step_count, norm=norm, z=Ez[0, 0].real / (n * norm),
                    x2=E2[0, 0].real / (n * n * norm), log_fidelity=self.log_fidelity,
                    fidelity=math.exp(self.log_fidelity))


class XYStateVector:
    """Exact Trotterised evolution of the same circuit (at most 20 qubits),
    qubit q at bit n-1-q of the basis index."""

    def __init__(self, grid: XYGrid, g: float, dt: float, tau: float = 0.0):
        n = grid.n
        if n > 20:
            raise ValueError("state vector limited to 20 qubits")
        self.grid, self.g, self.dt = grid, float(g), float(dt)
        idx = 0
        for q in range(n):
            if grid.sign(q) == 1:
                idx |= 1 << (n - 1 - q)
        self.psi = np.zeros(2 ** n, dtype=np.complex128)
        self.psi[idx] = 1.0
        nprep, dtau = prep_steps(self.g, float(tau))
        for _ in range(nprep):
            self._step(dtau)
        x = np.arange(2 ** n)
        hz = np.zeros(2 ** n)
        for q in range(n):
            hz += grid.sign(q) * (1 - 2 * ((x >> (n - 1 - q)) & 1))
        self.psi = np.exp(-1j * math.pi / 8 * hz) * self.psi
        self.step_count = 0

    def _bond(self, G: np.ndarray, q1: int, q2: int) -> None:
        n = self.grid.n
        t = self.psi.reshape([2] * n)
        t = np.moveaxis(t, (q1, q2), (0, 1))
        sh = t.shape
        t = (G @ t.reshape(4, -1)).reshape(sh)
        self.psi = np.moveaxis(t, (0, 1), (q1, q2)).reshape(-1)

    def _step(self, dt: float) -> None:
        for (name, variant) in STEP_LAYERS:
            G = xy_gate(self.g * dt / (4 if variant == 1 else 2))
            for (q1, q2) in self.grid.sublayer(name):
                self._bond(G, q1, q2)

    def step(self) -> None:
        self._step(self.dt)
        self.step_count += 1

    def measure(self) -> dict:
        n = self.grid.n
        x = np.arange(2 ** n)
        p = np.abs(self.psi) ** 2
        ztot = np.zeros(2 ** n)
        Mpsi = np.zeros_like(self.psi)
        for q in range(n):
            ztot += 1 - 2 * ((x >> (n - 1 - q)) & 1)
            Mpsi += self.grid.sign(q) * self.psi[x ^ (1 << (n - 1 - q))]
        norm = float(p.sum())
        return dict(step=self.step_count, norm=norm, z=float(p @ ztot) / (n * norm),
                    x2=float(np.vdot(Mpsi, Mpsi).real) / (n * n * norm))
