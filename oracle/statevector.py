"""Exact Trotterised state-vector evolution for at most 20 qubits.

The Trotter step of the paper (eq. "trotter_step", second order) and the
first-order form exp(-i dt H_X) exp(-i dt H_ZZ) are applied gate layer by gate
layer to a dense vector: the ZZ layer is the diagonal phase
exp(-i J dt sum_bonds z_q z_q') and the transverse layer applies exp(-i phi X)
to each qubit. Qubit q = r*C + c is bit n-1-q of the basis index.
"""
from __future__ import annotations

import math

import numpy as np

from .lattice import Grid, rx_hamiltonian

MAX_QUBITS = 20


def z_table(n: int) -> np.ndarray:
    """z[q, x] = +1 if bit of qubit q in x is 0 else -1 (int8)."""
    x = np.arange(2 ** n, dtype=np.int64)
    return np.stack([(1 - 2 * ((x >> (n - 1 - q)) & 1)).astype(np.int8)
                     for q in range(n)])


class StateVector:
    def __init__(self, grid: Grid, theta0: float, J: float, h: float,
                 dt: float, order: int = 1):
        if grid.n > MAX_QUBITS:
            raise ValueError("state vector limited to %d qubits" % MAX_QUBITS)
        self.grid, self.J, self.h, self.dt, self.order = grid, J, h, dt, order
        n = grid.n
        c, s = math.cos(theta0 / 2), math.sin(theta0 / 2)
        psi = np.ones(1, dtype=np.complex128)
        for _ in range(n):
            psi = np.kron(psi, np.array([c, s], dtype=np.complex128))
        self.psi = psi
        self.z = z_table(n)
        energy = np.zeros(2 ** n, dtype=np.float64)
        for (a, b) in grid.zz_bonds():
            energy += self.z[a].astype(np.float64) * self.z[b]
        self.zz_phase = np.exp(-1j * J * dt * energy)
        self.step_count = 0

    def _x_layer(self, phi: float) -> None:
        n = self.grid.n
        g = rx_hamiltonian(phi)
        psi = self.psi
        for q in range(n):
            v = psi.reshape(2 ** q, 2, 2 ** (n - q - 1))
            psi = np.einsum('st,atb->asb', g, v).reshape(-1)
        self.psi = psi

    def step(self) -> None:
        if self.order == 1:
            self.psi = self.zz_phase * self.psi
            self._x_layer(self.h * self.dt)
        else:
            self._x_layer(self.h * self.dt / 2)
            self.psi = self.zz_phase * self.psi
            self._x_layer(self.h * self.dt / 2)
        self.step_count += 1

    def measure(self) -> dict:
        n = self.grid.n
        p = np.abs(self.psi) ** 2
        norm = float(p.sum())
        ztot = self.z.sum(axis=0).astype(np.float64)
        zj = (self.z.astype(np.float64) @ p) / norm
        return dict(step=self.step_count, norm=norm,
                    z=float(p @ ztot) / (n * norm),
                    z2=float(p @ (ztot * ztot)) / (n * n * norm),
                    z_sites=zj)


def run(grid: Grid, theta0: float, J: float, h: float, dt: float,
        nsteps: int, order: int = 1) -> list[dict]:
    sv = StateVector(grid, theta0, J, h, dt, order)
    out = [sv.measure()]
    for _ in range(nsteps):
        sv.step()
        out.append(sv.measure())
    return out
