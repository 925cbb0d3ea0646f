"""Grid geometry, half-row blocks, snake order and Trotter gate tables.

Follows the paper's model section (TFIM Hamiltonian with periodic boundary
conditions, eq. "hamiltonian"; product initial state, eq. "initial_state") and
its block grouping (results section and the figure showing a 7x8 grouping:
each grid row is split into two groups and the qubits of a group are fused
into one MPS site of local dimension 2^w).

Conventions (readings where the paper is silent):
  * grid R x C = rows x row length; qubit (r, c) has index q = r*C + c;
  * Z|0> = +|0>, so z = +1 for bit 0 and -1 for bit 1;
  * block L_r holds columns [0, ceil(C/2)), block R_r holds [ceil(C/2), C);
    block id = 2*r + side (side 0 = L, 1 = R);
  * fused index s of a block: its first column is the most significant bit;
  * snake: even rows are stored L then R, odd rows R then L;
  * ZZ bonds: every unordered nearest-neighbour pair with periodic wrap on
    both axes, each pair counted once (matters only when R or C equals 2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Grid:
    rows: int
    cols: int
    periodic: bool = True

    @property
    def n(self) -> int:
        return self.rows * self.cols

    @property
    def w_left(self) -> int:
        return (self.cols + 1) // 2

    @property
    def w_right(self) -> int:
        return self.cols // 2

    def qubit(self, r: int, c: int) -> int:
        return r * self.cols + c

    # ---- blocks -------------------------------------------------------
    def block_columns(self, block: int) -> list[int]:
        side = block % 2
        if side == 0:
            return list(range(0, self.w_left))
        return list(range(self.w_left, self.cols))

    def block_qubits(self, block: int) -> list[int]:
        r = block // 2
        return [self.qubit(r, c) for c in self.block_columns(block)]

    def block_dim(self, block: int) -> int:
        return 2 ** len(self.block_columns(block))

    def block_width(self, block: int) -> int:
        return len(self.block_columns(block))

    @property
    def n_blocks(self) -> int:
        return 2 * self.rows

    def snake(self) -> list[int]:
        """Block id held by each MPS site in the initial snake order."""
        pos = []
        for r in range(self.rows):
            if r % 2 == 0:
                pos += [2 * r, 2 * r + 1]
            else:
                pos += [2 * r + 1, 2 * r]
        return pos

    # ---- bonds --------------------------------------------------------
    def zz_bonds(self) -> list[tuple[int, int]]:
        """Unordered nearest-neighbour pairs of H_ZZ, each counted once."""
        seen = set()
        out = []
        R, C = self.rows, self.cols
        for r in range(R):
            for c in range(C):
                nbrs = []
                if c + 1 < C:
                    nbrs.append((r, c + 1))
                elif self.periodic and C > 1:
                    nbrs.append((r, 0))
                if r + 1 < R:
                    nbrs.append((r + 1, c))
                elif self.periodic and R > 1:
                    nbrs.append((0, c))
                for (r2, c2) in nbrs:
                    a, b = self.qubit(r, c), self.qubit(r2, c2)
                    if a == b:
                        continue
                    key = (min(a, b), max(a, b))
                    if key not in seen:
                        seen.add(key)
                        out.append(key)
        return out

    def block_of_qubit(self) -> dict[int, int]:
        m = {}
        for b in range(self.n_blocks):
            for q in self.block_qubits(b):
                m[q] = b
        return m


@dataclass(frozen=True)
class Cube:
    """Lx x Ly x Lz cubic lattice with one qubit per MPS site (local dimension
    2), the three-dimensional generalisation in the paper's supplement (open
    boundaries by default).

    Qubit (x, y, z) has index q = (x*Ly + y)*Lz + z and is its own block.
    Snake: x slowest; inside layer x the rows y run forward for even x and
    backward for odd x; inside the t-th row visited (counting over all
    layers) z runs forward for even t and backward for odd t. Consecutive
    qubits of the snake are nearest neighbours.
    """
    lx: int
    ly: int
    lz: int
    periodic: bool = False

    @property
    def n(self) -> int:
        return self.lx * self.ly * self.lz

    @property
    def rows(self) -> int:
        return self.lx

    @property
    def n_blocks(self) -> int:
        return self.n

    def qubit(self, x: int, y: int, z: int) -> int:
        return (x * self.ly + y) * self.lz + z

    def block_qubits(self, block: int) -> list[int]:
        return [block]

    def block_columns(self, block: int) -> list[int]:
        return [0]

    def block_width(self, block: int) -> int:
        return 1

    def block_dim(self, block: int) -> int:
        return 2

    def snake(self) -> list[int]:
        pos = []
        t = 0
        for x in range(self.lx):
            ys = range(self.ly) if x % 2 == 0 else range(self.ly - 1, -1, -1)
            for y in ys:
                zs = range(self.lz) if t % 2 == 0 else range(self.lz - 1, -1, -1)
                for z in zs:
                    pos.append(self.qubit(x, y, z))
                t += 1
        return pos

    def zz_bonds(self) -> list[tuple[int, int]]:
        seen = set()
        out = []
        dims = (self.lx, self.ly, self.lz)
        for x in range(self.lx):
            for y in range(self.ly):
                for z in range(self.lz):
                    c = (x, y, z)
                    for ax in range(3):
                        nb = list(c)
                        nb[ax] += 1
                        if nb[ax] >= dims[ax]:
                            if not self.periodic or dims[ax] < 2:
                                continue
                            nb[ax] = 0
                        a, b = self.qubit(*c), self.qubit(*nb)
                        if a == b:
                            continue
                        key = (min(a, b), max(a, b))
                        if key not in seen:
                            seen.add(key)
                            out.append(key)
        return out

    def block_of_qubit(self) -> dict[int, int]:
        return {q: q for q in range(self.n)}


def z_of(bits_index: int, w: int, j: int) -> int:
    """z eigenvalue (+1 for bit 0) of the j-th qubit of a w-qubit fused index,
    j = 0 being the most significant bit."""
    bit = (bits_index >> (w - 1 - j)) & 1
    return 1 - 2 * bit


def block_z_values(grid, block: int) -> np.ndarray:
    """z-array of shape (d, w): z of each qubit of the block for every s."""
    w = grid.block_width(block)
    d = 2 ** w
    out = np.empty((d, w), dtype=np.int64)
    for s in range(d):
        for j in range(w):
            out[s, j] = z_of(s, w, j)
    return out


def pair_phase(grid, a: int, b: int, J: float, dt: float) -> np.ndarray:
    """D_ab[s_a, s_b] = exp(-i J dt sum over bonds crossing blocks a, b of z z').

    The ZZ layer exp(-i dt H_ZZ) is diagonal; restricted to the bonds between
    two blocks it is this d_a x d_b phase table (eq. "hamiltonian" and the
    Trotter step, eq. "trotter_step")."""
    qa = grid.block_qubits(a)
    qb = grid.block_qubits(b)
    za = block_z_values(grid, a)
    zb = block_z_values(grid, b)
    ia = {q: j for j, q in enumerate(qa)}
    ib = {q: j for j, q in enumerate(qb)}
    energy = np.zeros((len(za), len(zb)), dtype=np.float64)
    for (q1, q2) in grid.zz_bonds():
        if q1 in ia and q2 in ib:
            energy += np.outer(za[:, ia[q1]], zb[:, ib[q2]])
        elif q2 in ia and q1 in ib:
            energy += np.outer(za[:, ia[q2]], zb[:, ib[q1]])
    return np.exp(-1j * J * dt * energy)


def pair_coupled(grid, a: int, b: int) -> bool:
    qa, qb = set(grid.block_qubits(a)), set(grid.block_qubits(b))
    for (q1, q2) in grid.zz_bonds():
        if (q1 in qa and q2 in qb) or (q1 in qb and q2 in qa):
            return True
    return False


def intra_phase(grid, a: int, J: float, dt: float) -> np.ndarray:
    """D_a[s] = exp(-i J dt sum over bonds inside block a of z z')."""
    qa = grid.block_qubits(a)
    za = block_z_values(grid, a)
    ia = {q: j for j, q in enumerate(qa)}
    energy = np.zeros(len(za), dtype=np.float64)
    for (q1, q2) in grid.zz_bonds():
        if q1 in ia and q2 in ia:
            energy += za[:, ia[q1]] * za[:, ia[q2]]
    return np.exp(-1j * J * dt * energy)


def rx_hamiltonian(phi: float) -> np.ndarray:
    """exp(-i phi X) for one qubit (the transverse-field factor of the
    Trotter step with phi = h*dt, or h*dt/2 for the half layers)."""
    c, s = math.cos(phi), math.sin(phi)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def block_x_layer(w: int, phi: float) -> np.ndarray:
    """Kronecker power of exp(-i phi X) over the w qubits of a block, with the
    first qubit as the most significant factor."""
    u = np.ones((1, 1), dtype=np.complex128)
    g = rx_hamiltonian(phi)
    for _ in range(w):
        u = np.kron(u, g)
    return u


def product_site(w: int, theta0: float) -> np.ndarray:
    """Amplitudes of the fused block state for eq. "initial_state":
    every qubit in cos(theta/2)|0> + sin(theta/2)|1>."""
    d = 2 ** w
    c, s = math.cos(theta0 / 2), math.sin(theta0 / 2)
    v = np.empty(d, dtype=np.complex128)
    for idx in range(d):
        amp = 1.0
        for j in range(w):
            amp *= c if ((idx >> (w - 1 - j)) & 1) == 0 else s
        v[idx] = amp
    return v


def theta_min(J: float, h: float, coordination: int = 4) -> float:
    """Mean-field minimum-energy angle theta_min = asin(h / (coordination*J))
    from the model section (coordination 4 on the square lattice)."""
    return math.asin(h / (coordination * J))


def theta_from_delta(delta: float, J: float, h: float) -> float:
    """Absolute initial angle theta = theta_min + delta_theta."""
    return theta_min(J, h) + delta
