"""Seeded synthetic workloads (grid shapes, bond dimensions, couplings and
initial angles) for the TFIM block-MPS evolution.

This module only draws and names inputs; it holds none of the method's
arithmetic, so both the HIP path and the CPU reference can use it. Parameter
values follow the paper's model section (J = -1, h = 2, dt = 0.25, 20 steps,
product initial state of angle theta0).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

PAPER_J, PAPER_H, PAPER_DT, PAPER_STEPS = -1.0, 2.0, 0.25, 20


@dataclass
class Instance:
    rows: int
    cols: int
    chi: int
    J: float = PAPER_J
    h: float = PAPER_H
    dt: float = PAPER_DT
    theta0: float = math.pi / 18
    steps: int = PAPER_STEPS
    order: int = 1
    precision: str = "fp64"          # fp64 | c64 | bf16x3
    schedule: int = 1                # 1: routed wrap pairs, 2: rotating rows
    eig_batch: int = 0               # eigenvectors per band inverse-iteration launch (0: 1024)
    name: str = ""

    def as_dict(self):
        return asdict(self)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def small_4x4(seed: int = 0, chi: int = 16) -> Instance:
    """4x4 grid, blocks of 2 qubits (d = 4), chi = 16, theta0 ~ U(0, 2pi/9)."""
    th = float(rng(seed).uniform(0.0, 2 * math.pi / 9))
    return Instance(4, 4, chi, theta0=th, name="4x4_chi%d_seed%d" % (chi, seed))


def mid_5x6(chi: int = 64, precision: str = "c64") -> Instance:
    """5x6 grid, blocks of 3 qubits (d = 8), chi in {64, 128, 256, 512}."""
    return Instance(5, 6, chi, theta0=math.pi / 18, precision=precision,
                    name="5x6_chi%d" % chi)


def metric_6x8(chi: int = 1024, theta0: float = math.pi / 18,
               precision: str = "fp64") -> Instance:
    """6x8 grid, blocks of 4 qubits (d = 16), chi in {256, 512, 1024}."""
    return Instance(6, 8, chi, theta0=theta0, precision=precision,
                    name="6x8_chi%d" % chi)


def batched(count: int = 64, seed: int = 2511) -> list[Instance]:
    """Independent instances: grids {4x5, 5x5, 5x6, 6x6}, chi {32..256},
    J ~ U[-1.5, -0.5], h ~ U[0.5, 3], theta0 ~ U[0, pi/2]."""
    g = rng(seed)
    grids = [(4, 5), (5, 5), (5, 6), (6, 6)]
    chis = [32, 64, 128, 256]
    out = []
    for k in range(count):
        r, c = grids[int(g.integers(len(grids)))]
        out.append(Instance(r, c, chis[int(g.integers(len(chis)))],
                            J=float(g.uniform(-1.5, -0.5)),
                            h=float(g.uniform(0.5, 3.0)),
                            theta0=float(g.uniform(0.0, math.pi / 2)),
                            precision="c64", name="batch%d" % k))
    return out


@dataclass
class Request:
    arrival_s: float
    inst: Instance


def serving_trace(count: int = 200, rate: float = 50.0, seed: int = 2511,
                  chi_max: int = 1024) -> list[Request]:
    """Poisson arrivals; grids R ~ U{4..7}, C ~ U{4..8}; chi = 2^U(6, 10)
    rounded; J, h, theta0 as the batched set; 10..40 steps."""
    g = rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += float(g.exponential(1.0 / rate))
        r, c = int(g.integers(4, 8)), int(g.integers(4, 9))
        chi = min(chi_max, int(round(2 ** g.uniform(6, 10))))
        out.append(Request(t, Instance(
            r, c, chi, J=float(g.uniform(-1.5, -0.5)), h=float(g.uniform(0.5, 3.0)),
            theta0=float(g.uniform(0.0, math.pi / 2)),
            steps=int(g.integers(10, 41)), precision="c64", name="req%d" % k)))
    return out


def snake_dims(rows: int, cols: int) -> list[int]:
    """Local dimension of each site in the initial snake order (even rows
    left block first, odd rows right block first)."""
    dl, dr = 2 ** ((cols + 1) // 2), 2 ** (cols // 2)
    out = []
    for r in range(rows):
        out += [dl, dr] if r % 2 == 0 else [dr, dl]
    return out


def random_mps(rows: int, cols: int, chi: int, seed: int,
               centre: int | None = None, dims: list[int] | None = None
               ) -> tuple[list[np.ndarray], int]:
    """Seeded random normalised MPS in mixed canonical form: sites left of
    `centre` left-orthonormal, sites right of it right-orthonormal, the norm
    on site `centre` (default: the last site); bonds at min(chi, products of
    local dims). `dims` overrides the local dimensions of the grid's snake
    (e.g. [2] * n for a lattice with one qubit per site).

    A symmetry-free input state: the lattice symmetries of a uniform product
    state give exactly degenerate Schmidt values, which make truncations
    non-unique; a random state has none."""
    g = rng(seed)
    if dims is None:
        dims = snake_dims(rows, cols)
    N = len(dims)
    c = N - 1 if centre is None else int(centre)
    bonds = [1]
    for p in range(1, N):
        left = int(np.prod(dims[:p], dtype=np.float64)) if p < 40 else 10 ** 12
        right = int(np.prod(dims[p:], dtype=np.float64)) if N - p < 40 else 10 ** 12
        bonds.append(int(min(chi, left, right)))
    bonds.append(1)
    sites = []
    for p in range(N):
        b0, d, b1 = bonds[p], dims[p], bonds[p + 1]
        x = g.standard_normal((b0 * d, b1)) + 1j * g.standard_normal((b0 * d, b1))
        if p < c:
            q, _ = np.linalg.qr(x)
            sites.append(q[:, :b1].reshape(b0, d, b1))
        elif p > c:
            y = x.reshape(b0, d * b1)
            q, _ = np.linalg.qr(y.conj().T)
            sites.append(q[:, :b0].conj().T.reshape(b0, d, b1))
        else:
            sites.append((x / np.linalg.norm(x)).reshape(b0, d, b1))
    return sites, c
