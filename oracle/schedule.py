"""Step schedule of block-pair updates (the reading adopted for the paper's
TEBD step on the snake-ordered block MPS).

The paper applies the gates of one Trotter step (eq. "trotter_step") to a
snake-ordered MPS of half-row blocks (results section; supplement section
"MPS Ordering"). Every ZZ coupling between two blocks is applied as one
diagonal d_a x d_b phase gate on the two sites, and blocks that are not
neighbours in the chain are brought together by SWAP updates. One step:

  A  vertical pairs between rows r and r+1 that face each other in the chain;
  B  the horizontal pair of every row, fused with a SWAP (each row reverses);
  C  the vertical pairs that face each other after B;
  W  (periodic, R >= 3) the wrap pairs between row R-1 and row 0: the row
     R-1 block is swapped leftwards until it neighbours its row-0 partner,
     the gate is applied, and it is swapped back;
  X  the single-site layer exp(-i h dt X) (times the intra-block ZZ phases).

Schedule 2 (rotating rows) replaces W: phases A and C skip the facing pair
between the last two chain rows; after B the last chain row moves to the
chain front by SWAP updates (its first block to site 0, then its second to
site 1), and the crossings with the blocks it is coupled to (same side in
chain rows R-2 and 0) carry the phase gate. For odd R one pure SWAP first
reverses the moving row so that chain rows keep facing same-side blocks.
The chain order of the rows rotates by one row per step.

Schedule 3 (route and return) works for any lattice, and is the schedule of
the cubic lattice with one qubit per site (supplement, three-dimensional
generalisation): the coupled block pairs are taken in the order of their
chain positions at the start of the step; for a pair at sites pa < pb the
block at pb is swapped leftwards to pa+1, the phase gate is applied on
(pa, pa+1), and the block is swapped back, so every pair starts from the same
chain order and the order is unchanged after the step.

Schedule 4 (gate by gate) is the paper's own path (results section): every
ZZ bond between two different blocks is its own gate, applied to the block
MPS as a rank-2 matrix product operator that doubles the virtual bonds
between the two blocks, each followed by truncation of those bonds; bonds
inside a block are applied locally with the single-site layer. Blocks never
move. The gates are taken in the order of (site of the first block, site of
the second block, bit of the first qubit, bit of the second qubit).

Ops are tuples:
  ("U2", site, swap, gate, block_at_site, block_at_site_plus_1)
  ("ZZ", site_a, site_b, bit_a, bit_b)  site_a < site_b; bit j of the fused
                                        index of the block (j = 0 the most
                                        significant)
  ("U1", site, variant, block)   variant 0: U_X(h dt) * D_intra   (order 1)
                                 variant 1: D_intra * U_X(h dt/2) (order 2, first)
                                 variant 2: U_X(h dt/2)           (order 2, last)
"""
from __future__ import annotations

from .lattice import Grid, pair_coupled


def coupled_pairs(grid) -> list[tuple[int, int]]:
    """Unordered block pairs joined by at least one ZZ bond."""
    blk = grid.block_of_qubit()
    out = set()
    for (q1, q2) in grid.zz_bonds():
        a, b = blk[q1], blk[q2]
        if a != b:
            out.add((min(a, b), max(a, b)))
    return sorted(out)


def route_return_ops(grid, pos: list[int], order: int) -> list[tuple]:
    ops: list[tuple] = []

    def u2(site: int, swap: bool, gate: bool):
        a, b = pos[site], pos[site + 1]
        ops.append(("U2", site, int(swap), int(gate), a, b))
        if swap:
            pos[site], pos[site + 1] = pos[site + 1], pos[site]

    if order == 2:
        for p in range(len(pos)):
            ops.append(("U1", p, 1, pos[p]))
    where = {b: i for i, b in enumerate(pos)}
    pairs = sorted(coupled_pairs(grid),
                   key=lambda ab: (min(where[ab[0]], where[ab[1]]), max(where[ab[0]], where[ab[1]])))
    for (a, b) in pairs:
        pa, pb = sorted((where[a], where[b]))
        for p in range(pb - 1, pa, -1):
            u2(p, True, False)
        u2(pa, False, True)
        for p in range(pa + 1, pb):
            u2(p, True, False)
    for p in range(len(pos)):
        ops.append(("U1", p, 0 if order == 1 else 2, pos[p]))
    return ops


def gate_by_gate_ops(grid, pos: list[int], order: int) -> list[tuple]:
    """Schedule 4: one op per ZZ bond joining two different blocks."""
    ops: list[tuple] = []
    if order == 2:
        for p in range(len(pos)):
            ops.append(("U1", p, 1, pos[p]))
    blk = grid.block_of_qubit()
    where = {b: i for i, b in enumerate(pos)}
    gates = []
    for (q1, q2) in grid.zz_bonds():
        b1, b2 = blk[q1], blk[q2]
        if b1 == b2:
            continue
        s1, s2 = where[b1], where[b2]
        if s1 > s2:
            q1, q2, b1, b2, s1, s2 = q2, q1, b2, b1, s2, s1
        j1 = grid.block_qubits(b1).index(q1)
        j2 = grid.block_qubits(b2).index(q2)
        gates.append((s1, s2, j1, j2))
    for (s1, s2, j1, j2) in sorted(gates):
        ops.append(("ZZ", s1, s2, j1, j2))
    for p in range(len(pos)):
        ops.append(("U1", p, 0 if order == 1 else 2, pos[p]))
    return ops


def step_ops(grid, pos: list[int], order: int = 1, schedule: int = 1) -> list[tuple]:
    """Ops of one Trotter step starting from chain order ``pos``; ``pos`` is
    updated in place to the order at the end of the step."""
    if schedule == 3:
        return route_return_ops(grid, pos, order)
    if schedule == 4:
        return gate_by_gate_ops(grid, pos, order)
    R = grid.rows
    rotating = schedule == 2 and grid.periodic and R >= 3
    ops: list[tuple] = []

    def u2(site: int, swap: bool, gate: bool):
        a, b = pos[site], pos[site + 1]
        if gate and not pair_coupled(grid, a, b):
            gate = False
        ops.append(("U2", site, int(swap), int(gate), a, b))
        if swap:
            pos[site], pos[site + 1] = pos[site + 1], pos[site]

    if order == 2:
        for p in range(len(pos)):
            ops.append(("U1", p, 1, pos[p]))
    nfacing = R - 2 if rotating else R - 1
    for r in range(nfacing):                    # A
        u2(2 * r + 1, False, True)
    for r in range(R):                          # B
        u2(2 * r, True, True)
    for r in range(nfacing):                    # C
        u2(2 * r + 1, False, True)
    if rotating:                                # last row to the front
        if R % 2 == 1:
            u2(2 * R - 2, True, False)
        for p in range(2 * R - 3, -1, -1):
            u2(p, True, True)
        for p in range(2 * R - 2, 0, -1):
            u2(p, True, True)
    elif grid.periodic and R >= 3:              # W
        for p0 in (1, 0):
            target = 2 * (R - 1) + (pos[p0] % 2)
            t = pos.index(target)
            for p in range(t - 1, p0, -1):
                u2(p, True, False)
            u2(p0, False, True)
            for p in range(p0 + 1, t):
                u2(p, True, False)
    for p in range(len(pos)):                   # X
        ops.append(("U1", p, 0 if order == 1 else 2, pos[p]))
    return ops


def schedule(grid, nsteps: int, order: int = 1, schedule_id: int = 1) -> list[tuple]:
    pos = grid.snake()
    out = []
    for _ in range(nsteps):
        out += step_ops(grid, pos, order, schedule_id)
    return out
