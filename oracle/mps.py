"""Block MPS time evolution with two-site SVD truncation (the paper's TEBD,
results section) and transfer-matrix measurement of <Z_tot> and <Z_tot^2>
(eqs. "Z_tot" and "z2_tot").

Plain numpy complex128, written for readability, not speed:
  * the orthogonality centre is moved onto the two sites before every
    truncation by QR / LQ sweeps (the paper moves the centre to the bond
    before the decomposition);
  * theta = A_i A_{i+1} with the diagonal block-pair phase (and SWAP) applied,
    reshaped to (b_i d_i) x (d_{i+1} b_{i+2}) and decomposed by numpy's SVD;
  * exactly q = min(chi, rank bound) singular values are kept (zeros
    included); the truncation fidelity f = kept weight / total weight is
    multiplied into F_MPS (stored as log F) and the kept part is renormalised
    to unit norm (results section: normalise after each truncation, track the
    truncation fidelity separately; F_MPS(s) is the product of the
    truncation fidelities of every gate application);
  * observables are measured with full left environments after the whole
    step, independent of the canonical form.
"""
from __future__ import annotations

import math

import numpy as np

from .lattice import (Grid, block_x_layer, intra_phase, pair_phase,
                      product_site)
from .schedule import step_ops


class BlockMPS:
    def __init__(self, grid: Grid, chi: int, theta0: float, J: float,
                 h: float, dt: float, order: int = 1, schedule: int = 1):
        self.grid = grid
        self.chi = int(chi)
        self.J, self.h, self.dt = float(J), float(h), float(dt)
        self.order = int(order)
        self.schedule = int(schedule)
        self.pos = grid.snake()
        self.sites = []
        for b in self.pos:
            w = grid.block_width(b)
            self.sites.append(product_site(w, theta0).reshape(1, 2 ** w, 1))
        self.centre = 0
        self.log_fidelity = 0.0
        self.step_count = 0
        self.update_log: list[dict] = []     # per-U2 diagnostics
        self._pair_cache: dict = {}

    @classmethod
    def from_sites(cls, grid: Grid, chi: int, sites, centre: int, J: float, h: float,
                   dt: float, order: int = 1, schedule: int = 1) -> "BlockMPS":
        """Start from given sites (snake block order, mixed canonical form
        with the norm on site ``centre``)."""
        m = cls(grid, chi, 0.0, J, h, dt, order, schedule)
        m.sites = [np.array(a, dtype=np.complex128) for a in sites]
        m.centre = int(centre)
        return m

    # ---- gates ---------------------------------------------------------
    def _pair(self, a: int, b: int) -> np.ndarray:
        key = (a, b)
        if key not in self._pair_cache:
            self._pair_cache[key] = pair_phase(self.grid, a, b, self.J, self.dt)
        return self._pair_cache[key]

    def _gate_theta(self, theta: np.ndarray, i: int, gate: int) -> np.ndarray:
        """The block-pair ZZ phase D_ab[s_a, s_b] on theta[a, s_a, s_b, c]."""
        return theta * self._pair(self.pos[i], self.pos[i + 1])[None, :, :, None]

    def _single_site_gate(self, block: int, variant: int) -> np.ndarray:
        w = self.grid.block_width(block)
        dintra = np.diag(intra_phase(self.grid, block, self.J, self.dt))
        if variant == 0:
            return block_x_layer(w, self.h * self.dt) @ dintra
        if variant == 1:
            return dintra @ block_x_layer(w, self.h * self.dt / 2)
        return block_x_layer(w, self.h * self.dt / 2)

    # ---- canonical form --------------------------------------------------
    def move_centre(self, target: int) -> None:
        while self.centre < target:
            c = self.centre
            A = self.sites[c]
            b, d, k = A.shape
            Q, Rm = np.linalg.qr(A.reshape(b * d, k))
            self.sites[c] = Q.reshape(b, d, Q.shape[1])
            self.sites[c + 1] = np.einsum('ij,jsk->isk', Rm, self.sites[c + 1])
            self.centre += 1
        while self.centre > target:
            c = self.centre
            A = self.sites[c]
            k, d, b = A.shape
            Q, Rm = np.linalg.qr(A.reshape(k, d * b).conj().T)
            L = Rm.conj().T
            self.sites[c] = Q.conj().T.reshape(Q.shape[1], d, b)
            self.sites[c - 1] = np.einsum('isj,jk->isk', self.sites[c - 1], L)
            self.centre -= 1

    # ---- updates ---------------------------------------------------------
    def apply_u2(self, i: int, swap: bool, gate: bool) -> float:
        """Two-site update on sites (i, i+1); returns the truncation fidelity."""
        if self.centre < i:
            self.move_centre(i)
        elif self.centre > i + 1:
            self.move_centre(i + 1)
        A, B = self.sites[i], self.sites[i + 1]
        theta = np.einsum('asb,btc->astc', A, B)
        if gate:
            theta = self._gate_theta(theta, i, gate)
        if swap:
            theta = theta.transpose(0, 2, 1, 3)
        b, d1, d2, c = theta.shape
        M = theta.reshape(b * d1, d2 * c)
        U, S, Vh = np.linalg.svd(M, full_matrices=False)
        q = min(self.chi, len(S))
        total = float(np.sum(S ** 2))
        kept = float(np.sum(S[:q] ** 2))
        f = kept / total
        self.log_fidelity += math.log(f)
        Sk = S[:q] / math.sqrt(kept)
        self.sites[i] = U[:, :q].reshape(b, d1, q)
        self.sites[i + 1] = (Sk[:, None] * Vh[:q]).reshape(q, d2, c)
        self.centre = i + 1
        if swap:
            self.pos[i], self.pos[i + 1] = self.pos[i + 1], self.pos[i]
        gap = math.inf
        if q < len(S) and S[0] > 0:
            gap = float((S[q - 1] - S[q]) / S[0])
        self.update_log.append(dict(site=i, swap=swap, gate=gate, norm2=total,
                                    f=f, sv=S.copy(), q=q, gap=gap))
        return f

    def bond_cap(self, bond: int) -> int:
        """Largest rank bond ``bond`` (between sites bond-1 and bond) can
        carry: the smaller of the Hilbert-space dimensions on its two sides."""
        dims = [A.shape[1] for A in self.sites]
        left = math.prod(dims[:bond])
        right = math.prod(dims[bond:])
        return min(left, right)

    def apply_zz_mpo(self, sa: int, sb: int, ja: int, jb: int) -> list[float]:
        """One ZZ gate exp(-i J dt Z Z') between bit ja of the block at site
        sa and bit jb of the block at site sb > sa, as a rank-2 matrix product
        operator (results section): exp(-i phi Z Z') = cos(phi) I I
        - i sin(phi) Z Z', the operator index k in {0, 1} runs along the
        chain from sa to sb, so every bond between them doubles (new bond
        index = 2 * old + k). The MPS is then brought back to canonical form
        (centre on site sa, sites sa+1..sb right-orthonormal by LQ sweeps) and
        the doubled bonds are truncated one by one from left to right, each by
        the SVD of the centre site with the centre on that bond, keeping
        q = min(chi, rank bound) values. Returns the truncation fidelities."""
        phi = self.J * self.dt
        self.move_centre(sa)
        wa = int(round(math.log2(self.sites[sa].shape[1])))
        wb = int(round(math.log2(self.sites[sb].shape[1])))
        za = np.array([1 - 2 * ((s >> (wa - 1 - ja)) & 1) for s in range(2 ** wa)], dtype=float)
        zb = np.array([1 - 2 * ((s >> (wb - 1 - jb)) & 1) for s in range(2 ** wb)], dtype=float)
        # first site: right bond gains k with weights (cos phi, -i sin phi z)
        A = self.sites[sa]
        b0, d, b1 = A.shape
        X = np.empty((b0, d, b1, 2), dtype=np.complex128)
        X[..., 0] = math.cos(phi) * A
        X[..., 1] = -1j * math.sin(phi) * za[None, :, None] * A
        self.sites[sa] = X.reshape(b0, d, 2 * b1)
        # sites strictly between: k passes through unchanged
        for p in range(sa + 1, sb):
            A = self.sites[p]
            b0, d, b1 = A.shape
            X = np.zeros((b0, 2, d, b1, 2), dtype=np.complex128)
            X[:, 0, :, :, 0] = A
            X[:, 1, :, :, 1] = A
            self.sites[p] = X.reshape(2 * b0, d, 2 * b1)
        # last site: left bond gains k with weights (1, z')
        A = self.sites[sb]
        b0, d, b1 = A.shape
        X = np.empty((b0, 2, d, b1), dtype=np.complex128)
        X[:, 0] = A
        X[:, 1] = zb[None, :, None] * A
        self.sites[sb] = X.reshape(2 * b0, d, b1)
        # canonical form again: LQ sweeps from sb down to sa+1
        self.centre = sb
        self.move_centre(sa)
        out = []
        for p in range(sa, sb):
            out.append(self._truncate_bond(p))
        return out

    def _truncate_bond(self, p: int) -> float:
        """Truncate the bond between sites p and p+1 with the centre on site
        p: SVD of the site as a (b d) x b' matrix, keep the top q singular
        values, renormalise, and move the centre to p+1."""
        assert self.centre == p
        A = self.sites[p]
        b0, d, b1 = A.shape
        U, S, Vh = np.linalg.svd(A.reshape(b0 * d, b1), full_matrices=False)
        q = min(self.chi, self.bond_cap(p + 1), len(S))
        total = float(np.sum(S ** 2))
        kept = float(np.sum(S[:q] ** 2))
        f = kept / total
        self.log_fidelity += math.log(f)
        Sk = S[:q] / math.sqrt(kept)
        self.sites[p] = U[:, :q].reshape(b0, d, q)
        self.sites[p + 1] = np.einsum('ij,jsk->isk', Sk[:, None] * Vh[:q], self.sites[p + 1])
        self.centre = p + 1
        gap = math.inf
        if q < len(S) and S[0] > 0:
            gap = float((S[q - 1] - S[q]) / S[0])
        self.update_log.append(dict(site=p, swap=False, gate=True, norm2=total,
                                    f=f, sv=S.copy(), q=q, gap=gap))
        return f

    def apply_u1(self, p: int, U: np.ndarray) -> None:
        self.sites[p] = np.einsum('st,atb->asb', U, self.sites[p])

    def step(self) -> None:
        for op in step_ops(self.grid, list(self.pos), self.order, self.schedule):
            if op[0] == "U2":
                _, site, swap, gate, a, b = op
                assert (self.pos[site], self.pos[site + 1]) == (a, b)
                self.apply_u2(site, bool(swap), bool(gate))
            elif op[0] == "ZZ":
                _, sa, sb, ja, jb = op
                self.apply_zz_mpo(sa, sb, ja, jb)
            else:
                _, site, variant, block = op
                assert self.pos[site] == block
                self.apply_u1(site, self._single_site_gate(block, variant))
        self.step_count += 1

    # ---- measurement -------------------------------------------------------
    def block_zsum(self, block: int) -> np.ndarray:
        """z_p(s) = sum over the block's qubits of (1 - 2 bit)."""
        w = self.grid.block_width(block)
        s = np.arange(2 ** w)
        bits = np.array([(s >> (w - 1 - j)) & 1 for j in range(w)])
        return (1 - 2 * bits).sum(axis=0).astype(np.float64)

    def measure(self) -> dict:
        """Left sweep of three environments (bond-3 MPO for Z_tot, Z_tot^2)."""
        E0 = np.ones((1, 1), dtype=np.complex128)
        E1 = np.zeros((1, 1), dtype=np.complex128)
        E2 = np.zeros((1, 1), dtype=np.complex128)

        def T(E, A, w):
            # sum_s w_s A_s^H E A_s, as two contractions
            X = np.tensordot(E, A, axes=([1], [0]))            # (a, s, d)
            return np.tensordot(A.conj() * w[None, :, None], X,
                                axes=([0, 1], [0, 1]))          # (b, d)

        for p, A in enumerate(self.sites):
            z = self.block_zsum(self.pos[p])
            one = np.ones_like(z)
            n0 = T(E0, A, one)
            n1 = T(E1, A, one) + T(E0, A, z)
            n2 = T(E2, A, one) + 2 * T(E1, A, z) + T(E0, A, z * z)
            E0, E1, E2 = n0, n1, n2
        n = self.grid.n
        norm = E0[0, 0].real
        return dict(step=self.step_count, norm=norm,
                    z=E1[0, 0].real / (n * norm),
                    z2=E2[0, 0].real / (n * n * norm),
                    log_fidelity=self.log_fidelity,
                    fidelity=math.exp(self.log_fidelity))

    # ---- diagnostics ---------------------------------------------------------
    def bond_dims(self) -> list[int]:
        return [1] + [A.shape[2] for A in self.sites]

    def to_statevector(self) -> np.ndarray:
        """Dense state (n <= 20) with qubit q = r*C + c at bit n-1-q."""
        g = self.grid
        T = self.sites[0]
        for A in self.sites[1:]:
            T = np.tensordot(T, A, axes=([T.ndim - 1], [0]))
        T = T.reshape(T.shape[1:-1])
        n = g.n
        x = np.arange(2 ** n, dtype=np.int64)
        flat = np.zeros_like(x)
        stride = 1
        for p in reversed(range(len(self.pos))):
            qs = g.block_qubits(self.pos[p])
            w = len(qs)
            s = np.zeros_like(x)
            for j, q in enumerate(qs):
                s |= ((x >> (n - 1 - q)) & 1) << (w - 1 - j)
            flat += s * stride
            stride *= 2 ** w
        return T.reshape(-1)[flat]

    def bond_spectrum(self, bond: int) -> np.ndarray:
        """Singular values across bond ``bond`` (between sites bond-1, bond)."""
        self.move_centre(bond - 1)
        A = self.sites[bond - 1]
        b, d, k = A.shape
        return np.linalg.svd(A.reshape(b * d, k), compute_uv=False)


def run(grid: Grid, chi: int, theta0: float, J: float, h: float, dt: float,
        nsteps: int, order: int = 1, schedule: int = 1) -> list[dict]:
    """Measurements at s = 0..nsteps (step 0 before any gate)."""
    m = BlockMPS(grid, chi, theta0, J, h, dt, order, schedule)
    out = [m.measure()]
    for _ in range(nsteps):
        m.step()
        out.append(m.measure())
    return out
