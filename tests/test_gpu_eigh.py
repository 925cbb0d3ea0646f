"""The truncation eigensolver on chosen spectra (mps_eigh_top), both paths.

A Hermitian G = W diag(lam) W^H is planted with a seeded random unitary W
(or written out directly), and the solver's top-q eigenpairs are checked
against what the mathematics fixes, whatever the multiplicities:

* the eigenvalues equal numpy's (LAPACK) to 1e-12 ||G||;
* the vectors are orthonormal;
* they span an invariant subspace: ||G U - U (U^H G U)|| <= 1e-10 ||G||
  (when the cut splits a multiplet of equal eigenvalues the top-q subspace
  is not unique, but every valid choice is invariant);
* the kept weight trace(U^H G U) equals the sum of the q largest
  eigenvalues (the truncation's f relies on exactly this).

Spectra: distinct, a multiplet inside the kept set, a multiplet cut by the
truncation, exact rank deficiency with zeros kept, an exactly diagonal
matrix with zero rows, and matrices whose non-leading part is 1e-48 of
the leading one (residues of that size appear in the updates of a product
state) or 1e-170 (whose squares underflow: the reflectors must take such
columns as zero).
"""
import numpy as np
import pytest

from paper_2511_23438_amd import mpsim

pytestmark = pytest.mark.gpu


def _unitary(n, rng):
    z = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _planted(lam, seed):
    rng = np.random.default_rng(seed)
    W = _unitary(len(lam), rng)
    G = (W * np.asarray(lam, dtype=float)) @ W.conj().T
    return 0.5 * (G + G.conj().T)


def _tiny_tail(n, eps, seed):
    """e0 e0^H plus eps times a rank-3 PSD part on the first 7 coordinates;
    rows and columns 7.. are exactly zero."""
    rng = np.random.default_rng(seed)
    G = np.zeros((n, n), dtype=np.complex128)
    G[0, 0] = 1.0
    R = rng.normal(size=(7, 3)) + 1j * rng.normal(size=(7, 3))
    G[:7, :7] += eps * (R @ R.conj().T)
    return 0.5 * (G + G.conj().T)


def _cases():
    rng = np.random.default_rng(0)
    out = []
    out.append(("distinct", _planted(np.sort(rng.uniform(0, 1, 100))[::-1], 1), 30))
    lam = np.sort(rng.uniform(0, 1, 80))[::-1]
    lam[10:18] = 0.5                                   # multiplet inside the kept set
    out.append(("multiplet kept", _planted(lam, 2), 30))
    lam = np.sort(rng.uniform(0, 1, 80))[::-1]
    lam[26:34] = lam[26]                                # cut at 30 splits it
    out.append(("multiplet cut", _planted(lam, 3), 30))
    lam = np.zeros(64)
    lam[:10] = rng.uniform(0.1, 1, 10)
    out.append(("rank 10, 22 zeros kept", _planted(lam, 4), 32))
    d = np.zeros(16, dtype=np.complex128)
    d[0] = 1.0
    out.append(("diag(1, 0, ...) all kept", np.diag(d), 16))
    out.append(("diag(1, 0, ...) 4 kept", np.diag(d), 4))
    out.append(("tail 1e-48", _tiny_tail(16, 1e-48, 5), 16))
    out.append(("tail 1e-170", _tiny_tail(16, 1e-170, 6), 16))
    out.append(("tail 1e-48, 64 wide", _tiny_tail(64, 1e-48, 7), 40))
    out.append(("distinct 600", _planted(np.sort(rng.uniform(0, 1, 600))[::-1], 8), 100))
    return out


CASES = _cases()


@pytest.mark.parametrize("path", [1, 2])
@pytest.mark.parametrize("k", range(len(CASES)), ids=[c[0] for c in CASES])
def test_planted_spectrum(k, path):
    name, G, q = CASES[k]
    n = G.shape[0]
    print("case", name, "n", n, "q", q, "path", path, flush=True)
    lam, U = mpsim.eigh_top(G, q, eig_path=path, seed=11)
    ref = np.linalg.eigvalsh(G)[::-1][:q]
    gn = np.linalg.norm(G, 2)
    assert np.all(np.isfinite(lam)) and np.all(np.isfinite(U))
    assert np.max(np.abs(lam - ref)) <= 1e-12 * gn
    assert np.max(np.abs(U.conj().T @ U - np.eye(q))) < 1e-12
    GU = G @ U
    H = U.conj().T @ GU
    res = np.linalg.norm(GU - U @ H) / gn
    assert res <= 1e-10, res
    assert abs(np.trace(H).real - ref.sum()) <= 1e-12 * gn * max(1, q)
    print("  eig err %.1e residual %.1e" % (np.max(np.abs(lam - ref)) / gn, res), flush=True)

