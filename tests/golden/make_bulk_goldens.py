"""Oracle results of single bulk two-site updates of the 6x8 grid (d = 16)
at the bond dimensions of the metric workload: Gram sides 4096 (chi = 256),
8192 (chi = 512) and 16384 (chi = 1024), each with and without SWAP.

For each case: the seeded random MPS in mixed canonical form with the
centre on the update's site (workloads.random_mps), the update on (site,
site + 1) with the block-pair phase gate (and SWAP) applied by the oracle
(numpy SVD of theta, results section), and what a float64 implementation
must reproduce whatever its gauge: the truncation fidelity f, the kept
singular values of the new bond (normalised), and sampled entries of the new
two-site block A_site A_site+1 (the normalised kept part of theta, unique
when the cut is not degenerate). The relative gap at the cut is stored to
show that it is not.

Calls only oracle/ and the seeded input generator. Usage (from the
repository root, takes about an hour on 8 cores, ~30 GB of memory at the
largest case):

    python tests/golden/make_bulk_goldens.py [chi ...]
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mps as omps          # noqa: E402
from oracle.lattice import Grid         # noqa: E402
from paper_2511_23438_amd import workloads  # noqa: E402

J, H, DT = -1.0, 2.0, 0.25
ROWS, COLS, SITE = 6, 8, 5
NSAMPLES = 64
CASES = [  # (chi, swap, seed)
    (256, 0, 4101), (256, 1, 4102),
    (512, 1, 4103), (512, 0, 4104),
    (1024, 1, 4105), (1024, 0, 4106),
]


def golden_path(chi: int, swap: int) -> str:
    return os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "bulk_update_6x8_chi%d_%s.json" % (chi, "swap" if swap else "noswap"))


def make(chi: int, swap: int, seed: int) -> dict:
    t0 = time.perf_counter()
    sites, centre = workloads.random_mps(ROWS, COLS, chi, seed, centre=SITE)
    grid = Grid(ROWS, COLS)
    m = omps.BlockMPS.from_sites(grid, chi, sites, centre, J, H, DT)
    blocks = (m.pos[SITE], m.pos[SITE + 1])
    del sites
    f = m.apply_u2(SITE, bool(swap), True)
    rec = m.update_log[-1]
    S, q = rec["sv"], rec["q"]
    kept = float(np.sum(S[:q] ** 2))
    A, B = m.sites[SITE], m.sites[SITE + 1]
    rows_, cols_ = A.shape[0] * A.shape[1], B.shape[1] * B.shape[2]
    g = workloads.rng(seed + 7)
    r = g.integers(0, rows_, NSAMPLES)
    c = g.integers(0, cols_, NSAMPLES)
    Am = A.reshape(rows_, q)
    Bm = B.reshape(q, cols_)
    vals = np.einsum('kq,qk->k', Am[r], Bm[:, c])
    out = {
        "grid": [ROWS, COLS], "chi": chi, "seed": seed, "centre": SITE, "site": SITE,
        "swap": swap, "gate": 1, "J": J, "h": H, "dt": DT,
        "blocks": [int(blocks[0]), int(blocks[1])],
        "theta_shape": [int(rows_), int(cols_)],
        "gram_side": int(min(len(S), rows_, cols_)),
        "q": int(q), "f": float(f), "relative_gap": float(rec["gap"]),
        "sv_kept": [float(x) for x in S[:q] / math.sqrt(kept)],
        "first_discarded_over_largest": float(S[q] / S[0]) if q < len(S) else 0.0,
        "samples": [[int(a), int(b), float(v.real), float(v.imag)]
                    for a, b, v in zip(r, c, vals)],
        "oracle_seconds": time.perf_counter() - t0,
    }
    return out


def main() -> None:
    want = {int(a) for a in sys.argv[1:]}
    for chi, swap, seed in CASES:
        if want and chi not in want:
            continue
        path = golden_path(chi, swap)
        print("chi %d swap %d seed %d ..." % (chi, swap, seed), flush=True)
        out = make(chi, swap, seed)
        with open(path, "w") as fh:
            json.dump(out, fh, indent=0)
        print("  f = %.17g  q = %d  gap = %.3e  (%.0fs) -> %s" % (
            out["f"], out["q"], out["relative_gap"], out["oracle_seconds"],
            os.path.relpath(path, ROOT)), flush=True)


if __name__ == "__main__":
    main()
