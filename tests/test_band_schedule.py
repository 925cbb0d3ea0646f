"""Host-side checks of two properties the band-reduction kernels rely on.

1. Bulge chasing (band -> tridiagonal, half-width HB = 32): sweep j removes
   column j below the subdiagonal and chases the bulge down in steps of HB
   rows; step k of sweep j runs in time slot 3 j + k, all steps of one slot in
   one launch. That is a valid reordering of the sequential sweeps only if
   the element windows of one slot are disjoint and every pair of steps that
   touch a common element keeps its sequential order. The windows below are
   the index ranges the step kernel reads and writes (reflector column,
   block left of the diagonal block, diagonal block, block below it).
2. The wave sums exchange values between lanes i and i^1, i^2, i^7, i^15,
   i^16, i^32 (DPP quad permutations, half-row and row mirrors, row swaps):
   every lane must end with the sum over its group.
"""
import pytest

HB = 32


def _steps(n, j):
    return (n - 1 - j + HB - 1) // HB


def _window(n, j, k):
    r = j + 1 + k * HB
    c = j if k == 0 else r - HB
    L = min(HB, n - r)
    if L < 2:
        return None
    Lb = min(HB, n - r - L)
    nl = r - c - 1
    w = set()
    for i in range(L):
        w.add((r + i, c))
        for jj in range(nl):
            w.add((r + i, c + 1 + jj))
        for jj in range(i + 1):
            w.add((r + i, r + jj))
    for i in range(Lb):
        for jj in range(L):
            w.add((r + L + i, r + jj))
    return w


def _violations(n, lag):
    last = {}
    per_slot = {}
    bad = 0
    for j in range(n - 2):                       # sequential order: sweep by sweep
        for k in range(_steps(n, j)):
            w = _window(n, j, k)
            if w is None:
                continue
            slot = lag * j + k
            for e in w:
                if e in last and last[e] >= slot:
                    bad += 1                     # an earlier step would not run first
                last[e] = slot
            per_slot.setdefault(slot, []).append(w)
    for ws in per_slot.values():
        seen = set()
        for w in ws:
            bad += len(seen & w)                 # two steps of one launch share elements
            seen |= w
    return bad


@pytest.mark.parametrize("n", [3, 4, 33, 34, 65, 66, 97, 130, 200])
def test_bulge_chasing_slots_reorder_the_sequential_sweeps(n):
    assert _violations(n, 3) == 0


def test_two_step_lag_would_overlap():
    # the lower block of step k-2 of sweep j+1 shares its corner with the
    # bulge column of step k of sweep j
    assert _violations(97, 2) > 0


_PARTNER = {1: 1, 2: 2, 4: 7, 8: 15, 16: 16, 32: 32}


def _reduce(vals, bits):
    v = list(vals)
    for m in bits:
        v = [v[i] + v[i ^ _PARTNER[m]] for i in range(64)]
    return v


def test_wave_sum_exchange_pattern():
    vals = [(i * 7919) % 1009 for i in range(64)]
    assert _reduce(vals, [1, 2, 4, 8, 16, 32]) == [sum(vals)] * 64


def test_eight_lane_sum_exchange_pattern():
    vals = [(i * 104729) % 997 for i in range(64)]
    out = _reduce(vals, [1, 2, 4])
    assert out == [sum(vals[(i // 8) * 8:(i // 8) * 8 + 8]) for i in range(64)]
