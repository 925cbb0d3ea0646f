"""Fidelity-rescaled estimators (results section).

  * magnetisation: <Z_tot> ~= F_MPS * <Z_tot>_MPS          (eq. "Z_tot_via_F")
  * order parameter: <Z_tot^2>_gamma = <Z_tot^2>_MPS * F_MPS^gamma
                                                         (eq. "z2_tot_rescaled")
  * gamma_fit = a * log2(chi) / n + b with (a, b) per initial temperature from
    the paper's table of gamma scaling ("tab:gamma_scaling").

Test infrastructure only (tests, the smoke check and the CPU baseline use
it). Pins: z_rescaled by the results section's single-truncation identity
<Z>_exact = F <Z>_MPS + (1 - F) <Z>_perp and by full bond dimension;
z2_rescaled by full bond dimension (F = 1), gamma = 0 and products of step
fidelities; gamma_fit by the printed values. The exponent of z2_rescaled at
F < 1 and gamma > 0 has no closed form to compare with: parity partially
unpinned there.
"""
from __future__ import annotations

import math

# (a, b) of gamma_fit = a*log2(chi)/n + b, keyed by delta_theta (table
# "Scaling of gamma_fit", 2D TFIM): low, mid and high temperature.
GAMMA_FIT_TABLE = {
    "low": (0.0, 2.588, 0.0),
    "mid": (2 * math.pi / 9, 1.8252, 0.0),
    "high": (3 * math.pi / 9, 1.641, -0.1298),
}


def gamma_fit(delta_theta: float, chi: int, n: int, tol: float = 1e-9) -> float:
    for (_, (dth, a, b)) in GAMMA_FIT_TABLE.items():
        if abs(delta_theta - dth) <= tol:
            return a * math.log2(chi) / n + b
    raise KeyError("no gamma_fit entry for delta_theta=%r" % delta_theta)


def z_rescaled(z_mps: float, fidelity: float) -> float:
    return fidelity * z_mps


def z2_rescaled(z2_mps: float, fidelity: float, gamma: float) -> float:
    return z2_mps * fidelity ** gamma
