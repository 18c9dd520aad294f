"""Error parameters from reported gate fidelities (App. B) -- TEST
INFRASTRUCTURE.  Only tests use this module.

* eq. (fidelities_relation): the average fidelity F of a d-dimensional map
  and its entanglement fidelity F_e satisfy F = (d F_e + 1) / (d + 1).
* eq. (fe1) and its two-qubit counterpart: depolarising p and dephasing q
  give F_e = 1 - p - q + c p q, c = 4/3 for one qubit, 16/15 for two.
* A reported F is split into depolarising x eps and dephasing (1 - x) eps
  (x = 1 all depolarising); eps solves F_e(x eps, (1 - x) eps) = F_e(F).
  Here eps is found by bisection on [0, 1], where F_e falls monotonically.
* Angle-scaled errors (App. C, general notes): eps |theta| / pi.
"""
from __future__ import annotations

import math


def ent_from_avg(F: float, nq: int) -> float:
    d = 2 ** nq
    return ((d + 1) * F - 1) / d


def ent_fidelity(p_depol: float, p_deph: float, nq: int) -> float:
    c = 4.0 / 3.0 if nq == 1 else 16.0 / 15.0
    return 1.0 - p_depol - p_deph + c * p_depol * p_deph


def severity(F: float, nq: int, x: float):
    """(depolarising, dephasing) parameters reproducing average fidelity F."""
    target = ent_from_avg(F, nq)

    def f(eps):
        return ent_fidelity(x * eps, (1 - x) * eps, nq)

    if not (f(1.0) <= target <= 1.0):
        raise ValueError("fidelity out of range")
    lo, hi = 0.0, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > target:
            lo = mid
        else:
            hi = mid
    eps = 0.5 * (lo + hi)
    return x * eps, (1 - x) * eps


def angle_scaled(eps: float, theta: float) -> float:
    return eps * abs(theta) / math.pi


def zz_strength(J: float, delta_ct: float, alpha_c: float, alpha_t: float) -> float:
    """Sec. 8: static ZZ coupling of two transmons, J^2 (1/(Delta_ct - alpha_t)
    - 1/(Delta_ct + alpha_c)), in the unit of its inputs."""
    return J * J * (1.0 / (delta_ct - alpha_t) - 1.0 / (delta_ct + alpha_c))
