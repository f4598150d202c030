"""Map comparison metric (Eq. nrmsse, Sec. 4.A).

The printed expression is garbled (a 1/100 where a percentage factor is meant,
and a misplaced sum).  Read as the normalised root-sum-square difference
    eps = sqrt(sum_R (I_a(R) - I_b(R))^2) / sqrt(sum_R I_b(R)^2),
times 100 for a percentage.
"""
from __future__ import annotations

import numpy as np


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    den = np.sqrt(np.sum(b * b))
    if den == 0.0:
        return float(np.sqrt(np.sum(a * a)))
    return float(np.sqrt(np.sum((a - b) ** 2)) / den)


def max_rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
