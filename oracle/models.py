"""Operation-count and memory models of Sec. 3 (cost formulas, float64).

These are the paper's cost expressions written out; they feed tests only.  The runtime
estimators (Eqs. TMS, TPRISM1, TPRISM2) are not kept: the paper evaluates them with
primitive timings measured at each grid size, which it does not print, so no printed
estimate can pin them.
"""
from __future__ import annotations

import math


def ms_ops_sum(n_states: int, n_z: int) -> int:
    """Multislice operations per probe of the conventional algorithm, as the sum
    sum_{iz=0}^{n_z-1} n_states (n_z - iz) + n_z (Sec. 3, after the first algorithm)."""
    return sum(n_states * (n_z - iz) for iz in range(n_z)) + n_z


def ms_ops_printed(n_states: int, n_z: int) -> float:
    """The printed closed form n_states n_z (n_z - 1)/2 + n_z.  It does not equal the sum
    above (which is n_states n_z (n_z + 1)/2 + n_z); only cost models use it."""
    return n_states * n_z * (n_z - 1) / 2 + n_z


def nyquist_probe_step(alpha_rad: float, lam_A: float) -> float:
    """Probe step 1/(4 alpha) with alpha in inverse length (alpha_rad / lambda), so that
    a cell of side L needs (4 L alpha)^2 probes (Sec. 3, runtime model)."""
    return 1.0 / (4.0 * alpha_rad / lam_A)


def beam_count_estimate(alpha_rad: float, lam_A: float, L: float, f: int) -> float:
    """pi alpha^2 L^2 / f^2 with alpha in inverse length (Sec. 3)."""
    a = alpha_rad / lam_A
    return math.pi * a * a * L * L / (f * f)


def memory_bytes(N: int, n_z: int, N1: int, N2: int, bytes_per_complex: int = 8):
    """Sec. 3 memory discussion: (multislice minimum of 4 N x N arrays, transmission stack
    of n_z arrays, both S-matrices of (N1 + N2) arrays of (N/2) x (N/2))."""
    ms_min = 4 * N * N * bytes_per_complex
    trans = n_z * N * N * bytes_per_complex
    smat = (N1 + N2) * (N // 2) ** 2 * bytes_per_complex
    return ms_min, trans, smat
