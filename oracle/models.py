"""Operation-count, runtime and memory models of Sec. 3 (cost formulas, float64).

These are the paper's cost expressions written out; they feed tests only.
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


def prism_ops(n_z: int, N1: int, N2: int) -> int:
    """Multislice operations of the PRISM STEM-EELS algorithm n_z [N_1 + N_2 (n_z + 1)]."""
    return n_z * (N1 + N2 * (n_z + 1))


def nyquist_probe_step(alpha_rad: float, lam_A: float) -> float:
    """Probe step 1/(4 alpha) with alpha in inverse length (alpha_rad / lambda), so that
    a cell of side L needs (4 L alpha)^2 probes (Sec. 3, runtime model)."""
    return 1.0 / (4.0 * alpha_rad / lam_A)


def beam_count_estimate(alpha_rad: float, lam_A: float, L: float, f: int) -> float:
    """pi alpha^2 L^2 / f^2 with alpha in inverse length (Sec. 3)."""
    a = alpha_rad / lam_A
    return math.pi * a * a * L * L / (f * f)


def t_ms(A, B, N, L, alpha_inv, n_states, n_z):
    """Eq. TMS: 2 (4 L alpha)^2 (n_states n_z (n_z-1)/2 + n_z)(A N^2 log N + B N^2)."""
    return 2 * (4 * L * alpha_inv) ** 2 * ms_ops_printed(n_states, n_z) * (A * N * N * math.log(N) + B * N * N)


def t_prism_multislice(A, B, N, L, f, alpha_inv, beta_inv, n_z):
    """Eq. TPRISM1."""
    return (2 * (math.pi * alpha_inv ** 2 + 2 * (n_z - 1) * math.pi * beta_inv ** 2) * L * L / f ** 2
            * n_z * (A * N * N * math.log(N) + B * N * N))


def t_prism_products(B, C, N, L, f, alpha_inv, beta_inv):
    """Eq. TPRISM2: the three matrix-product terms."""
    return (B * (N / 2) ** 2 * math.pi * alpha_inv ** 2 * L ** 2 / f ** 2
            + C * (N / 2) ** 2 * math.pi ** 2 * alpha_inv ** 2 * beta_inv ** 2 * L ** 4 / f ** 6
            + 4 * C * math.pi ** 2 * alpha_inv ** 4 * beta_inv ** 2 * L ** 6 / f ** 6)


def memory_bytes(N: int, n_z: int, N1: int, N2: int, bytes_per_complex: int = 8):
    """Sec. 3 memory discussion: (multislice minimum of 4 N x N arrays, transmission stack
    of n_z arrays, both S-matrices of (N1 + N2) arrays of (N/2) x (N/2))."""
    ms_min = 4 * N * N * bytes_per_complex
    trans = n_z * N * N * bytes_per_complex
    smat = (N1 + N2) * (N // 2) ** 2 * bytes_per_complex
    return ms_min, trans, smat
