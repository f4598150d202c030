"""Problem set-up shared by the two oracle algorithms (oracle-internal)."""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import physics as ph


@dataclasses.dataclass
class Setup:
    lam: float
    sigma: float
    T: np.ndarray            # complex128 [nz, ny, nx]
    P: np.ndarray            # complex128 [nz, ny, nx]
    ab1: np.ndarray          # aperture lattice coordinates [N1, 2]
    ix1: np.ndarray
    iy1: np.ndarray
    ab2: np.ndarray          # detector lattice coordinates [N2, 2]
    ix2: np.ndarray
    iy2: np.ndarray
    n1_fine: int             # aperture beam count at f = 1
    C: np.ndarray            # complex128 [N1, P] probe coefficients
    win: Optional[Tuple[int, int]]
    sites_by_slice: Dict[int, List[int]]


class BandLimitError(ValueError):
    pass


def make_setup(prob, lam: Optional[float] = None, sigma: Optional[float] = None) -> Setup:
    lam = ph.wavelength_A(prob.energy_eV) if lam is None else lam
    sigma = ph.sigma_per_VA(prob.energy_eV) if sigma is None else sigma
    nx, ny, lx, ly = prob.nx, prob.ny, prob.lx, prob.ly
    f = int(prob.interp_f)
    T = np.stack([ph.transmission(prob.V[j], sigma) for j in range(prob.n_slices)])
    P = np.stack([ph.propagator(nx, ny, lx, ly, lam, float(prob.dz[j]), prob.bandlimit)
                  for j in range(prob.n_slices)])
    alpha = prob.aperture_mrad * 1e-3
    ab1, ix1, iy1 = ph.lattice_beams(nx, ny, lx, ly, f, lam, 0.0, alpha)
    ab2, ix2, iy2 = ph.lattice_beams(nx, ny, lx, ly, f, lam, prob.det_inner_mrad * 1e-3,
                                     prob.det_outer_mrad * 1e-3)
    kmax = ph.band_radius(nx, ny, lx, ly, prob.bandlimit)
    for ab in (ab1, ab2):
        if ab.size:
            kk = np.sqrt((f * ab[:, 0] / lx) ** 2 + (f * ab[:, 1] / ly) ** 2)
            if np.any(kk > kmax):
                raise BandLimitError("beam outside the band limit")
    ab_f1, _, _ = ph.lattice_beams(nx, ny, lx, ly, 1, lam, 0.0, alpha)
    n1_fine = ab_f1.shape[0]
    C = ph.probe_coefficients(ab1, lx, ly, f, lam, prob.probes, n1_fine,
                              prob.defocus_A, prob.cs_A)
    win = ph.window_geometry(nx, ny, lx, ly, prob.window_A)
    if f > 1 and win is None:
        raise ValueError("interpolation factor > 1 needs a crop window")
    sbs: Dict[int, List[int]] = {}
    for s in range(prob.n_sites):
        sbs.setdefault(int(prob.site_slice[s]), []).append(s)
    return Setup(lam, sigma, T, P, ab1, ix1, iy1, ab2, ix2, iy2, n1_fine, C, win, sbs)


def site_window(prob, st: Setup, s: int):
    """(rows, cols) pixel indices of site s's contraction window (full cell if no crop)."""
    x, y = prob.site_xy[s]
    if st.win is None:
        return np.arange(prob.ny), np.arange(prob.nx)
    ix0, iy0 = ph.site_pixel(x, y, prob.nx, prob.ny, prob.lx, prob.ly)
    hx, hy = st.win
    return ph.window_indices(ix0, iy0, hx, hy, prob.nx, prob.ny)


def site_eligible(prob, st: Setup, s: int) -> np.ndarray:
    if int(prob.interp_f) == 1:
        return np.ones(prob.n_probes, dtype=bool)
    x, y = prob.site_xy[s]
    ix0, iy0 = ph.site_pixel(x, y, prob.nx, prob.ny, prob.lx, prob.ly)
    hx, hy = st.win
    return ph.eligible(ix0, iy0, hx, hy, prob.nx, prob.ny, prob.lx, prob.ly,
                       int(prob.interp_f), prob.probes)


def site_H(prob, s: int, n: int) -> np.ndarray:
    """Transition potential n of site s on its window, float64 complex."""
    return np.asarray(prob.H[int(prob.site_hoff[s]) + n], dtype=np.complex128)
