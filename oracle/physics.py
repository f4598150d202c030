"""Physical constants, sampling grids and the diagonal operators of the multislice method.

Conventions (paper Sec. 2, footnote to Eq. 4): the forward transform carries
exp(-2 pi i r.g); numpy's unnormalised ``fft2`` is the forward transform and
``ifft2`` (scaled by 1/N^2) its inverse.  Arrays are indexed [y, x].
"""
from __future__ import annotations

import math

import numpy as np

# CODATA 2018 exact / recommended values (SI)
H_PLANCK = 6.62607015e-34
M_ELECTRON = 9.1093837015e-31
Q_ELECTRON = 1.602176634e-19
C_LIGHT = 299792458.0


def wavelength_A(energy_eV: float) -> float:
    """Relativistic electron wavelength (Sec. 2, text after Eq. Schro): lambda = h / p with
    p^2 = 2 m0 e E (1 + e E / (2 m0 c^2)); returned in Angstrom."""
    eE = Q_ELECTRON * energy_eV
    p = math.sqrt(2.0 * M_ELECTRON * eE * (1.0 + eE / (2.0 * M_ELECTRON * C_LIGHT ** 2)))
    return H_PLANCK / p * 1e10


def sigma_per_VA(energy_eV: float) -> float:
    """Interaction constant sigma = 2 pi m e lambda / h^2 with the relativistic mass
    m = gamma m0 (Sec. 2, text after Eq. Schro); returned in rad / (V * Angstrom)."""
    gamma = 1.0 + Q_ELECTRON * energy_eV / (M_ELECTRON * C_LIGHT ** 2)
    lam_m = wavelength_A(energy_eV) * 1e-10
    s = 2.0 * math.pi * gamma * M_ELECTRON * Q_ELECTRON * lam_m / H_PLANCK ** 2   # rad/(V m)
    return s * 1e-10


def kgrid(nx: int, ny: int, lx: float, ly: float):
    """Spatial frequencies (1/Angstrom) of the FFT grid, arrays [ny, nx] (kx, ky)."""
    kx = np.fft.fftfreq(nx, d=lx / nx)
    ky = np.fft.fftfreq(ny, d=ly / ny)
    KX, KY = np.meshgrid(kx, ky, indexing="xy")
    return KX, KY


def band_radius(nx, ny, lx, ly, bandlimit=2.0 / 3.0) -> float:
    """Anti-aliasing radius b * k_Nyquist (Sec. 3, runtime discussion: the multislice
    output is band-limited to 1/2 or 2/3 of the array; here a circle, inclusive)."""
    return bandlimit * min(nx / (2.0 * lx), ny / (2.0 * ly))


def band_mask(nx, ny, lx, ly, bandlimit=2.0 / 3.0) -> np.ndarray:
    KX, KY = kgrid(nx, ny, lx, ly)
    return (np.sqrt(KX ** 2 + KY ** 2) <= band_radius(nx, ny, lx, ly, bandlimit)).astype(np.float64)


def propagator(nx, ny, lx, ly, lam, dz, bandlimit=2.0 / 3.0) -> np.ndarray:
    """Fresnel free-space factor exp(-i pi lambda dz g^2) of Eq. MSop, times the band mask."""
    KX, KY = kgrid(nx, ny, lx, ly)
    k2 = KX ** 2 + KY ** 2
    return band_mask(nx, ny, lx, ly, bandlimit) * np.exp(-1j * math.pi * lam * dz * k2)


def transmission(V_slice: np.ndarray, sigma: float) -> np.ndarray:
    """Transmission function exp(i sigma V) of Eq. MSop, V the projected potential (V*A)."""
    return np.exp(1j * sigma * np.asarray(V_slice, dtype=np.float64))


def lattice_beams(nx, ny, lx, ly, f, lam, theta_min_rad, theta_max_rad):
    """Plane waves on the PRISM lattice k = (f a / lx, f b / ly) with
    theta_min <= lambda |k| <= theta_max (Sec. 3, beam counts N_1 and N_2).

    Returns (a, b) integer lattice coordinates ordered by (b, a), and the FFT
    pixel indices (f a mod nx, f b mod ny)."""
    amax = int(math.floor(theta_max_rad / lam * lx / f)) + 1
    bmax = int(math.floor(theta_max_rad / lam * ly / f)) + 1
    out = []
    for b in range(-bmax, bmax + 1):
        for a in range(-amax, amax + 1):
            kx, ky = f * a / lx, f * b / ly
            th = lam * math.sqrt(kx * kx + ky * ky)
            if theta_min_rad <= th <= theta_max_rad:
                out.append((a, b))
    ab = np.array(out, dtype=np.int64).reshape(-1, 2)
    ix = np.mod(f * ab[:, 0], nx)
    iy = np.mod(f * ab[:, 1], ny)
    return ab, ix, iy


def aberration_chi(k2: np.ndarray, lam: float, defocus_A: float = 0.0, cs_A: float = 0.0):
    """Aberration phase chi(k) = pi lambda k^2 (Cs lambda^2 k^2 / 2 - defocus) (Eq. illum)."""
    return math.pi * lam * k2 * (0.5 * cs_A * lam * lam * k2 - defocus_A)


def probe_coefficients(ab, lx, ly, f, lam, probes, n1_fine, defocus_A=0.0, cs_A=0.0):
    """Illumination coefficients c_k(R) = s A(k) exp(-i chi(k)) exp(-2 pi i k.R) (Eq. illum,
    scan phase of the conventional algorithm's initialisation), shape [N_1, P].

    s = f^2 / sqrt(N_1 at f = 1): for f = 1 the probe has unit norm in reciprocal
    space; for f > 1 the coarse-lattice probe equals the true probe periodised with
    period L/f."""
    kx = f * ab[:, 0] / lx
    ky = f * ab[:, 1] / ly
    k2 = kx ** 2 + ky ** 2
    chi = aberration_chi(k2, lam, defocus_A, cs_A)
    R = np.asarray(probes, dtype=np.float64).reshape(-1, 2)
    phase = kx[:, None] * R[None, :, 0] + ky[:, None] * R[None, :, 1]
    s = f * f / math.sqrt(n1_fine)
    return s * np.exp(-1j * chi)[:, None] * np.exp(-2j * math.pi * phase)


def window_geometry(nx, ny, lx, ly, window_A):
    """Crop window half-widths (hx, hy) = floor(W/(2 dx) + 1/2) (Sec. 4.B); None = full cell."""
    if window_A <= 0:
        return None
    hx = int(math.floor(window_A / (2.0 * lx / nx) + 0.5))
    hy = int(math.floor(window_A / (2.0 * ly / ny) + 0.5))
    if 2 * hx + 1 >= nx or 2 * hy + 1 >= ny:
        return None
    return hx, hy


def site_pixel(x, y, nx, ny, lx, ly):
    """Nearest pixel (ix, iy) of a position: floor(x/dx + 1/2) mod nx."""
    ix = int(math.floor(x / (lx / nx) + 0.5)) % nx
    iy = int(math.floor(y / (ly / ny) + 0.5)) % ny
    return ix, iy


def window_indices(ix0, iy0, hx, hy, nx, ny):
    """Row and column pixel indices of a (2hy+1) x (2hx+1) window centred on (ix0, iy0)."""
    cols = np.mod(ix0 - hx + np.arange(2 * hx + 1), nx)
    rows = np.mod(iy0 - hy + np.arange(2 * hy + 1), ny)
    return rows, cols


def eligible(ix0, iy0, hx, hy, nx, ny, lx, ly, f, probes):
    """PRISM interpolation (f > 1): a transition contributes to probe R iff its crop box
    lies inside R's (L/f) box, compared with minimum-image distances."""
    R = np.asarray(probes, dtype=np.float64).reshape(-1, 2)
    if f == 1:
        return np.ones(R.shape[0], dtype=bool)
    dx, dy = lx / nx, ly / ny
    ddx = ix0 * dx - R[:, 0]
    ddy = iy0 * dy - R[:, 1]
    ddx = ddx - lx * np.floor(ddx / lx + 0.5)
    ddy = ddy - ly * np.floor(ddy / ly + 0.5)
    return (np.abs(ddx) + hx * dx <= lx / (2.0 * f)) & (np.abs(ddy) + hy * dy <= ly / (2.0 * f))
