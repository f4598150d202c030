"""Elastic companion images of an EELS map, in float64 (test infrastructure).

The Results' nanoparticle discussion shows, beside the EELS map, an incoherent bright-field
(iBF) image recorded with a detector of the same angular extent as the EELS aperture, an
annular dark-field (ADF) image with a 60 mrad inner angle, and the EELS map divided by the
iBF image.  A detector image is the elastic exit intensity inside a ring of angles:

    I_D(R) = sum_{g : beta_in <= lambda |g| <= beta_out} |psi_hat(g, n_z; R)|^2

with psi_hat(., n_z; R) the elastic multislice exit wave of probe R (Eq. illum, Eq. MSop
applied n_z times; the same propagation as the conventional oracle).  With the probe
normalisation of Eq. illum (sum_k |c_k|^2 = 1) it is a fraction of the incident beam.
An outer angle of None (or <= 0) means the band limit.  Defined for f = 1.
"""
from __future__ import annotations

import numpy as np

from . import physics as ph
from .common import make_setup


def ring_mask(prob, lam, inner_mrad, outer_mrad=None) -> np.ndarray:
    """Indicator of beta_in <= lambda |g| <= beta_out on the FFT grid (inclusive)."""
    KX, KY = ph.kgrid(prob.nx, prob.ny, prob.lx, prob.ly)
    th = lam * np.sqrt(KX ** 2 + KY ** 2)
    m = th >= inner_mrad * 1e-3
    if outer_mrad is not None and outer_mrad > 0:
        m &= th <= outer_mrad * 1e-3
    return m.astype(np.float64)


def exit_waves(prob, probe_idx=None, lam=None, sigma=None) -> np.ndarray:
    """Elastic exit waves psi_hat[P][ny][nx] of the selected probes (f = 1)."""
    if int(prob.interp_f) != 1:
        raise ValueError("companion images are defined for f = 1 only")
    st = make_setup(prob, lam, sigma)
    idx = np.arange(prob.n_probes) if probe_idx is None else np.asarray(probe_idx)
    psi = np.zeros((len(idx), prob.ny, prob.nx), dtype=np.complex128)
    psi[:, st.iy1, st.ix1] = st.C[:, idx].T
    for j in range(prob.n_slices):
        psi = st.P[j] * np.fft.fft2(st.T[j] * np.fft.ifft2(psi, axes=(-2, -1)), axes=(-2, -1))
    return psi


def detector_images(prob, rings, probe_idx=None, lam=None, sigma=None) -> np.ndarray:
    """I_D(R) for each ring (inner_mrad, outer_mrad) -> float64 [len(rings)][P]."""
    lam = ph.wavelength_A(prob.energy_eV) if lam is None else lam
    psi = exit_waves(prob, probe_idx, lam, sigma)
    inten = np.abs(psi) ** 2
    out = []
    for (a, b) in rings:
        m = ring_mask(prob, lam, a, b)
        out.append(np.einsum("pyx,yx->p", inten, m))
    return np.array(out)


def bf_corrected(eels_map, ibf) -> np.ndarray:
    """The EELS map divided by the iBF image (same probe order)."""
    return np.asarray(eels_map, dtype=np.float64) / np.asarray(ibf, dtype=np.float64)
