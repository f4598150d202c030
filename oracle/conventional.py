"""O1: conventional multislice STEM-EELS (Sec. 3, first algorithm) in float64.

This is the plain definition of the map:

    for every probe R:   psi_hat(g, 0) = c(R)                          (Eq. illum)
      for every slice j:  psi = F^-1 psi_hat        (wave at the slice entrance)
        for every transition n acting in slice j:
          phi = H_n psi                                                  (Eq. Hn0Psi)
          phi_hat = M_{n_z-1} ... M_{j+1} M_j phi    multislice to the exit (Eq. MSop)
          I(R) += sum_{g in detector} |phi_hat(g)|^2
        psi_hat = M_j psi_hat                       advance the elastic wave

with M_j(x) = P_j * fft2(T_j * x) applied to a real-space x.  The loop covers all
n_z slices (the printed loop bound n_z - 1 is read as a slip, see models.py).
Cropped transitions are the same transition potential set to zero outside its
window.  Only interpolation factor f = 1 is defined here.

Cost is quadratic in the number of slices; use on small cells only.
"""
from __future__ import annotations

import math

import numpy as np

from . import physics as ph
from .common import make_setup, site_H, site_window


def detector_mask(prob, lam) -> np.ndarray:
    """D(g) on the FFT grid: beta_in <= lambda |g| <= beta_out (inclusive)."""
    KX, KY = ph.kgrid(prob.nx, prob.ny, prob.lx, prob.ly)
    th = lam * np.sqrt(KX ** 2 + KY ** 2)
    return ((th >= prob.det_inner_mrad * 1e-3) & (th <= prob.det_outer_mrad * 1e-3)).astype(np.float64)


def conventional_map(prob, probe_chunk: int = 64, lam=None, sigma=None) -> np.ndarray:
    if int(prob.interp_f) != 1:
        raise ValueError("the conventional algorithm is defined for f = 1 only")
    st = make_setup(prob, lam, sigma)
    D = detector_mask(prob, st.lam)
    nz, ny, nx = prob.n_slices, prob.ny, prob.nx
    I = np.zeros(prob.n_probes, dtype=np.float64)
    # full-plane transition potentials (zero outside a crop window)
    Hfull = {}
    for s in range(prob.n_sites):
        rows, cols = site_window(prob, st, s)
        for n in range(int(prob.site_ntrans[s])):
            h = np.zeros((ny, nx), dtype=np.complex128)
            h[np.ix_(rows, cols)] = site_H(prob, s, n)
            Hfull[(s, n)] = h
    for p0 in range(0, prob.n_probes, probe_chunk):
        p1 = min(prob.n_probes, p0 + probe_chunk)
        psi_hat = np.zeros((p1 - p0, ny, nx), dtype=np.complex128)
        psi_hat[:, st.iy1, st.ix1] = st.C[:, p0:p1].T
        for j in range(nz):
            psi = np.fft.ifft2(psi_hat)
            for s in st.sites_by_slice.get(j, []):
                for n in range(int(prob.site_ntrans[s])):
                    phi_hat = st.P[j] * np.fft.fft2(st.T[j] * Hfull[(s, n)] * psi)
                    for jj in range(j + 1, nz):
                        phi_hat = st.P[jj] * np.fft.fft2(st.T[jj] * np.fft.ifft2(phi_hat))
                    I[p0:p1] += (np.abs(phi_hat) ** 2 * D).sum(axis=(-2, -1))
            psi_hat = st.P[j] * np.fft.fft2(st.T[j] * psi)
    return I


def elastic_exit(prob, probe_index: int, lam=None, sigma=None) -> np.ndarray:
    """Elastic exit wave psi_hat(g, n_z) of one probe (Eq. 4 applied n_z times)."""
    st = make_setup(prob, lam, sigma)
    psi_hat = np.zeros((prob.ny, prob.nx), dtype=np.complex128)
    psi_hat[st.iy1, st.ix1] = st.C[:, probe_index]
    for j in range(prob.n_slices):
        psi_hat = st.P[j] * np.fft.fft2(st.T[j] * np.fft.ifft2(psi_hat))
    return psi_hat
