"""O2: PRISM STEM-EELS (Sec. 3, second algorithm; Eqs. Hn0op/SHn0, MSop, MSTop) in float64.

Scattering matrices (rows are plane waves, columns real-space pixels):

* S_1(j)[k] = F^-1 M_{j-1} ... M_0 e_k : the plane wave k of the aperture
  multisliced to the entrance of slice j (S_1(0) = plane waves);
* S_2(j)[q]: the real-space row that projects a wave phi present at the
  entrance of slice j onto detector beam q after multislicing to the exit,
      sum_r S_2(j)[q](r) phi(r) = [M_{n_z-1} ... M_j phi]_q .
  Since M_j = P_j F T_j F^-1 and the DFT matrices are symmetric, the exact
  transpose is M_j^T x = F^-1 T_j F P_j x, so with x_{n_z} = e_q and
  x_j = M_j^T x_{j+1}:  S_2(j)[q] = T_j * fft2(P_j * x_{j+1}).
  (Eq. MSTop prints the operator factors in another order; that form differs
  by a parity flip unless V is centrosymmetric.  The exact transpose is used
  because it is the one for which the contraction equals the conventional map.)

Contraction at slice j for site s, transition n (Eq. SHn0 with S_1 acting first):

    A_n(q, R) = sum_{r in window} S_2(j)[q](r) H_n(r) sum_k c_k(R) S_1(j)[k](r)
    I(R)     += f^2 sum_q |A_n(q, R)|^2      over probes R eligible for s.

The window is the full cell unless a crop is requested (Sec. 4.B).  With f = 1
every probe is eligible; with f > 1 (PRISM interpolation, Sec. 3 beam counts)
the probe sees a transition only when the crop box lies inside its L/f box.
The paper never states the f > 1 case for EELS; it is pinned by an identity: on a
specimen made of f x f copies of a small cell, the f > 1 map at a probe that sees a
copy equals the small cell's conventional multislice map times f^2 N_1 / N_1(f = 1).
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np

from .common import make_setup, site_H, site_window, site_eligible


def forward_s1_iter(prob, st, j_last: int):
    """Yield (j, S_1(j)) for j = 0 .. j_last (complex128 [N1, ny, nx]), one slice at a time:
    the aperture plane waves e_k multisliced, S_1(j) = ifft2(M_{j-1} ... M_0 e_k)."""
    N1 = st.ab1.shape[0]
    x = np.zeros((N1, prob.ny, prob.nx), dtype=np.complex128)
    x[np.arange(N1), st.iy1, st.ix1] = 1.0
    for j in range(j_last + 1):
        psi = np.fft.ifft2(x)
        yield j, psi
        if j < j_last:
            x = st.P[j] * np.fft.fft2(st.T[j] * psi)


def forward_s1(prob, st, slices) -> Dict[int, np.ndarray]:
    """S_1(j) for every j in ``slices`` (complex128 [N1, ny, nx])."""
    need = set(int(j) for j in slices)
    if not need:
        return {}
    return {j: psi for j, psi in forward_s1_iter(prob, st, max(need)) if j in need}


def inverse_s1(prob, st, slices) -> Dict[int, np.ndarray]:
    """S_1(j) the inverse-multislice way (Sec. 4.C, Eq. MSinvop): the aperture plane waves
    are multisliced through all slices to the exit, then retreated one slice at a time with
    the conjugated operators in reverse order,
        x_j = M_j^-1 x_{j+1} = fft2(conj(T_j) * ifft2(conj(P_j) * x_{j+1})),
    and S_1(j) = ifft2(x_j).  Exact where no intensity left the band limit (P_j unitary on
    what it meets); otherwise approximate."""
    need = set(int(j) for j in slices)
    out: Dict[int, np.ndarray] = {}
    if not need:
        return out
    N1 = st.ab1.shape[0]
    x = np.zeros((N1, prob.ny, prob.nx), dtype=np.complex128)
    x[np.arange(N1), st.iy1, st.ix1] = 1.0
    for j in range(prob.n_slices):
        x = st.P[j] * np.fft.fft2(st.T[j] * np.fft.ifft2(x))
    for j in range(prob.n_slices - 1, min(need) - 1, -1):
        x = np.fft.fft2(np.conj(st.T[j]) * np.fft.ifft2(np.conj(st.P[j]) * x))
        if j in need:
            out[j] = np.fft.ifft2(x)
    return out


def inverse_s2(prob, st, slices) -> Dict[int, np.ndarray]:
    """S_2(j) the way Sec. 4.C prints the inverse multislice: S_2 is first formed for the
    entrance (slice 0) by the exact transposed sweep from the exit, x_0 = M_0^T ... M_{n_z-1}^T e_q,
    then retreated one slice at a time towards the exit with the inverse of each transposed
    step, the transmission and propagator conjugated and their order reversed,
        x_{j+1} = (M_j^T)^-1 x_j = conj(P_j) * ifft2(conj(T_j) * fft2(x_j)),
    and S_2(j) = fft2(x_j) (the transposed sweep's S_2(j) = T_j * fft2(P_j * x_{j+1}) has
    ifft2(S_2(j)) = x_j).  Exact where nothing left the band limit; otherwise approximate."""
    need = set(int(j) for j in slices)
    out: Dict[int, np.ndarray] = {}
    if not need:
        return out
    N2 = st.ab2.shape[0]
    x = np.zeros((N2, prob.ny, prob.nx), dtype=np.complex128)
    x[np.arange(N2), st.iy2, st.ix2] = 1.0
    for j in range(prob.n_slices - 1, -1, -1):
        x = np.fft.ifft2(st.T[j] * np.fft.fft2(st.P[j] * x))
    for j in range(0, max(need) + 1):
        if j in need:
            out[j] = np.fft.fft2(x)
        x = np.conj(st.P[j]) * np.fft.ifft2(np.conj(st.T[j]) * np.fft.fft2(x))
    return out


def reverse_s2(prob, st, j_stop: int = 0):
    """Yield (j, S_2(j)) for j = n_z-1 down to j_stop (exact transposed multislice)."""
    N2 = st.ab2.shape[0]
    x = np.zeros((N2, prob.ny, prob.nx), dtype=np.complex128)
    x[np.arange(N2), st.iy2, st.ix2] = 1.0
    for j in range(prob.n_slices - 1, j_stop - 1, -1):
        S2 = st.T[j] * np.fft.fft2(st.P[j] * x)
        yield j, S2
        x = np.fft.ifft2(S2)


def contract_windows(S1w: np.ndarray, S2w: np.ndarray, C_el: np.ndarray, Hs, f2: float) -> np.ndarray:
    """One site's contribution to its eligible probes, f^2 sum_n sum_q |A_n(q, R)|^2, from
    its windows S1w [N1, K] and S2w [N2, K], the probe coefficients C_el [N1, Pe] and the
    transition potentials Hs (each [K]) on the window pixels."""
    Psi = S1w.T @ C_el                                       # [K, Pe]  probe waves on the window
    out = np.zeros(C_el.shape[1], dtype=np.float64)
    for h in Hs:
        A = S2w @ (h[:, None] * Psi)                         # [N2, Pe]
        out += f2 * (np.abs(A) ** 2).sum(axis=0)
    return out


def contract_site(prob, st, s: int, S1j: np.ndarray, S2j: np.ndarray, I: np.ndarray):
    """Add site s's transitions to the map I (in place)."""
    rows, cols = site_window(prob, st, s)
    N1, N2 = S1j.shape[0], S2j.shape[0]
    S1w = S1j[:, rows][:, :, cols].reshape(N1, -1)          # [N1, K]
    S2w = S2j[:, rows][:, :, cols].reshape(N2, -1)          # [N2, K]
    el = site_eligible(prob, st, s)
    if not np.any(el):
        return
    Hs = [site_H(prob, s, n).reshape(-1) for n in range(int(prob.site_ntrans[s]))]
    I[el] += contract_windows(S1w, S2w, st.C[:, el], Hs, float(int(prob.interp_f) ** 2))


def prism_map(prob, lam=None, sigma=None, st=None, s1_mode: str = "stored") -> np.ndarray:
    """The map; s1_mode "stored" uses the forward S_1 and the transposed S_2 sweep (exact),
    "inverse" the inverse-multislice S_1, "inverse_s2" the inverse-multislice S_2 (Sec. 4.C
    as printed: S_2 retreated towards the exit)."""
    st = make_setup(prob, lam, sigma) if st is None else st
    I = np.zeros(prob.n_probes, dtype=np.float64)
    ion = sorted(st.sites_by_slice.keys())
    if not ion:
        return I
    if s1_mode == "inverse_s2":
        S1 = forward_s1(prob, st, ion)
        S2 = inverse_s2(prob, st, ion)
        for j in reversed(ion):
            for s in st.sites_by_slice.get(j, []):
                contract_site(prob, st, s, S1[j], S2[j], I)
        return I
    S1 = forward_s1(prob, st, ion) if s1_mode == "stored" else inverse_s1(prob, st, ion)
    for j, S2 in reverse_s2(prob, st, j_stop=min(ion)):
        for s in st.sites_by_slice.get(j, []):
            contract_site(prob, st, s, S1[j], S2, I)
    return I


def frozen_phonon_map(configs) -> np.ndarray:
    """Average of the maps of the given thermal configurations (same probes)."""
    return np.mean([prism_map(c) for c in configs], axis=0)


def site_maps(prob, lam=None, sigma=None) -> np.ndarray:
    """Per-site contributions [S, P] (for additivity tests)."""
    st = make_setup(prob, lam, sigma)
    out = np.zeros((prob.n_sites, prob.n_probes))
    ion = sorted(st.sites_by_slice.keys())
    if not ion:
        return out
    S1 = forward_s1(prob, st, ion)
    for j, S2 in reverse_s2(prob, st, j_stop=min(ion)):
        for s in st.sites_by_slice.get(j, []):
            contract_site(prob, st, s, S1[j], S2, out[s])
    return out


# ---------------------------------------------------------------------------------------
# The same map with the two sweeps split over disjoint beam subsets.  Each beam is
# multisliced on its own, so the map of Eq. SHn0 regroups exactly:
#   Psi_s(r, R) = sum_k S_1(j)[k](r) c_k(R) is a sum over aperture beams, and
#   I(R) = f^2 sum_n sum_q |A_n(q, R)|^2 is a sum over detector beams.
# This bounds memory for large cells (a few beams at a time); prism_map is the reference.

def _beam_subset(st, which: int, beams):
    import dataclasses
    b = np.asarray(beams, dtype=np.int64)
    if which == 1:
        return dataclasses.replace(st, ab1=st.ab1[b], ix1=st.ix1[b], iy1=st.iy1[b], C=st.C[b])
    return dataclasses.replace(st, ab2=st.ab2[b], ix2=st.ix2[b], iy2=st.iy2[b])


def window_rows(Sj: np.ndarray, rows, cols) -> np.ndarray:
    """The rows of a scattering matrix restricted to a window: [n_beams, K] (K = rows x cols)."""
    return Sj[:, rows[:, None], cols[None, :]].reshape(Sj.shape[0], -1)


def probe_waves_partial(prob, beams, chunk: int = 16, st=None, sink=None) -> Dict[int, np.ndarray]:
    """For every site s: the part of Psi_s = S_1w^T c (window pixels x eligible probes) that
    comes from the aperture beams `beams`, processed `chunk` beams at a time.  With a `sink`,
    each ionised slice's parts are handed to sink(j, {s: part}) as the sweep passes the slice
    (nothing is kept); otherwise they are summed and returned."""
    st = make_setup(prob) if st is None else st
    ion = sorted(st.sites_by_slice.keys())
    out: Dict[int, np.ndarray] = {}
    if not ion:
        return out
    beams = np.asarray(beams, dtype=np.int64)
    for c0 in range(0, len(beams), chunk):
        sub = _beam_subset(st, 1, beams[c0:c0 + chunk])
        for j, S1j in forward_s1_iter(prob, sub, ion[-1]):
            parts = {}
            for s in st.sites_by_slice.get(j, []):
                el = site_eligible(prob, st, s)
                if not np.any(el):
                    continue
                rows, cols = site_window(prob, st, s)
                parts[s] = window_rows(S1j, rows, cols).T @ sub.C[:, el]
            if sink is not None:
                if parts:
                    sink(j, parts)
                continue
            for s, part in parts.items():
                out[s] = out[s] + part if s in out else part
    return out


def intensity_partial(prob, psi: Dict[int, np.ndarray], beams, chunk: int = 16, st=None) -> np.ndarray:
    """f^2 sum_n sum_{q in beams} |A_n(q, R)|^2 for every probe, with A_n = S_2w (H_n * Psi_s)
    and the complete Psi of every site; detector beams `beams`, `chunk` at a time."""
    st = make_setup(prob) if st is None else st
    I = np.zeros(prob.n_probes, dtype=np.float64)
    ion = sorted(st.sites_by_slice.keys())
    if not ion:
        return I
    f2 = float(int(prob.interp_f) ** 2)
    beams = np.asarray(beams, dtype=np.int64)
    for c0 in range(0, len(beams), chunk):
        sub = _beam_subset(st, 2, beams[c0:c0 + chunk])
        for j, S2 in reverse_s2(prob, sub, j_stop=min(ion)):
            for s in st.sites_by_slice.get(j, []):
                if s not in psi:
                    continue
                el = site_eligible(prob, st, s)
                rows, cols = site_window(prob, st, s)
                S2w = window_rows(S2, rows, cols)
                for n in range(int(prob.site_ntrans[s])):
                    h = site_H(prob, s, n).reshape(-1)
                    A = S2w @ (h[:, None] * psi[s])
                    I[el] += f2 * (np.abs(A) ** 2).sum(axis=0)
    return I


def _psi_job(args):
    prob, beams, chunk = args
    return probe_waves_partial(prob, beams, chunk)


def _int_job(args):
    prob, psi, beams, chunk = args
    return intensity_partial(prob, psi, beams, chunk)


def prism_map_by_beams(prob, n_parts: int = 1, chunk: int = 16, map_fn=map) -> np.ndarray:
    """prism_map regrouped by beams: the aperture beams in n_parts disjoint sets (their Psi
    parts summed), then the detector beams in n_parts sets (their intensities summed).
    map_fn runs the independent parts (the builtin map, or a process pool's map)."""
    st = make_setup(prob)
    n1, n2 = st.ab1.shape[0], st.ab2.shape[0]
    parts1 = [b for b in np.array_split(np.arange(n1), n_parts) if len(b)]
    psi: Dict[int, np.ndarray] = {}
    for part in map_fn(_psi_job, [(prob, b, chunk) for b in parts1]):
        for s, v in part.items():
            psi[s] = psi[s] + v if s in psi else v
    parts2 = [b for b in np.array_split(np.arange(n2), n_parts) if len(b)]
    I = np.zeros(prob.n_probes, dtype=np.float64)
    for part in map_fn(_int_job, [(prob, psi, b, chunk) for b in parts2]):
        I += part
    return I
