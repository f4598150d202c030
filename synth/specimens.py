"""Seeded synthetic specimens shaped like the paper's workloads.

The paper simulates a SrTiO3-type perovskite crystal (Sec. 4.A) and an FePt
nanoparticle reconstructed from tomography (Sec. 4.D).  Neither the atomic
potentials nor the coordinates nor the transition potentials used there are
available, so these generators emit stand-ins with the same structure:

* projected potentials: every atom is a sum of two isotropic Gaussians
  a1*exp(-d^2/(2 w1^2)) + a2*exp(-d^2/(2 w2^2))   [V*Angstrom],
  d the minimum-image in-plane distance (periodic cell), summed on a square
  pixel patch of half-width ceil(6*max(w)/dx) pixels (at most (n-1)//2);
* transition potentials: H(r) = exp(-|r-r0|^2/(2 w^2)) * exp(i m phi), phi the
  azimuth of the minimum-image displacement measured from +x, with
  atan2(0, 0) = 0 (the same form as Eq. Hn0Psi's H_n0 only in its localisation
  and angular-momentum phase; the radial parts of Eq. Hn0def are not modelled);
* probes: a regular raster of positions, row-major with x fastest.

A ``Problem`` bundles the geometry, optics, the sites and the device-ready
arrays (V float32, H complex64).  Both the oracle and the HIP path read it.

Rounding rule used for pixel positions and window sizes: floor(x + 0.5).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

ENERGY_300KEV = 300e3


def _rhalf(x):
    return np.floor(np.asarray(x, dtype=np.float64) + 0.5).astype(np.int64)


@dataclasses.dataclass
class Problem:
    """One STEM-EELS map request: geometry, optics, sites and input arrays."""

    name: str
    nx: int
    ny: int
    lx: float
    ly: float
    dz: np.ndarray                       # [n_slices] slice thicknesses (Angstrom)
    V: np.ndarray                        # float32 [n_slices, ny, nx] projected potential (V*A)
    H: np.ndarray                        # complex64 [n_trans, nwy, nwx] (window) or [n_trans, ny, nx]
    site_slice: np.ndarray               # int32 [S]
    site_xy: np.ndarray                  # float64 [S, 2]  (x, y) of the ionised atom (A)
    site_ntrans: np.ndarray              # int32 [S]
    site_hoff: np.ndarray                # int64 [S] first transition index of the site in H
    probes: np.ndarray                   # float64 [P, 2]  (x, y) probe positions (A)
    probe_shape: Tuple[int, int]         # (nsy, nsx) raster shape of ``probes``
    energy_eV: float = ENERGY_300KEV
    aperture_mrad: float = 20.0
    det_inner_mrad: float = 0.0
    det_outer_mrad: float = 40.0
    interp_f: int = 1
    bandlimit: float = 2.0 / 3.0
    window_A: float = 0.0                # 0 -> contraction over the full cell
    defocus_A: float = 0.0
    cs_A: float = 0.0

    @property
    def n_slices(self) -> int:
        return int(len(self.dz))

    @property
    def n_sites(self) -> int:
        return int(len(self.site_slice))

    @property
    def n_probes(self) -> int:
        return int(self.probes.shape[0])

    @property
    def n_trans(self) -> int:
        return int(self.H.shape[0])

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# ----------------------------------------------------------------------------
# window geometry (input-format convention shared by the producer of H)
# ----------------------------------------------------------------------------

def window_shape(nx: int, ny: int, lx: float, ly: float, window_A: float) -> Optional[Tuple[int, int]]:
    """(nwy, nwx) of the crop window, or None when the contraction covers the cell.

    Half-widths h = floor(W/(2 dx) + 1/2) pixels, side 2h+1; a window that would
    not be smaller than the cell in both axes means "full cell".
    """
    if window_A <= 0:
        return None
    hx = int(_rhalf(window_A / (2.0 * lx / nx)))
    hy = int(_rhalf(window_A / (2.0 * ly / ny)))
    if 2 * hx + 1 >= nx or 2 * hy + 1 >= ny:
        return None
    return (2 * hy + 1, 2 * hx + 1)


# ----------------------------------------------------------------------------
# potentials
# ----------------------------------------------------------------------------

def _min_image(d, L):
    return d - L * np.floor(d / L + 0.5)


def projected_potential(nx, ny, lx, ly, n_slices, atom_slice, atom_xy, atom_amp, atom_w,
                        batch=4096) -> np.ndarray:
    """Sum of per-atom Gaussian pairs, one plane per slice, float64 [nz, ny, nx]."""
    dx, dy = lx / nx, ly / ny
    V = np.zeros((n_slices, ny * nx), dtype=np.float64)
    atom_slice = np.asarray(atom_slice, dtype=np.int64)
    atom_xy = np.asarray(atom_xy, dtype=np.float64).reshape(-1, 2)
    atom_amp = np.asarray(atom_amp, dtype=np.float64).reshape(-1, 2)
    atom_w = np.asarray(atom_w, dtype=np.float64).reshape(-1, 2)
    if atom_slice.size == 0:
        return V.reshape(n_slices, ny, nx)
    wmax = float(atom_w.max())
    hwx = min(int(math.ceil(6.0 * wmax / dx)), (nx - 1) // 2)
    hwy = min(int(math.ceil(6.0 * wmax / dy)), (ny - 1) // 2)
    ox = np.arange(-hwx, hwx + 1)
    oy = np.arange(-hwy, hwy + 1)
    for j in range(n_slices):
        sel = np.nonzero(atom_slice == j)[0]
        for b0 in range(0, sel.size, batch):
            s = sel[b0:b0 + batch]
            x0, y0 = atom_xy[s, 0], atom_xy[s, 1]
            ix0, iy0 = _rhalf(x0 / dx), _rhalf(y0 / dy)
            px = ix0[:, None] + ox[None, :]               # [A, wx]
            py = iy0[:, None] + oy[None, :]               # [A, wy]
            ddx = _min_image(px * dx - x0[:, None], lx)
            ddy = _min_image(py * dy - y0[:, None], ly)
            d2 = ddy[:, :, None] ** 2 + ddx[:, None, :] ** 2  # [A, wy, wx]
            a, w = atom_amp[s], atom_w[s]
            val = (a[:, 0, None, None] * np.exp(-d2 / (2.0 * w[:, 0, None, None] ** 2))
                   + a[:, 1, None, None] * np.exp(-d2 / (2.0 * w[:, 1, None, None] ** 2)))
            idx = (np.mod(py, ny)[:, :, None] * nx + np.mod(px, nx)[:, None, :])
            V[j] += np.bincount(idx.ravel(), weights=val.ravel(), minlength=ny * nx)
    return V.reshape(n_slices, ny, nx)


def transitions_lm(lmax: int = 2, widths=(0.3, 0.4, 0.5)) -> List[Tuple[int, int, float]]:
    """(l', m', width) for every l' <= lmax and every m' (9 for lmax = 2)."""
    out = []
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            out.append((l, m, float(widths[l])))
    return out


def transition_potentials(nx, ny, lx, ly, window_A, site_xy, trans: Sequence[Tuple[int, int, float]],
                          batch=256, dtype=np.complex64) -> np.ndarray:
    """H for every (site, transition), [S*len(trans), nwy, nwx] or [.., ny, nx], evaluated in
    float64 and stored as ``dtype``."""
    dx, dy = lx / nx, ly / ny
    site_xy = np.asarray(site_xy, dtype=np.float64).reshape(-1, 2)
    S = site_xy.shape[0]
    shp = window_shape(nx, ny, lx, ly, window_A)
    if shp is None:
        nwy, nwx = ny, nx
    else:
        nwy, nwx = shp
    out = np.zeros((S * len(trans), nwy, nwx), dtype=dtype)
    for b0 in range(0, S, batch):
        xs = site_xy[b0:b0 + batch, 0]
        ys = site_xy[b0:b0 + batch, 1]
        if shp is None:
            px = np.broadcast_to(np.arange(nx)[None, :], (xs.size, nx))
            py = np.broadcast_to(np.arange(ny)[None, :], (ys.size, ny))
        else:
            hx, hy = (nwx - 1) // 2, (nwy - 1) // 2
            px = (np.mod(_rhalf(xs / dx), nx) - hx)[:, None] + np.arange(nwx)[None, :]
            py = (np.mod(_rhalf(ys / dy), ny) - hy)[:, None] + np.arange(nwy)[None, :]
        ddx = _min_image(px * dx - xs[:, None], lx)
        ddy = _min_image(py * dy - ys[:, None], ly)
        DX = np.broadcast_to(ddx[:, None, :], (xs.size, nwy, nwx))
        DY = np.broadcast_to(ddy[:, :, None], (xs.size, nwy, nwx))
        d2 = DX ** 2 + DY ** 2
        phi = np.arctan2(DY, DX)
        for t, (l, m, w) in enumerate(trans):
            val = np.exp(-d2 / (2.0 * w * w)) * np.exp(1j * m * phi)
            rows = (np.arange(b0, b0 + xs.size) * len(trans) + t)
            out[rows] = val
    return out


def probe_grid(nsx, nsy, step_x, step_y, x0=0.0, y0=0.0) -> np.ndarray:
    """Probe positions, row-major: p = iy*nsx + ix -> (x0 + ix*step_x, y0 + iy*step_y)."""
    ix = np.arange(nsx)
    iy = np.arange(nsy)
    X, Y = np.meshgrid(x0 + ix * step_x, y0 + iy * step_y, indexing="xy")
    return np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float64)


def thermal_displacement(atom_xy, lx, ly, u_rms_A: float, seed: int) -> np.ndarray:
    """Frozen-phonon configuration: every atom displaced in-plane by independent Gaussian
    offsets of rms u_rms_A per axis (seeded), wrapped into the periodic cell.  u = 0 returns
    the positions unchanged."""
    xy = np.asarray(atom_xy, dtype=np.float64)
    if not u_rms_A > 0:
        return xy
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.normal(0.0, u_rms_A, size=xy.shape)
    out = xy + d
    out[:, 0] %= lx
    out[:, 1] %= ly
    return out


def _finish(name, nx, ny, lx, ly, dz, atom_slice, atom_xy, atom_amp, atom_w,
            site_slice, site_xy, trans, probes, probe_shape, **optics) -> Problem:
    dz = np.asarray(dz, dtype=np.float64)
    V = projected_potential(nx, ny, lx, ly, len(dz), atom_slice, atom_xy, atom_amp, atom_w)
    site_xy = np.asarray(site_xy, dtype=np.float64).reshape(-1, 2)
    H = transition_potentials(nx, ny, lx, ly, optics.get("window_A", 0.0), site_xy, trans, dtype=np.complex64)
    S = site_xy.shape[0]
    nt = len(trans)
    return Problem(
        name=name, nx=nx, ny=ny, lx=float(lx), ly=float(ly), dz=dz,
        V=V.astype(np.float32), H=H,
        site_slice=np.asarray(site_slice, dtype=np.int32),
        site_xy=site_xy,
        site_ntrans=np.full(S, nt, dtype=np.int32),
        site_hoff=(np.arange(S, dtype=np.int64) * nt),
        probes=np.asarray(probes, dtype=np.float64), probe_shape=tuple(probe_shape),
        **optics)


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------

def config1(seed: int = 1) -> Problem:
    """64x64 px, 10x10 A cell, 4 slices of 2 A; 3x3 atoms per slice, jitter +-0.05 A;
    Gaussian pair (40, 10) V*A at widths (0.3, 0.8) A; 300 keV; 20 mrad aperture;
    detector 0-40 mrad; f = 1; one ionised atom (centre, slice index 1) with
    m in {-1, 0, 1}, w = 0.4 A; 4x4 probes at 2.5 A steps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L, nz = 10.0, 4
    a_slice, a_xy = [], []
    centre = None
    for j in range(nz):
        for iy in range(3):
            for ix in range(3):
                x = (ix + 0.5) * L / 3 + rng.uniform(-0.05, 0.05)
                y = (iy + 0.5) * L / 3 + rng.uniform(-0.05, 0.05)
                a_slice.append(j)
                a_xy.append((x, y))
                if j == 1 and ix == 1 and iy == 1:
                    centre = (x, y)
    n = len(a_slice)
    amp = np.tile([[40.0, 10.0]], (n, 1))
    wid = np.tile([[0.3, 0.8]], (n, 1))
    trans = [(1, m, 0.4) for m in (-1, 0, 1)]
    probes = probe_grid(4, 4, 2.5, 2.5)
    return _finish("config1", 64, 64, L, L, [2.0] * nz, a_slice, a_xy, amp, wid,
                   [1], [centre], trans, probes, (4, 4),
                   energy_eV=ENERGY_300KEV, aperture_mrad=20.0, det_inner_mrad=0.0,
                   det_outer_mrad=40.0, interp_f=1, window_A=0.0)


def perovskite_atoms(ncell=5, a=4.0, c=3.9, thickness=100.0, dzs=2.0):
    """ABO3-like lattice: A (0,0,0), B (1/2,1/2,1/2), O at the three face centres.

    Returns (slice, xy, amp, width, species) with species 0=A, 1=B, 2=O."""
    frac = [((0.0, 0.0, 0.0), 0), ((0.5, 0.5, 0.5), 1),
            ((0.5, 0.5, 0.0), 2), ((0.5, 0.0, 0.5), 2), ((0.0, 0.5, 0.5), 2)]
    pairs = {0: (60.0, 15.0), 1: (40.0, 10.0), 2: (15.0, 4.0)}
    sl, xy, amp, wid, sp = [], [], [], [], []
    nlay = int(math.ceil(thickness / c))
    for m in range(nlay):
        for iy in range(ncell):
            for ix in range(ncell):
                for (fx, fy, fz), s in frac:
                    z = (m + fz) * c
                    if z >= thickness:
                        continue
                    sl.append(int(math.floor(z / dzs)))
                    xy.append(((ix + fx) * a, (iy + fy) * a))
                    amp.append(pairs[s])
                    wid.append((0.3, 0.8))
                    sp.append(s)
    return (np.array(sl), np.array(xy), np.array(amp), np.array(wid), np.array(sp))


def config2(seed: int = 2, n_scan: int = 64, window_A: float = 0.0, displace_A: float = 0.0,
            displace_seed: int = 0) -> Problem:
    """256x256 px, 20x20 A cell (5x5 perovskite cells of 4.0 A, 3.9 A along z),
    50 slices of 2 A; 21 mrad aperture; detector 0-50 mrad; every B atom ionised
    with the 9 (l' <= 2, m') transitions; 64x64 probes at 0.3125 A steps.
    displace_A > 0: one frozen-phonon configuration (see thermal_displacement)."""
    del seed  # the crystal is deterministic (no jitter); kept for a uniform signature
    sl, xy, amp, wid, sp = perovskite_atoms()
    xy = thermal_displacement(xy, 20.0, 20.0, displace_A, displace_seed)
    b = np.nonzero(sp == 1)[0]
    trans = transitions_lm(2)
    L = 20.0
    step = L / n_scan
    probes = probe_grid(n_scan, n_scan, step, step)
    return _finish("config2", 256, 256, L, L, [2.0] * 50, sl, xy, amp, wid,
                   sl[b], xy[b], trans, probes, (n_scan, n_scan),
                   energy_eV=ENERGY_300KEV, aperture_mrad=21.0, det_inner_mrad=0.0,
                   det_outer_mrad=50.0, interp_f=1, window_A=window_A)


def _bcc_sphere(a=2.87, radius=40.0, centre=(50.0, 50.0, 40.0)):
    n = int(math.ceil(radius / a)) + 1
    g = np.arange(-n, n + 1)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    base = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1).astype(np.float64) * a
    pts = np.concatenate([base, base + 0.5 * a], axis=0)
    r2 = (pts ** 2).sum(axis=1)
    pts = pts[r2 <= radius * radius + 1e-9]
    return pts + np.asarray(centre)[None, :]


def _amorphous(rng, n_atoms, lx, ly, z0, z1, dmin):
    """Random sequential addition in a slab, periodic in x and y."""
    cell = dmin
    ncx, ncy = int(lx // cell), int(ly // cell)
    ncz = int(math.ceil((z1 - z0) / cell)) + 1
    csx, csy = lx / ncx, ly / ncy
    grid = {}
    pts = []
    d2min = dmin * dmin
    tries = 0
    while len(pts) < n_atoms:
        tries += 1
        if tries > 200 * n_atoms:
            raise RuntimeError("amorphous packing failed")
        p = (rng.uniform(0, lx), rng.uniform(0, ly), rng.uniform(z0, z1))
        cx, cy, cz = int(p[0] // csx) % ncx, int(p[1] // csy) % ncy, int((p[2] - z0) // cell)
        ok = True
        for ddx in (-1, 0, 1):
            for ddy in (-1, 0, 1):
                for ddz in (-1, 0, 1):
                    for q in grid.get(((cx + ddx) % ncx, (cy + ddy) % ncy, cz + ddz), ()):
                        dx_ = _min_image(p[0] - q[0], lx)
                        dy_ = _min_image(p[1] - q[1], ly)
                        if dx_ * dx_ + dy_ * dy_ + (p[2] - q[2]) ** 2 < d2min:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            pts.append(p)
            grid.setdefault((cx, cy, cz), []).append(p)
    return np.array(pts)


def config3_atoms(seed=3, n_support=20000):
    rng = np.random.Generator(np.random.PCG64(seed))
    sphere = _bcc_sphere()
    support = _amorphous(rng, n_support, 100.0, 100.0, 80.0, 100.0, 1.2)
    return sphere, support


def config3(seed: int = 3, n_scan: int = 256, det_outer_mrad: float = 20.0,
            n_support: int = 20000, ionise_all: bool = True) -> Problem:
    """1024x1024 px, 100x100 A cell, 50 slices of 2 A: an 80 A bcc sphere
    (a = 2.87 A, pair (50, 12.5) V*A) on a 20 A amorphous support (0.1 atoms/A^3,
    pair (10, 2.5) V*A, 1.2 A minimum distance); f = 4, 4 A crop window; every
    sphere atom ionised with 9 transitions; 256x256 probes at 100/256 A steps."""
    sphere, support = config3_atoms(seed, n_support)
    xy = np.concatenate([sphere[:, :2], support[:, :2]])
    z = np.concatenate([sphere[:, 2], support[:, 2]])
    sl = np.floor(z / 2.0).astype(np.int64)
    amp = np.concatenate([np.tile([[50.0, 12.5]], (len(sphere), 1)),
                          np.tile([[10.0, 2.5]], (len(support), 1))])
    wid = np.tile([[0.3, 0.8]], (len(xy), 1))
    ion = np.arange(len(sphere)) if ionise_all else np.arange(0)
    probes = probe_grid(n_scan, n_scan, 100.0 / n_scan, 100.0 / n_scan)
    return _finish("config3", 1024, 1024, 100.0, 100.0, [2.0] * 50, sl, xy, amp, wid,
                   sl[ion], xy[ion], transitions_lm(2), probes, (n_scan, n_scan),
                   energy_eV=ENERGY_300KEV, aperture_mrad=20.0, det_inner_mrad=0.0,
                   det_outer_mrad=det_outer_mrad, interp_f=4, window_A=4.0)


def config3_subproblem(seed: int = 3, n: int = 256, L: float = 25.0, nz: int = 6,
                       n_scan: int = 8, f: int = 2, window_A: float = 4.0,
                       det_outer_mrad: float = 20.0) -> Problem:
    """A reduced nanoparticle-like cell with the same ingredients (bcc cluster on an
    amorphous layer, f > 1, cropped windows) at a size the oracle finishes fast."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = 2.87
    R = 0.3 * L
    c = (L / 2, L / 2, R)
    pts = _bcc_sphere(a=a, radius=R, centre=c)
    thick = nz * 2.0
    pts = pts[pts[:, 2] < thick - 2.0]
    sup = _amorphous(rng, int(0.02 * L * L * 2.0), L, L, thick - 2.0, thick - 1e-6, 1.2)
    xy = np.concatenate([pts[:, :2], sup[:, :2]])
    z = np.concatenate([pts[:, 2], sup[:, 2]])
    sl = np.floor(z / 2.0).astype(np.int64)
    amp = np.concatenate([np.tile([[50.0, 12.5]], (len(pts), 1)),
                          np.tile([[10.0, 2.5]], (len(sup), 1))])
    wid = np.tile([[0.3, 0.8]], (len(xy), 1))
    # ionise a seeded handful of cluster atoms
    k = min(6, len(pts))
    ion = np.sort(rng.choice(len(pts), size=k, replace=False))
    step = L / (n_scan * f)
    x0 = L / 2 - step * n_scan / 2
    probes = probe_grid(n_scan, n_scan, step, step, x0, x0)
    return _finish("config3_sub", n, n, L, L, [2.0] * nz, sl, xy, amp, wid,
                   sl[ion], xy[ion], transitions_lm(1), probes, (n_scan, n_scan),
                   energy_eV=ENERGY_300KEV, aperture_mrad=20.0, det_inner_mrad=0.0,
                   det_outer_mrad=det_outer_mrad, interp_f=f, window_A=window_A)


def tiled_problem(p: Problem, f: int, probes) -> Problem:
    """The cell of ``p`` repeated f x f times (potential arrays tiled, every site copied into
    each tile with its transition potentials), requested with interpolation factor f at the
    given probe positions.  The copies sit whole numbers of pixels apart, so their windowed
    transition potentials are the same arrays."""
    f = int(f)
    nt = np.asarray(p.site_ntrans, dtype=np.int64)
    shifts = [(i * p.lx, j * p.ly) for j in range(f) for i in range(f)]
    site_xy = np.concatenate([p.site_xy + np.asarray(d)[None, :] for d in shifts])
    blocks = [p.H[int(p.site_hoff[s]):int(p.site_hoff[s]) + int(nt[s])] for s in range(p.n_sites)]
    H = np.concatenate(blocks * len(shifts)) if blocks else p.H[:0]
    ntr = np.tile(nt, len(shifts))
    probes = np.asarray(probes, dtype=np.float64).reshape(-1, 2)
    return p.replace(name=f"{p.name}_tiled{f}", nx=f * p.nx, ny=f * p.ny, lx=f * p.lx, ly=f * p.ly,
                     V=np.tile(p.V, (1, f, f)), H=H, site_slice=np.tile(p.site_slice, len(shifts)),
                     site_xy=site_xy, site_ntrans=ntr.astype(np.int32),
                     site_hoff=np.concatenate([[0], np.cumsum(ntr)[:-1]]).astype(np.int64),
                     probes=probes, probe_shape=(1, probes.shape[0]), interp_f=f)


def random_problem(seed: int, n: int = 32, ny: Optional[int] = None, L: float = 8.0,
                   Ly: Optional[float] = None, nz: int = 3, atoms_per_slice: int = 4,
                   n_sites: int = 2, n_trans: int = 2, window_A: float = 0.0,
                   interp_f: int = 1, aperture_mrad: float = 15.0,
                   det_inner_mrad: float = 0.0, det_outer_mrad: float = 20.0,
                   n_scan: int = 3, amp=(30.0, 8.0), dz=None, probes=None,
                   energy_eV: float = ENERGY_300KEV, defocus_A: float = 0.0,
                   cs_A: float = 0.0, widths=(0.3, 0.8), displace_A: float = 0.0,
                   displace_seed: int = 0) -> Problem:
    """Random atoms and sites on a small periodic cell (test workloads).  `widths`: the two
    Gaussian widths (A) of every atom's projected potential; narrow ones scatter to high
    angles (a 0.3 A Gaussian sends ~1e-14 of the beam beyond 60 mrad at 300 keV).
    displace_A > 0: one frozen-phonon configuration, every atom (and with it its transition
    potentials) displaced in-plane by N(0, displace_A^2) per axis, seeded by displace_seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ny = n if ny is None else ny
    Ly = L if Ly is None else Ly
    na = nz * atoms_per_slice
    a_slice = np.repeat(np.arange(nz), atoms_per_slice)
    a_xy = np.stack([rng.uniform(0, L, na), rng.uniform(0, Ly, na)], axis=1)
    amp_arr = np.tile([list(amp)], (na, 1)) * rng.uniform(0.5, 1.5, (na, 1))
    wid = np.tile([list(widths)], (na, 1))
    sites = rng.choice(na, size=min(n_sites, na), replace=False)
    a_xy = thermal_displacement(a_xy, L, Ly, displace_A, displace_seed)
    allt = transitions_lm(2)
    trans = [allt[i] for i in rng.choice(len(allt), size=n_trans, replace=False)]
    if probes is None:
        probes = np.stack([rng.uniform(0, L, n_scan * n_scan),
                           rng.uniform(0, Ly, n_scan * n_scan)], axis=1)
        shape = (n_scan, n_scan)
    else:
        probes = np.asarray(probes, dtype=np.float64).reshape(-1, 2)
        shape = (1, probes.shape[0])
    dz = [2.0] * nz if dz is None else list(dz)
    return _finish(f"random{seed}", n, ny, L, Ly, dz, a_slice, a_xy, amp_arr, wid,
                   a_slice[sites], a_xy[sites], trans, probes, shape,
                   energy_eV=energy_eV, aperture_mrad=aperture_mrad,
                   det_inner_mrad=det_inner_mrad, det_outer_mrad=det_outer_mrad,
                   interp_f=interp_f, window_A=window_A, defocus_A=defocus_A, cs_A=cs_A)


def random_lattice_specimen(rng, n, nz, n_ion, nt_range=(3, 9), px=0.1, dz=2.0, window_A=4.0,
                            aperture_mrad=20.0, det_outer_mrad=40.0, n_scan=None, name="specimen"):
    """One specimen of the batching workload: a random rectangular lattice (spacing
    U(2.5, 4) A, amplitudes U(15, 60) V*A) on an n x n grid at `px` A/px, f = n/128,
    n_ion ionised lattice atoms with a random number of transitions each."""
    L = n * px
    f = max(1, n // 128)
    a = rng.uniform(2.5, 4.0)
    nc = max(1, int(L // a))
    a = L / nc
    sl, xy, amp = [], [], []
    for j in range(nz):
        off = rng.uniform(0, a, 2)
        for iy in range(nc):
            for ix in range(nc):
                sl.append(j)
                xy.append(((ix * a + off[0]) % L, (iy * a + off[1]) % L))
                A = rng.uniform(15.0, 60.0)
                amp.append((A, A / 4.0))
    sl, xy, amp = np.array(sl), np.array(xy), np.array(amp)
    wid = np.tile([[0.3, 0.8]], (len(sl), 1))
    ion = np.sort(rng.choice(len(sl), size=min(n_ion, len(sl)), replace=False))
    allt = transitions_lm(2)
    nt = int(rng.integers(nt_range[0], nt_range[1] + 1))
    trans = allt[:nt]
    ns = int(n_scan) if n_scan is not None else int(rng.integers(16, 65))
    probes = probe_grid(ns, ns, L / ns, L / ns)
    return _finish(name, n, n, L, L, [dz] * nz, sl, xy, amp, wid, sl[ion], xy[ion], trans, probes,
                   (ns, ns), energy_eV=ENERGY_300KEV, aperture_mrad=aperture_mrad, det_inner_mrad=0.0,
                   det_outer_mrad=det_outer_mrad, interp_f=f, window_A=window_A)


def _pool_one(args):
    seed, n, nz, ni, ns, name = args
    return random_lattice_specimen(np.random.Generator(np.random.PCG64(seed)), n, nz, ni, n_scan=ns, name=name)


def specimen_pool(seed: int, n_specimens: int, sizes, slices, ions, scans, prefix: str = "specimen",
                  workers: int = 1) -> List[Problem]:
    """Random-lattice specimens with sizes, slice counts, ionised atoms and probe rasters
    drawn from a seed; every specimen has its own sub-seed, so `workers` processes give
    the same result as one."""
    rng = np.random.Generator(np.random.PCG64(seed))
    args = []
    for k in range(n_specimens):
        n = int(rng.choice(sizes))
        nz = int(rng.integers(slices[0], slices[1] + 1))
        ni = int(rng.integers(ions[0], ions[1] + 1))
        ns = int(rng.integers(scans[0], scans[1] + 1))
        args.append((int(rng.integers(0, 2**62)), n, nz, ni, ns, f"{prefix}_{k}"))
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            return pool.map(_pool_one, args)
    return [_pool_one(a) for a in args]


def config4(seed: int = 4, n_specimens: int = 64, sizes=(128, 256, 384, 512), slices=(10, 80),
            ions=(1, 20), scans=(16, 64), workers: int = 1) -> List[Problem]:
    """The batching workload: specimens of uneven size drawn from a seed (grids 128^2, 256^2,
    384^2 and 512^2 at 0.1 A/px with f = N/128, 10-80 slices of 2 A, 1-20 ionised atoms with
    3-9 transitions each, 16^2 to 64^2 probes, 4 A crop, 20 mrad aperture, 0-40 mrad
    detector)."""
    return specimen_pool(seed, n_specimens, sizes, slices, ions, scans, "config4", workers)


def config5_stream(seed: int = 5, rate_per_s: float = 1.0, n_requests: int = 40, repeat_frac: float = 0.3,
                   pool=None):
    """Poisson request stream for the serving workload: (arrival time, specimen index,
    probe shift).  A fraction `repeat_frac` of requests repeats an earlier specimen with
    a shifted probe raster (S-matrix residency)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    reqs = []
    seen = []
    n_pool = len(pool) if pool is not None else n_requests
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        if seen and rng.uniform() < repeat_frac:
            k = int(rng.choice(seen))
            shift = float(rng.uniform(0.0, 1.0))
        else:
            k = int(rng.integers(0, n_pool))
            shift = 0.0
        seen.append(k)
        reqs.append((t, k, shift))
    return reqs
