"""Seeded synthetic inputs for the direct scattering sum.

This module only builds inputs: atom sites, displacement fields, per-atom
scattering factors and reciprocal-space point lists.  It contains none of the
sum's own arithmetic, imports neither the GPU library nor the CPU oracle, and is
the one module both sides draw their inputs from.

Conventions (Favre-Nicolin et al., 2010):

* positions r in lattice units and S in reciprocal-lattice units (r.l.u.), so S.r
  is in cycles -- Section 4.2 converts orthonormal coordinates to fractional ones
  before calling the sum;
* inputs are built in float64 and rounded once to float32; the float32 arrays are
  the problem both sides evaluate;
* atoms are listed with the x cell index slowest, z fastest and the fcc basis
  innermost; point grids with h fastest, then k, then l (any order is valid for
  the sum, Section 3 notes that shape and order are irrelevant);
* ``f`` is None when every atom has f_j = 1 (the unit-occupancy sum of Section 3
  and of the speed tests of Section 2.2), else a complex64 array.

The five named workloads are the synthetic stand-ins for the paper's strained
nanostructures (its coordinate files and scripts are not available):

* ``c1`` 16^3 simple-cubic block, Gaussian disorder 0.02, f=1, 64x64 map at l=4;
* ``c2`` Ge-like truncated-pyramid dot on an fcc lattice with radial strain and a
  20->80 % composition profile (cf. the Ge dot of Section 4.3), 128^3 grid at (404);
* ``c3`` 100^3 simple-cubic crystal (the Section 4.1 cube size), disorder 0.01,
  256x256 map near (8,8,8): phases up to ~2.4e3 cycles;
* ``c4`` 29^3-cell fcc cube with a sinusoidal displacement field, 64^3 grid at (220),
  plus the perturbed target structure whose intensity is fitted;
* ``c5`` fcc nanowire segment with radial and axial strain, core/shell species,
  256^3 grid at (004), plus a target structure with strain x1.1.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# fcc basis in lattice units (a = 1)
FCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])

# two species' complex scattering factors (Ge-like and a lighter partner), constant
# over the small S windows used here
F_SPECIES_0 = complex(31.0, 1.0)
F_SPECIES_1 = complex(22.0, 3.5)


@dataclass(frozen=True)
class RegularGrid:
    """A regular grid of points given exactly: point (i1, i2, i3) is origin + i1 step1 +
    i2 step2 + i3 step3 (float64), 0 <= i_a < n_a, listed with i1 fastest."""
    origin: tuple
    step1: tuple
    step2: tuple
    step3: tuple
    n1: int
    n2: int = 1
    n3: int = 1

    @property
    def size(self) -> int:
        return self.n1 * self.n2 * self.n3

    def points(self, idx=None) -> np.ndarray:
        """The grid points (or those of the flat indices idx), float64 (K, 3)."""
        k = np.arange(self.size, dtype=np.int64) if idx is None else np.asarray(idx, dtype=np.int64)
        i1 = (k % self.n1).astype(np.float64)
        i2 = ((k // self.n1) % self.n2).astype(np.float64)
        i3 = (k // (self.n1 * self.n2)).astype(np.float64)
        return (np.asarray(self.origin, np.float64)[None, :] + i1[:, None] * np.asarray(self.step1)[None, :]
                + i2[:, None] * np.asarray(self.step2)[None, :] + i3[:, None] * np.asarray(self.step3)[None, :])


def axis_grid(h, k, l) -> RegularGrid:
    """The grid of grid_points(h, k, l) for axes given as (start, step, count) or as a
    single value: h along x (fastest), k along y, l along z."""
    axes = []
    for v in (h, k, l):
        axes.append((float(v[0]), float(v[1]), int(v[2])) if isinstance(v, tuple) else (float(v), 0.0, 1))
    (h0, dh, nh), (k0, dk, nk), (l0, dl, nl) = axes
    return RegularGrid((h0, k0, l0), (dh, 0.0, 0.0), (0.0, dk, 0.0), (0.0, 0.0, dl), nh, nk, nl)


def linspace_axis(lo: float, hi: float, n: int, centre: float = 0.0):
    """(start, step, count) of centre + linspace(lo, hi, n)."""
    return (centre + lo, (hi - lo) / (n - 1), n)


@dataclass
class Workload:
    """One synthetic problem: atoms, factors, points (all float32 / complex64).  Where the
    points are a regular grid, ``grid`` gives it exactly (S is that grid rounded to
    float32, the list the point-list calls take)."""
    name: str
    xyz: np.ndarray                      # (N, 3) float32
    f: Optional[np.ndarray]              # (N,) complex64 or None for f_j = 1
    S: np.ndarray                        # (K, 3) float32
    target_xyz: Optional[np.ndarray] = None   # (N, 3) float32: structure whose |A|^2 is fitted
    meta: dict = field(default_factory=dict)
    grid: Optional[RegularGrid] = None

    @property
    def n_atoms(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_points(self) -> int:
        return int(self.S.shape[0])


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def cubic_sites(nx: int, ny: int, nz: int, origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Simple-cubic sites n = (ix, iy, iz) + origin, x slowest, z fastest, float64."""
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    p = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    return p + np.asarray(origin, dtype=np.float64)


def fcc_sites(xr, yr, zr) -> np.ndarray:
    """fcc sites for cells ix in range(*xr) etc., basis innermost, float64."""
    ix, iy, iz = np.meshgrid(np.arange(*xr), np.arange(*yr), np.arange(*zr), indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    return (cells[:, None, :] + FCC_BASIS[None, :, :]).reshape(-1, 3)


def grid_points(h, k, l) -> np.ndarray:
    """All (h, k, l) combinations with h fastest, then k, then l, float64 (K, 3)."""
    h = np.atleast_1d(np.asarray(h, dtype=np.float64))
    k = np.atleast_1d(np.asarray(k, dtype=np.float64))
    l = np.atleast_1d(np.asarray(l, dtype=np.float64))
    L, K, H = np.meshgrid(l, k, h, indexing="ij")
    return np.stack([H.ravel(), K.ravel(), L.ravel()], axis=1)


# ----------------------------------------------------------------------------- named workloads

def c1(seed: int = 1001, sigma: float = 0.02) -> Workload:
    """16^3 simple-cubic block (4096 atoms) + N(0, sigma^2) per component, f = 1;
    64x64 map (h, k, 4), h, k in linspace(-0.5, 0.5, 64)."""
    rng = np.random.default_rng(seed)
    p = cubic_sites(16, 16, 16)
    if sigma:
        p = p + rng.normal(0.0, sigma, size=p.shape)
    d = np.linspace(-0.5, 0.5, 64)
    S = grid_points(d, d, 4.0)
    a = linspace_axis(-0.5, 0.5, 64)
    return Workload("c1", _f32(p), None, _f32(S), meta=dict(sigma=sigma, seed=seed),
                    grid=axis_grid(a, a, 4.0))


def _pyramid_mask(p):
    z = p[:, 2]
    half = 32.0 - 16.0 * z / 21.0
    return (z >= 0) & (z < 21) & (np.abs(p[:, 0]) < half) & (np.abs(p[:, 1]) < half)


def _radial_displacement(p, amp, R=16.0):
    """u = amp * R * (1 - exp(-rho/R)) * rho_hat about the origin (strain amp*exp(-rho/R))."""
    rho = np.linalg.norm(p, axis=1)
    scale = np.zeros_like(rho)
    nz = rho > 0
    scale[nz] = amp * R * (1.0 - np.exp(-rho[nz] / R)) / rho[nz]
    return p * scale[:, None]


def c2(seed: int = 1002, n_grid: int = 128, strain: float = 0.04) -> Workload:
    """Ge-like truncated square pyramid on fcc (a=1): 0 <= z < 21, |x|,|y| < 32 - 16 z/21
    (203,557 atoms); radial strain eps(rho) = strain*exp(-rho/16) about the base centre;
    species Bernoulli(p = 0.2 + 0.6 z/21) -> F_SPECIES_0 else F_SPECIES_1;
    grid (4+d, d, 4+d), d in linspace(-0.05, 0.05, n_grid)^3.  The target structure
    (for a fit step) has the strain scaled by 1.1."""
    rng = np.random.default_rng(seed)
    p0 = fcc_sites((-32, 32), (-32, 32), (0, 21))
    p0 = p0[_pyramid_mask(p0)]
    ge = rng.random(p0.shape[0]) < (0.2 + 0.6 * p0[:, 2] / 21.0)
    f = np.where(ge, F_SPECIES_0, F_SPECIES_1).astype(np.complex64)
    p = p0 + _radial_displacement(p0, strain)
    pt = p0 + _radial_displacement(p0, strain * 1.1)
    d = np.linspace(-0.05, 0.05, n_grid)
    S = grid_points(4.0 + d, d, 4.0 + d)
    return Workload("c2", _f32(p), f, _f32(S), target_xyz=_f32(pt),
                    meta=dict(seed=seed, strain=strain),
                    grid=axis_grid(linspace_axis(-0.05, 0.05, n_grid, 4.0), linspace_axis(-0.05, 0.05, n_grid),
                                   linspace_axis(-0.05, 0.05, n_grid, 4.0)))


def c3(seed: int = 1003, sigma: float = 0.01, n_side: int = 100, n_grid: int = 256) -> Workload:
    """100^3 simple-cubic crystal (1e6 atoms) + N(0, sigma^2), f = 1;
    map (8+d, 8+d, 8), d in linspace(-0.05, 0.05, 256)^2 (65,536 points)."""
    rng = np.random.default_rng(seed)
    p = cubic_sites(n_side, n_side, n_side)
    if sigma:
        p = p + rng.normal(0.0, sigma, size=p.shape)
    d = np.linspace(-0.05, 0.05, n_grid)
    S = grid_points(8.0 + d, 8.0 + d, 8.0)
    a = linspace_axis(-0.05, 0.05, n_grid, 8.0)
    return Workload("c3", _f32(p), None, _f32(S), meta=dict(seed=seed, sigma=sigma),
                    grid=axis_grid(a, a, 8.0))


def _sine_field(p0, amp, phase):
    """u = amp * (sin(2 pi z/20 + phase), sin(2 pi x/20 + phase), sin(2 pi y/20 + phase))."""
    w = 2.0 * np.pi / 20.0
    return amp * np.stack([np.sin(w * p0[:, 2] + phase),
                           np.sin(w * p0[:, 0] + phase),
                           np.sin(w * p0[:, 1] + phase)], axis=1)


def c4(seed: int = 1004, n_cells: int = 29, n_grid: int = 64) -> Workload:
    """fcc cube of 29^3 cells (97,556 atoms), u = 0.03 sin(2 pi (z, x, y)/20), f = 1;
    grid (2+d, 2+d, d), d in linspace(-0.08, 0.08, 64)^3 (262,144 points).
    Target structure: amplitude 0.033 and phase +0.3 rad in each sine."""
    p0 = fcc_sites((0, n_cells), (0, n_cells), (0, n_cells))
    p = p0 + _sine_field(p0, 0.03, 0.0)
    pt = p0 + _sine_field(p0, 0.033, 0.3)
    d = np.linspace(-0.08, 0.08, n_grid)
    S = grid_points(2.0 + d, 2.0 + d, d)
    a = linspace_axis(-0.08, 0.08, n_grid, 2.0)
    return Workload("c4", _f32(p), None, _f32(S), target_xyz=_f32(pt), meta=dict(seed=seed),
                    grid=axis_grid(a, a, linspace_axis(-0.08, 0.08, n_grid)))


def _wire_displacement(p0, scale):
    rho2 = p0[:, 0] ** 2 + p0[:, 1] ** 2
    rho = np.sqrt(rho2)
    u = np.zeros_like(p0)
    ur = scale * 0.005 * rho2 / 40.0             # radial, eps_rr = 0.01 rho/40
    nz = rho > 0
    u[nz, 0] = ur[nz] * p0[nz, 0] / rho[nz]
    u[nz, 1] = ur[nz] * p0[nz, 1] / rho[nz]
    u[:, 2] = scale * 0.002 * (p0[:, 2] - 100.0) * rho2 / 1600.0   # axial
    return u


def c5(seed: int = 1005, n_grid: int = 256) -> Workload:
    """fcc cylinder along z, rho < 40, 0 <= z < 200 (4,013,800 atoms); radial
    u_rho = 0.005 rho^2/40, axial u_z = 0.002 (z-100)(rho/40)^2; core (rho < 28)
    F_SPECIES_0, shell F_SPECIES_1; grid (d, d, 4+d), d in linspace(-0.05, 0.05, 256)^3
    (16,777,216 points).  Target structure: the same wire with strain x1.1."""
    p0 = fcc_sites((-40, 40), (-40, 40), (0, 200))
    rho = np.sqrt(p0[:, 0] ** 2 + p0[:, 1] ** 2)
    keep = rho < 40.0
    p0, rho = p0[keep], rho[keep]
    f = np.where(rho < 28.0, F_SPECIES_0, F_SPECIES_1).astype(np.complex64)
    p = p0 + _wire_displacement(p0, 1.0)
    pt = p0 + _wire_displacement(p0, 1.1)
    d = np.linspace(-0.05, 0.05, n_grid)
    S = grid_points(d, d, 4.0 + d)
    a = linspace_axis(-0.05, 0.05, n_grid)
    return Workload("c5", _f32(p), f, _f32(S), target_xyz=_f32(pt), meta=dict(seed=seed),
                    grid=axis_grid(a, a, linspace_axis(-0.05, 0.05, n_grid, 4.0)))


# ----------------------------------------------------------------------------- unstructured points

GE_A = 5.658            # Ge lattice constant (angstrom): converts r.l.u. to 1/angstrom
HC_KEV_A = 12.39842     # h c in keV.angstrom: wavelength = HC_KEV_A / energy


def _rotate(v, axis, angle):
    """Rodrigues rotation of the rows of v about the unit vector axis."""
    c, s = np.cos(angle), np.sin(angle)
    return v * c + np.cross(axis, v) * s + np.outer(v @ axis, axis) * (1.0 - c)


def ewald_geometry(hkl, a=GE_A, energy_kev=8.0):
    """Symmetric Bragg geometry for node hkl of a cubic crystal with lattice constant a:
    returns (wavelength, unit incident direction, unit exit direction, unit normal of
    the scattering plane), all in the crystal frame, with k_f - k_i = hkl / a (in
    1/angstrom, crystallographic convention, no 2 pi)."""
    G = np.asarray(hkl, dtype=np.float64) / a
    lam = HC_KEV_A / energy_kev
    sin_t = 0.5 * lam * np.linalg.norm(G)
    if not 0.0 < sin_t < 1.0:
        raise ValueError(f"node {hkl} is not reachable at {energy_kev} keV")
    cos_t = np.sqrt(1.0 - sin_t * sin_t)
    g = G / np.linalg.norm(G)
    ref = np.array([0.0, 1.0, 0.0]) if abs(g[1]) < 0.9 else np.array([1.0, 0.0, 0.0])
    n = ref - (ref @ g) * g
    n /= np.linalg.norm(n)
    ki = -sin_t * g + cos_t * n
    kf = sin_t * g + cos_t * n
    normal = np.cross(ki, kf)
    normal /= np.linalg.norm(normal)
    return lam, ki, kf, normal


def ewald_scan(hkl, a=GE_A, energy_kev=8.0, distance=0.5, pitch=55e-6, n_pix=(128, 128),
               n_frames=128, rock_deg=0.5) -> np.ndarray:
    """The reciprocal-space points (r.l.u., float64 (K, 3)) recorded by a flat 2D detector
    during a rocking scan about node hkl: the detector (n_pix pixels of size `pitch`, at
    `distance` metres, centred on the exit beam of the Bragg condition) measures points on
    Ewald's sphere, S = (k_hat - k_i_hat) / wavelength; rocking the crystal by omega about
    the normal of the scattering plane rotates that curved sheet in the crystal frame.
    n_frames = 1 gives one detector frame (no rotation).  Points are listed frame by
    frame, detector rows, then columns fastest.  Neither a frame nor the scan is a grid
    of the reciprocal lattice: this is the unstructured point set that motivates the
    direct sum (Section 1)."""
    lam, ki, kf, normal = ewald_geometry(hkl, a, energy_kev)
    e1 = np.cross(normal, kf)                   # in the scattering plane, across the beam
    e2 = normal
    n1, n2 = n_pix
    u = (np.arange(n1) - 0.5 * (n1 - 1)) * pitch
    v = (np.arange(n2) - 0.5 * (n2 - 1)) * pitch
    U, V = np.meshgrid(u, v, indexing="ij")
    p = distance * kf[None, :] + U.reshape(-1, 1) * e1[None, :] + V.reshape(-1, 1) * e2[None, :]
    k_hat = p / np.linalg.norm(p, axis=1, keepdims=True)
    frame = (k_hat - ki[None, :]) / lam * a                 # r.l.u.
    if n_frames == 1:
        return frame
    omegas = np.deg2rad(np.linspace(-rock_deg, rock_deg, n_frames))
    return np.concatenate([_rotate(frame, normal, w) for w in omegas])


def ewald(seed: int = 1002, n_pix: int = 128, n_frames: int = 128) -> Workload:
    """The C2 dot measured as an area detector records it: 8 keV, detector at 0.5 m with
    55 um pixels (128 x 128) centred on the (4,0,4) exit beam, 128 frames over a
    +-0.5 degree rocking scan: 2,097,152 points on curved sheets spanning about the C2
    window.  Atoms, factors and the fit target are those of C2."""
    w = c2(seed)
    S = ewald_scan((4.0, 0.0, 4.0), n_pix=(n_pix, n_pix), n_frames=n_frames)
    return Workload("ewald", w.xyz, w.f, _f32(S), target_xyz=w.target_xyz,
                    meta=dict(seed=seed, detector=dict(n_pix=n_pix, n_frames=n_frames)))


def cube41(strained: bool = False) -> Workload:
    """The Section 4.1 example: 100 x 100 x 100 simple-cubic cells, x, y in [-50, 50),
    z in [0, 100), f = 1, on the 200 x 200 map h in [-0.1, 0.1), k = 0, l in [3.9, 4.1)
    with 0.001 steps (40,000 points around (004)); strained: z += 1e-6 z (x^2 + y^2)."""
    x = np.arange(-50, 50, dtype=np.float32).astype(np.float64)
    z = np.arange(0, 100, dtype=np.float32).astype(np.float64)
    X, Y, Z = np.meshgrid(x, x, z, indexing="ij")
    if strained:
        Z = Z + 1e-6 * Z * (X * X + Y * Y)
    p = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    h = np.arange(-0.1, 0.1, 0.001)[:200]
    l = np.arange(3.9, 4.1, 0.001)[:200]
    S = grid_points(h, 0.0, l)
    return Workload("cube41s" if strained else "cube41", _f32(p), None, _f32(S),
                    meta=dict(strained=strained),
                    grid=axis_grid((-0.1, 0.001, 200), 0.0, (3.9, 0.001, 200)))


NAMED = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5, "ewald": ewald, "cube41": cube41,
         "cube41s": lambda: cube41(True)}


def named(name: str) -> Workload:
    return NAMED[name]()


# ----------------------------------------------------------------------------- generic inputs

def random_problem(n_atoms: int, n_points: int, seed: int, extent: float = 50.0,
                   s_range: float = 4.0, complex_f: bool = True):
    """Random atoms in [0, extent)^3, random S in [-s_range, s_range)^3 (the paper's
    speed test uses random atoms and random points, Section 2.2).  Returns
    (xyz float32 (N,3), f complex64 (N,) or None, S float32 (K,3))."""
    rng = np.random.default_rng(seed)
    xyz = _f32(rng.random((n_atoms, 3)) * extent)
    S = _f32((rng.random((n_points, 3)) * 2.0 - 1.0) * s_range)
    f = None
    if complex_f:
        f = (rng.uniform(0.5, 2.0, n_atoms) * np.exp(1j * rng.uniform(-np.pi, np.pi, n_atoms)))
        f = f.astype(np.complex64)
    return xyz, f, S


def random_seed_field(n_points: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """A seeded complex64 adjoint seed G (standard complex normal * scale)."""
    rng = np.random.default_rng(seed)
    g = (rng.normal(size=n_points) + 1j * rng.normal(size=n_points)) * scale
    return g.astype(np.complex64)


def random_amplitudes(n_points: int, seed: int, scale: float = 100.0):
    """Seeded complex64 amplitudes A and float32 intensities I of the same scale,
    for exercising the misfit step on its own."""
    rng = np.random.default_rng(seed)
    A = ((rng.normal(size=n_points) + 1j * rng.normal(size=n_points)) * scale).astype(np.complex64)
    I = (rng.gamma(1.0, 2.0 * scale * scale, size=n_points)).astype(np.float32)
    return A, I


def chain(n_atoms: int, sigma: float = 0.0, seed: int = 7, h_step: float = 0.001,
          h_max: float = 1.0):
    """The accuracy test of Section 2.3: atoms at 0, 1, ..., N-1 along x (optionally with
    Gaussian disorder sigma in each component) and H from 0 to h_max every h_step r.l.u.
    along x.  Returns (xyz float32, S float32)."""
    rng = np.random.default_rng(seed)
    p = np.zeros((n_atoms, 3))
    p[:, 0] = np.arange(n_atoms)
    if sigma:
        p = p + rng.normal(0.0, sigma, size=p.shape)
    h = np.arange(0.0, h_max + 0.5 * h_step, h_step)
    S = np.zeros((h.size, 3))
    S[:, 0] = h
    return _f32(p), _f32(S)


# ----------------------------------------------------------------------------- species inputs

def group_by_species(xyz: np.ndarray, f: np.ndarray):
    """Reorder the atoms species by species (stable within a species) for the
    species-factorised sum of Section 4.2.  Returns (xyz reordered, species_start
    list of n_species + 1 offsets, the distinct factors in species order, the
    permutation applied)."""
    vals, inv = np.unique(np.asarray(f), return_inverse=True)
    order = np.argsort(inv, kind="stable")
    counts = np.bincount(inv, minlength=len(vals))
    start = [0] + np.cumsum(counts).astype(int).tolist()
    return np.ascontiguousarray(xyz[order]), start, vals.astype(np.complex64), order


def species_factor_table(S: np.ndarray, f_species, b_iso=(1.2, 0.6), anomalous=None) -> np.ndarray:
    """S-dependent species factors fs[s, k] = Re(f_s) exp(-b_s |S|^2 / 4) + i Im(f_s)
    (+ an optional per-species anomalous complex term): a Debye-Waller-like decay of the
    normal part with |S| standing in for the tabulated f0(|S|) the paper folds out of
    the sum, and an S-independent resonant part.  complex64 (n_species, K)."""
    S = np.asarray(S, dtype=np.float64)
    s2 = np.sum(S * S, axis=1)
    rows = []
    for s, fv in enumerate(f_species):
        b = b_iso[s % len(b_iso)]
        row = np.real(fv) * np.exp(-b * s2 / 4.0) + 1j * np.imag(fv)
        if anomalous is not None:
            row = row + anomalous[s]
        rows.append(row)
    return np.asarray(rows).astype(np.complex64)
