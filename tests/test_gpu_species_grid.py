"""The species-factorised sum of Section 4.2 over a regular grid of points
(nx_scatter_fwd_species_grid, nx_scatter_bwd_species_grid): each species' unit-factor sum
walked over the grid as the grid entry points walk it, times that species' factor at each
point, against the FP64 oracle evaluated at the same FP64 grid points, element by element.

* Rows of a multiple of 64 points (the row kernels, every block shape the plan picks for
  species of a few hundred to 70,000 atoms) and rows of 50 points (the point-list kernels
  over FP64 grid points); empty species, species whose first atom is not a multiple of the
  group size, chunked launches, an empty grid.
* The adjoint: positions (each species' seed G conj(fs[s]) through the grid adjoint) and
  the factor gradient G conj(A_species[s])."""
import numpy as np
import pytest
import torch

import oracle
from paper_1010_2641_amd import api, workloads as wl
from tests import metrics as M
from tests.test_gpu_grid import oblique
from tests.test_gpu_species import cplx_t3, dev, host, species_scale

pytestmark = pytest.mark.gpu


def species_grid_problem(counts, grid, seed, extent=40.0):
    rng = np.random.default_rng(seed)
    n = int(sum(counts))
    xyz = (rng.random((n, 3)) * extent).astype(np.float32)
    start = [0] + np.cumsum(counts).astype(int).tolist()
    base = [complex(31, 1), complex(22, 3.5), complex(8, 0.2), complex(14, -0.5)]
    fs = wl.species_factor_table(grid.points(), [base[s % 4] for s in range(len(counts))],
                                 b_iso=(1.2, 0.6, 0.3, 0.9))
    return xyz, start, fs


CASES = [((128, 3, 2), (1200, 1801)),          # 8-atom groups: one point per lane
         ((128, 2, 2), (70001, 333, 66001)),   # 2 x 2 x 2 blocks beside one point per lane;
                                               # species starting off the group boundaries
         ((64, 4, 3), (0, 700, 1, 333)),       # empty species, a single atom
         ((256, 2, 3), (5, 9, 1000, 0, 17)),
         ((50, 7, 3), (2000, 1500))]           # rows of 50: the point-list kernels


@pytest.mark.parametrize("shape,counts", CASES)
def test_species_grid_forward(shape, counts):
    grid = oblique(*shape)
    xyz, start, fs = species_grid_problem(counts, grid, seed=sum(counts) + shape[0])
    print(f"case species grid fwd {shape} counts={counts}", flush=True)
    A, As = api.scatter_fwd_species_grid(dev(xyz), start, dev(fs), grid, return_species=True)
    A, As = host(A), host(As)
    A_ref, As_ref = oracle.forward_species(xyz, start, fs, grid.points())
    e = float(np.max(np.abs(A - A_ref) / species_scale(fs, start)))
    es = max(float(np.max(np.abs(As[s] - As_ref[s]))) / np.sqrt(max(start[s + 1] - start[s], 1))
             for s in range(len(counts)))
    print(f"  pointwise/scale={e:.3e} per-species={es:.3e}", flush=True)
    assert e <= M.INC_TOL and es <= M.INC_TOL


def test_species_grid_unit_factors_equal_the_grid_sum():
    """fs = None: every factor is 1, so the result is the grid sum of Eq. 2 with f = 1."""
    grid = oblique(128, 4, 2)
    xyz, start, _ = species_grid_problem((3000, 0, 2500), grid, seed=61)
    A = host(api.scatter_fwd_species_grid(dev(xyz), start, None, grid))
    B = host(api.scatter_fwd_grid(dev(xyz), None, grid))
    ref = oracle.forward(xyz, None, grid.points())
    assert M.incoherent(A, ref, None, len(xyz)) <= M.INC_TOL
    assert M.incoherent(A, B, None, len(xyz)) <= 2 * M.INC_TOL


@pytest.mark.parametrize("shape,counts", [((128, 3, 2), (1200, 1801)), ((64, 4, 3), (0, 700, 1, 333)),
                                          ((50, 7, 3), (2000, 1500)), ((128, 2, 2), (3, 0))])
def test_species_grid_adjoint(shape, counts):
    grid = oblique(*shape)
    xyz, start, fs = species_grid_problem(counts, grid, seed=2 * sum(counts) + shape[1])
    G = wl.random_seed_field(grid.size, seed=62)
    print(f"case species grid bwd {shape} counts={counts}", flush=True)
    _, As = api.scatter_fwd_species_grid(dev(xyz), start, dev(fs), grid, return_species=True)
    gx, gfs = api.scatter_bwd_species_grid(dev(xyz), start, dev(fs), grid, dev(G.astype(np.complex64)), As)
    gx, gfs = host(gx), host(gfs)
    _, As_ref = oracle.forward_species(xyz, start, fs, grid.points())
    gx_ref, gfs_ref = oracle.adjoint_species(xyz, start, fs, grid.points(), G, As_ref)
    en, em = M.t3(gx, gx_ref)
    fn_, fm = cplx_t3(gfs, gfs_ref)
    print(f"  grad_xyz T3 {en:.3e}/{em:.3e}  grad_fs T3 {fn_:.3e}/{fm:.3e}", flush=True)
    assert en <= M.T3_NORM_TOL and em <= M.T3_MAX_TOL
    assert fn_ <= M.T3_NORM_TOL and fm <= M.T3_MAX_TOL


def test_species_grid_chunked_launches(monkeypatch):
    """Species sums carried across launch chunks (forward) and the adjoint's chunks of
    points, with an empty species among them."""
    monkeypatch.setenv("NX_TUNE_LAUNCH_PAIRS", str(1 << 20))
    grid = oblique(128, 6, 4)
    xyz, start, fs = species_grid_problem((1500, 0, 2100), grid, seed=63)
    G = wl.random_seed_field(grid.size, seed=64)
    A, As = api.scatter_fwd_species_grid(dev(xyz), start, dev(fs), grid, return_species=True)
    gx, _ = api.scatter_bwd_species_grid(dev(xyz), start, dev(fs), grid, dev(G.astype(np.complex64)))
    A, gx = host(A), host(gx)
    A_ref, As_ref = oracle.forward_species(xyz, start, fs, grid.points())
    gx_ref, _ = oracle.adjoint_species(xyz, start, fs, grid.points(), G, As_ref)
    assert float(np.max(np.abs(A - A_ref) / species_scale(fs, start))) <= M.INC_TOL
    assert M.t3(gx, gx_ref)[0] <= M.T3_NORM_TOL


def test_species_grid_empty():
    """An empty grid: empty A; the position gradient is zero."""
    grid = oblique(64, 0, 3)
    xyz = np.random.default_rng(65).random((64, 3)).astype(np.float32) * 30
    start, fs = [0, 40, 64], np.zeros((2, 0), np.complex64)
    A, As = api.scatter_fwd_species_grid(dev(xyz), start, dev(fs), grid, return_species=True)
    assert A.numel() == 0 and As.shape == (2, 0)
    G = torch.zeros(0, dtype=torch.complex64, device="cuda:0")
    gx, gfs = api.scatter_bwd_species_grid(dev(xyz), start, dev(fs), grid, G, As)
    assert np.all(host(gx) == 0) and gfs.shape == (2, 0)


def test_species_grid_no_atoms():
    """Every species empty: A is zero at every point; the adjoint has no atoms to write and
    the factor gradient is G conj(0) = 0."""
    grid = oblique(128, 2, 2)
    xyz = np.zeros((0, 3), np.float32)
    fs = wl.species_factor_table(grid.points(), [complex(31, 1), complex(8, 0.2)], b_iso=(1.2, 0.6))
    A, As = api.scatter_fwd_species_grid(dev(xyz), [0, 0, 0], dev(fs), grid, return_species=True)
    assert host(A).shape == (grid.size,) and np.all(host(A) == 0) and np.all(host(As) == 0)
    G = dev(wl.random_seed_field(grid.size, seed=66).astype(np.complex64))
    gx, gfs = api.scatter_bwd_species_grid(dev(xyz), [0, 0, 0], dev(fs), grid, G, As)
    assert host(gx).shape == (0, 3) and np.all(host(gfs) == 0)


def test_c2_species_grid_every_point_against_the_f64_path():
    """C2 regrouped by species (two species, each factor constant over S) over its exact
    128^3 grid: the species-factorised forward against the all-FP64 per-atom path on every
    point (T1, T2), and its adjoint at a seed against the all-FP64 adjoint on 4,096 atoms
    and against the per-atom grid adjoint on every atom."""
    w = wl.c2()
    grid = w.grid
    xs, start, vals, order = wl.group_by_species(w.xyz, w.f)
    fs = np.repeat(vals[:, None], grid.size, axis=1).astype(np.complex64)
    f_sorted = w.f[order]
    print(f"case c2 species grid: {w.n_atoms} atoms in {len(vals)} species x {grid.size} points",
          flush=True)
    A = host(api.scatter_fwd_species_grid(dev(xs), start, dev(fs), grid))
    A64 = host(api.scatter_fwd_f64(dev(xs.astype(np.float64)), dev(f_sorted.astype(np.complex128)),
                                   dev(grid.points())))
    e1, e2 = M.t1(A, A64), M.t2(A, A64)
    print(f"  forward, every point: T1={e1:.3e} T2={e2:.3e}", flush=True)
    assert e1 <= M.T1_TOL and e2 <= M.T2_TOL
    G = dev(wl.random_seed_field(grid.size, seed=67).astype(np.complex64))
    gx, _ = api.scatter_bwd_species_grid(dev(xs), start, dev(fs), grid, G)
    gx = host(gx)
    gp = host(api.scatter_bwd_grid(dev(xs), dev(f_sorted), grid, G))
    pn, pm = M.t3(gx, gp)
    print(f"  adjoint vs per-atom grid adjoint: T3 norm={pn:.3e} max={pm:.3e}", flush=True)
    assert pn <= 2 * M.T3_NORM_TOL and pm <= 2 * M.T3_MAX_TOL
    atoms = np.sort(np.random.default_rng(68).choice(w.n_atoms, size=4096, replace=False))
    g64 = host(api.scatter_bwd_f64(dev(xs[atoms].astype(np.float64)),
                                   dev(f_sorted[atoms].astype(np.complex128)), dev(grid.points()),
                                   G.to(torch.complex128)))
    en, em = M.t3(gx[atoms], g64)
    print(f"  adjoint vs all-FP64 path (4096 atoms): T3 norm={en:.3e} max={em:.3e}", flush=True)
    assert en <= M.T3_NORM_TOL and em <= M.T3_MAX_TOL
