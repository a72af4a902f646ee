"""The grid entry points (nx_scatter_fwd_grid, nx_scatter_bwd_grid, nx_fit_step_grid): the
sums of Eq. 2 and its adjoint over a regular grid of points given exactly (FP64 origin and
steps), against the FP64 oracle evaluated at the same FP64 grid points.

* Rows of a multiple of 64 points take the row-walking kernels: the phase is i1 (step1.r)
  plus a row term formed once per atom and row.  Other grids take the point-list kernels
  with every grid point formed in FP64.  Both meet the point-list calls' tolerances
  (random atoms: pointwise error against sqrt(sum |f|^2); adjoint: T3).
* Oblique steps, complex and unit factors, ragged point and atom counts, chunked
  launches and stream splits, empty calls, tiles beyond the fixed-point range.
* The fit step in one call equals its three calls bitwise.
* C2 at full size (203,557 atoms, 128^3 points) in the launch configuration of a full call,
  on sampled points and atoms."""
import numpy as np
import pytest
import torch

import oracle
from paper_1010_2641_amd import api, workloads as wl
from tests import metrics as M

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def oblique(n1, n2, n3, origin=(3.9, 0.1, 4.1)):
    return wl.RegularGrid(origin, (0.013, 0.004, -0.002), (-0.003, 0.011, 0.001), (0.002, -0.001, 0.017),
                          n1, n2, n3)


def fwd(xyz, f, grid):
    A = api.scatter_fwd_grid(dev(xyz), dev(f), grid)
    torch.cuda.synchronize()
    return A.cpu().numpy().astype(np.complex128)


def bwd(xyz, f, grid, G):
    g = api.scatter_bwd_grid(dev(xyz), dev(f), grid, dev(G.astype(np.complex64)))
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.float64)


SHAPES = [((128, 5, 3), 70_000, True),    # rows of 128, n2 odd: two points per lane
          ((128, 2, 3), 900, True),       # few atoms (8-atom groups): one point per lane
          ((256, 4, 1), 20_000, False),   # the same
          ((128, 2, 2), 70_000, True),    # 16-atom groups, 2 x 2 x 2 blocks; 1 of 4 waves busy
          ((256, 2, 3), 70_000, False),   # 2 x 2 blocks
          ((64, 4, 2), 70_000, True),     # rows of 64: 1 x 2 x 2 blocks
          ((64, 2, 3), 66_000, False),    # 1 x 2 blocks
          ((64, 5, 1), 777, False),       # 320 points: a partly filled last work-group
          ((64, 1, 1), 70_000, True),     # one row, many atoms: stream splits
          ((50, 7, 3), 2500, True),       # rows of 50: the point-list kernels
          ((1, 3, 200), 1200, False),     # one-point rows
          ((192, 2, 2), 1, True)]         # a single atom


@pytest.mark.parametrize("shape,n,cplx", SHAPES)
def test_fwd_grid_vs_oracle(shape, n, cplx):
    grid = oblique(*shape)
    xyz, f, _ = wl.random_problem(n, 1, seed=n + shape[0], extent=60.0, s_range=1.0, complex_f=cplx)
    print(f"case fwd grid {shape} N={n} complex={cplx}", flush=True)
    A = fwd(xyz, f, grid)
    ref = oracle.forward(xyz, f, grid.points())
    e = M.incoherent(A, ref, f, n)
    print(f"  pointwise/sqrt(sum|f|^2) = {e:.3e}", flush=True)
    assert e <= M.INC_TOL


@pytest.mark.parametrize("shape,n,cplx", SHAPES)
def test_bwd_grid_vs_oracle(shape, n, cplx):
    grid = oblique(*shape)
    xyz, f, _ = wl.random_problem(n, 1, seed=2 * n + shape[1], extent=60.0, s_range=1.0, complex_f=cplx)
    G = wl.random_seed_field(grid.size, seed=n + 5)
    print(f"case bwd grid {shape} N={n} complex={cplx}", flush=True)
    g = bwd(xyz, f, grid, G)
    en, em = M.t3(g, oracle.adjoint(xyz, f, grid.points(), G))
    print(f"  T3 norm={en:.3e} max={em:.3e}", flush=True)
    assert en <= M.T3_NORM_TOL and em <= M.T3_MAX_TOL


@pytest.mark.parametrize("inline", ["0", "1"])
@pytest.mark.parametrize("shape,n,cplx", [((128, 2, 3), 900, True), ((256, 4, 1), 20_000, False),
                                          ((64, 5, 1), 777, True), ((192, 2, 2), 1, False)])
def test_small_grid_forward_inline_and_packed(shape, n, cplx, inline, monkeypatch):
    """Few records (one point per lane): by default the forward forms each lane's FP64 grid
    point and the atom records while staging (no pack dispatch); NX_TUNE_INLINE=0 keeps the
    row kernel and its packed records.  Both against the oracle, and against each other to
    rounding (their phases round differently)."""
    grid = oblique(*shape)
    xyz, f, _ = wl.random_problem(n, 1, seed=3 * n + shape[0], extent=60.0, s_range=1.0, complex_f=cplx)
    print(f"case small grid fwd {shape} N={n} complex={cplx} inline={inline}", flush=True)
    monkeypatch.setenv("NX_TUNE_INLINE", inline)
    A = fwd(xyz, f, grid)
    monkeypatch.setenv("NX_TUNE_INLINE", "1" if inline == "0" else "0")
    B = fwd(xyz, f, grid)
    ref = oracle.forward(xyz, f, grid.points())
    e, eb = M.incoherent(A, ref, f, n), M.incoherent(A, B, f, n)
    print(f"  pointwise/sqrt(sum|f|^2) = {e:.3e}, against the other form {eb:.3e}", flush=True)
    assert e <= M.INC_TOL and eb <= 2 * M.INC_TOL


@pytest.mark.parametrize("cplx", [True, False])
def test_row_kernels_agree_with_point_list_kernels(cplx, monkeypatch):
    """The same grid through the row kernels and (NX_TUNE_GRID=1) through the point-list
    kernels with FP64 grid points: the phases round differently (i1 (e1.r) + row term
    against S.r), so the results agree to rounding, not bitwise."""
    grid = oblique(256, 3, 2)
    n = 5000
    xyz, f, _ = wl.random_problem(n, 1, seed=71, extent=50.0, s_range=1.0, complex_f=cplx)
    G = wl.random_seed_field(grid.size, seed=72)
    print(f"case rows vs point-list kernels complex={cplx}", flush=True)
    A_rows, g_rows = fwd(xyz, f, grid), bwd(xyz, f, grid, G)
    monkeypatch.setenv("NX_TUNE_GRID", "1")
    A_list, g_list = fwd(xyz, f, grid), bwd(xyz, f, grid, G)
    e = M.incoherent(A_rows, A_list, f, n)
    en, em = M.t3(g_rows, g_list)
    print(f"  fwd gap {e:.3e}, adjoint T3 norm={en:.3e} max={em:.3e}", flush=True)
    assert e <= M.INC_TOL and en <= M.T3_NORM_TOL and em <= M.T3_MAX_TOL


def test_chunked_launches(monkeypatch):
    """Small launch chunks: several forward and adjoint launches carry their state."""
    grid = oblique(128, 4, 2)
    n = 9000
    xyz, f, _ = wl.random_problem(n, 1, seed=73, extent=40.0, s_range=1.0)
    G = wl.random_seed_field(grid.size, seed=74)
    monkeypatch.setenv("NX_TUNE_LAUNCH_PAIRS", str(1 << 20))
    print("case grid chunked launches", flush=True)
    A = fwd(xyz, f, grid)
    g = bwd(xyz, f, grid, G)
    P = grid.points()
    assert M.incoherent(A, oracle.forward(xyz, f, P), f, n) <= M.INC_TOL
    en, em = M.t3(g, oracle.adjoint(xyz, f, P, G))
    assert en <= M.T3_NORM_TOL and em <= M.T3_MAX_TOL


def test_empty_and_degenerate():
    grid = oblique(64, 2, 1)
    xyz, f, _ = wl.random_problem(10, 1, seed=75)
    print("case grid empty calls", flush=True)
    # no atoms: A = 0
    A = api.scatter_fwd_grid(torch.zeros((0, 3), dtype=torch.float32, device=DEV), None, grid)
    torch.cuda.synchronize()
    assert A.shape == (128,) and bool((A == 0).all())
    # no points: zero gradient, written by the library
    empty = oblique(64, 0, 1)
    g = api.scatter_bwd_grid(dev(xyz), dev(f), empty, torch.zeros(0, dtype=torch.complex64, device=DEV))
    torch.cuda.synchronize()
    assert g.shape == (10, 3) and bool((g == 0).all())
    assert api.scatter_fwd_grid(dev(xyz), dev(f), empty).numel() == 0
    # a zero step: every point of a row is the same point
    flat = wl.RegularGrid((1.0, 2.0, 3.0), (0.0, 0.0, 0.0), (0.1, 0.0, 0.0), (0.0, 0.0, 0.0), 64, 3, 1)
    A = fwd(xyz, f, flat).reshape(3, 64)
    assert np.all(A == A[:, :1])
    assert M.incoherent(A.ravel(), oracle.forward(xyz, f, flat.points()), f, 10) <= M.INC_TOL


@pytest.mark.parametrize("n,cplx", [(2000, True), (1500, False)])
def test_fit_step_grid_one_call_equals_three(n, cplx):
    grid = oblique(128, 6, 2)
    xyz, f, _ = wl.random_problem(n, 1, seed=76 + n, extent=40.0, s_range=1.0, complex_f=cplx)
    I = dev((np.abs(oracle.forward(xyz, f, grid.points())) ** 2).astype(np.float32) * 1.1)
    x, fd = dev(xyz), dev(f)
    print(f"case fit step grid N={n} complex={cplx}", flush=True)
    L, A, g, G = api.fit_step_grid(x, fd, grid, I, return_seed=True)
    A3 = api.scatter_fwd_grid(x, fd, grid)
    L3, G3 = api.loss_grad(A3, I)
    g3 = api.scatter_bwd_grid(x, fd, grid, G3)
    torch.cuda.synchronize()
    assert torch.equal(A, A3) and torch.equal(G, G3) and torch.equal(g, g3)
    assert float(L) == float(L3)


@pytest.mark.parametrize("inline", ["0", "1"])
def test_tiles_beyond_the_fixed_point_range(inline, monkeypatch):
    """Every other block of 700 atoms 300,000 lattice units out (their tiles exceed the
    fixed-point range: 300,000 x |S|_1 > 2^19) and every other group of points with
    |S_x| near 30,000 (the adjoint's tiles beyond the range for atoms within 40 units):
    those tiles reduce with rint and still meet the tolerances; the forward with its atom
    records formed while staging (the tile's bound from its own records) and packed."""
    monkeypatch.setenv("NX_TUNE_INLINE", inline)
    n = 3000
    xyz, f, _ = wl.random_problem(n, 1, seed=77, extent=40.0, s_range=1.0)
    far = (np.arange(n) // 700) % 2 == 1
    xyz = xyz.copy()
    xyz[far, 0] += np.float32(300_000.0)
    grid = oblique(128, 4, 2, origin=(3.0, 0.0, 0.0))
    print(f"case grid forward, out-of-range atom tiles, inline={inline}", flush=True)
    A = fwd(xyz, f, grid)
    assert M.incoherent(A, oracle.forward(xyz, f, grid.points()), f, n) <= M.INC_TOL
    # points: the second half of the grid's rows far out along x
    n2 = 1000
    xa, fa, _ = wl.random_problem(n2, 1, seed=78, extent=40.0, s_range=1.0)
    gfar = wl.RegularGrid((30_000.0, 0.0, 0.0), (0.013, 0.004, 0.0), (-29_997.0, 0.011, 0.0),
                          (0.0, 0.0, 0.017), 64, 2, 3)
    G = wl.random_seed_field(gfar.size, seed=79)
    print("case grid adjoint, out-of-range point tiles", flush=True)
    g = bwd(xa, fa, gfar, G)
    en, em = M.t3(g, oracle.adjoint(xa, fa, gfar.points(), G))
    print(f"  T3 norm={en:.3e} max={em:.3e}", flush=True)
    assert en <= M.T3_NORM_TOL and em <= M.T3_MAX_TOL


def central_lines(n):
    c = n // 2
    idx = [h + n * c + n * n * c for h in range(n)] + [c + n * k + n * n * c for k in range(n)]
    idx += [c + n * c + n * n * l for l in range(n)]
    return np.unique(np.array(idx, dtype=np.int64))


def test_c2_grid_fit_step_at_full_size():
    """C2's fit step over its exact 128^3 grid (one call, the benchmark's configuration):
    sampled A against the oracle at the FP64 grid points (T1, T2), L against an FP64
    recomputation from the returned A, the adjoint against the oracle on 24 sampled atoms
    and against the all-FP64 GPU adjoint fed the same seed on 4,096."""
    w = wl.c2()
    grid = w.grid
    P = grid.points()
    tx, tf = dev(w.xyz), dev(w.f)
    I = (api.scatter_fwd_grid(dev(w.target_xyz), tf, grid).abs() ** 2).float()
    print(f"case c2 grid fit step: {w.n_atoms} atoms x {grid.size} points", flush=True)
    L, A, g, G = api.fit_step_grid(tx, tf, grid, I, return_seed=True)
    torch.cuda.synchronize()
    A_np = A.cpu().numpy()
    rng = np.random.default_rng(81)
    idx = np.unique(np.concatenate([rng.choice(grid.size, 256, replace=False), central_lines(128)]))
    ref = oracle.forward(w.xyz, w.f, P[idx])
    e1, e2 = M.t1(A_np[idx], ref), M.t2(A_np[idx], ref)
    print(f"  fwd sampled T1={e1:.3e} T2={e2:.3e}", flush=True)
    assert e1 <= M.T1_TOL and e2 <= M.T2_TOL
    Ad = A_np.astype(np.complex128)
    e = np.abs(Ad) ** 2 - I.cpu().numpy().astype(np.float64)
    assert abs(float(L.cpu()) - np.sum(e * e)) <= 1e-12 * np.sum(e * e)
    G_np = G.cpu().numpy()
    g_np = g.cpu().numpy()
    atoms = np.sort(rng.choice(w.n_atoms, size=24, replace=False))
    en, em = M.t3(g_np[atoms], oracle.adjoint(w.xyz[atoms], w.f[atoms], P, G_np))
    print(f"  adjoint vs oracle (24 atoms): T3 norm={en:.3e} max={em:.3e}", flush=True)
    assert en <= M.T3_NORM_TOL and em <= M.T3_MAX_TOL
    atoms = np.sort(rng.choice(w.n_atoms, size=4096, replace=False))
    g64 = api.scatter_bwd_f64(dev(w.xyz[atoms].astype(np.float64)), dev(w.f[atoms].astype(np.complex128)),
                              dev(P), G.to(torch.complex128)).cpu().numpy()
    en, em = M.t3(g_np[atoms], g64)
    print(f"  adjoint vs all-FP64 path (4096 atoms): T3 norm={en:.3e} max={em:.3e}", flush=True)
    assert en <= M.T3_NORM_TOL and em <= M.T3_MAX_TOL


@pytest.mark.parametrize("step,n1,n2,atoms", [(0.0005, 128, 4, 24), (0.004, 128, 3, 24), (0.004, 128, 4, 24),
                                               (0.02, 256, 2, 24), (0.004, 128, 4, 44)])
def test_lattice_maps_pointwise(step, n1, n2, atoms, monkeypatch):
    """Perfect simple-cubic lattices (every atom of a plane shares step1.r, step2.r and
    step3.r), the case where a systematic rounding of the steps would add up coherently: T1
    against the oracle at the FP64 grid points with the stepped blocks (16-atom groups:
    2 x 2 x 2 for n2 even, two points per lane for n2 odd) and with one point per lane
    (NX_TUNE_P=1), over fine and coarse maps through (0, 0, 4)."""
    xyz = wl.cubic_sites(atoms, atoms, atoms).astype(np.float32)
    n = xyz.shape[0]
    grid = wl.RegularGrid((-0.5 * step * n1, 0.013, 3.98), (step, 0.0, 0.0), (0.0, 0.004, 0.0),
                          (0.0, 0.0, 0.01), n1, n2, 2)
    print(f"case lattice map: {n} atoms, step {step}, {n1} x {n2} x 2", flush=True)
    ref = oracle.forward(xyz, None, grid.points())
    monkeypatch.setenv("NX_TUNE_GRP", "16")       # (few atoms would take 8-atom groups)
    A2 = fwd(xyz, None, grid)
    monkeypatch.setenv("NX_TUNE_P", "1")
    A1 = fwd(xyz, None, grid)
    e2, e1 = M.t1(A2, ref), M.t1(A1, ref)
    print(f"  T1 stepped {e2:.3e}, one point per lane {e1:.3e}", flush=True)
    assert e2 <= M.T1_TOL and e1 <= M.T1_TOL


@pytest.mark.parametrize("cplx", [True, False])
def test_autograd_over_a_grid(cplx):
    """scatter_grid under torch autograd: L = sum (|A|^2 - I)^2 computed in torch, its
    gradient with respect to the positions through the grid adjoint, against the oracle's
    adjoint fed the oracle's own seed (T3), and against the one-call fit step."""
    grid = oblique(128, 2, 2)
    n = 3000
    xyz, f, _ = wl.random_problem(n, 1, seed=91, extent=30.0, s_range=1.0, complex_f=cplx)
    P = grid.points()
    I = (np.abs(oracle.forward(xyz, f, P)) ** 2 * 1.05).astype(np.float32)
    x = dev(xyz).requires_grad_(True)
    print(f"case autograd over a grid complex={cplx}", flush=True)
    A = api.scatter_grid(x, dev(f), grid)
    L = ((A.abs() ** 2 - dev(I)) ** 2).sum()
    L.backward()
    g = x.grad.cpu().numpy().astype(np.float64)
    _, G_ref = oracle.loss(oracle.forward(xyz, f, P), I)
    en, em = M.t3(g, oracle.adjoint(xyz, f, P, G_ref))
    print(f"  T3 norm={en:.3e} max={em:.3e}", flush=True)
    assert en <= M.T3_NORM_TOL and em <= M.T3_MAX_TOL
    _, _, g_step = api.fit_step_grid(dev(xyz), dev(f), grid, dev(I))
    torch.cuda.synchronize()
    en2, _ = M.t3(g, g_step.cpu().numpy())
    assert en2 <= M.T3_NORM_TOL


def test_c2_grid_every_point_against_the_f64_path():
    """C2's forward over its exact 128^3 grid against the all-FP64 GPU path at the same FP64
    points, on every one of the 2,097,152 points (the all-FP64 path is held to the oracle on
    its own samples): T1 and T2 over the whole map, the margin printed."""
    w = wl.c2()
    grid = w.grid
    print(f"case c2 grid every point vs f64: {w.n_atoms} atoms x {grid.size} points", flush=True)
    A = fwd(w.xyz, w.f, grid)
    A64 = api.scatter_fwd_f64(dev(w.xyz.astype(np.float64)), dev(w.f.astype(np.complex128)),
                              dev(grid.points()))
    torch.cuda.synchronize()
    A64 = A64.cpu().numpy()
    e1, e2 = M.t1(A, A64), M.t2(A, A64)
    print(f"  every point: T1={e1:.3e} (margin {M.T1_TOL / e1:.1f}x) T2={e2:.3e}", flush=True)
    assert e1 <= M.T1_TOL and e2 <= M.T2_TOL
