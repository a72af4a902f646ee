"""The largest counts the library accepts (NX_MAX_COUNT = 2^30 atoms or points) on the
GPU: 32-bit work-item and block arithmetic, multi-gigabyte workspaces and the forward's
L2-sized launch chunks at their extreme.  Inputs are built on the GPU from indices, so
their values are known exactly on the host: a 1024^3 simple-cubic block (its amplitude
is a product of three geometric series) and dyadic point coordinates."""
import numpy as np
import pytest
import torch

import oracle
from paper_1010_2641_amd import _lib, api
from tests import metrics as M

pytestmark = pytest.mark.gpu

MAX = _lib.NX_MAX_COUNT
SIDE = 1024                                   # 1024^3 = 2^30 atoms


def cube_sites_gpu():
    i = torch.arange(MAX, dtype=torch.int64, device="cuda")
    xyz = torch.stack([(i >> 20).float(), ((i >> 10) & 1023).float(), (i & 1023).float()], dim=1)
    del i
    return xyz.contiguous()


def cube_sites_host(idx):
    idx = np.asarray(idx, dtype=np.int64)
    return np.stack([idx >> 20, (idx >> 10) & 1023, idx & 1023], axis=1).astype(np.float64)


def geometric(s, n):
    """sum_{m<n} exp(2 i pi s m), s reduced mod 1 (FP64)."""
    t = np.asarray(s, dtype=np.float64)
    t = t - np.rint(t)
    out = np.full(t.shape, complex(n))
    nz = np.abs(t) > 1e-15
    out[nz] = (1 - np.exp(2j * np.pi * t[nz] * n)) / (1 - np.exp(2j * np.pi * t[nz]))
    return out


@pytest.fixture(scope="module")
def cube():
    assert SIDE ** 3 == MAX
    xyz = cube_sites_gpu()
    yield xyz
    del xyz
    torch.cuda.empty_cache()


def test_forward_max_atoms_against_closed_form(cube):
    """2^30 atoms x 64 points near (1, 1, 1): the forward against the Laue product."""
    d = (np.arange(8) - 3.5) / 4096.0
    S = np.stack(np.meshgrid(1 + d, 1 + d[::2], [1.0, 1 + 1 / 2048.0], indexing="ij"), -1).reshape(-1, 3)
    S = S.astype(np.float32)
    print(f"case max atoms: {MAX} atoms x {len(S)} points", flush=True)
    A = api.scatter_fwd(cube, None, torch.from_numpy(S).cuda()).cpu().numpy().astype(np.complex128)
    S64 = S.astype(np.float64)
    ref = geometric(S64[:, 0], SIDE) * geometric(S64[:, 1], SIDE) * geometric(S64[:, 2], SIDE)
    e2 = M.t2(A, ref)
    e1 = M.t1(A, ref, floor=1e-4)
    print(f"max atoms: T1(1e-4)={e1:.3e} T2={e2:.3e}", flush=True)
    assert e2 <= M.T2_TOL and e1 <= M.T1_TOL


def test_adjoint_max_atoms_sampled(cube):
    """The adjoint over 2^30 atoms (two million work-groups), sampled atoms against the
    oracle, with a random seed on 64 points."""
    rng = np.random.default_rng(91)
    S = (1 + rng.uniform(-0.01, 0.01, size=(64, 3))).astype(np.float32)
    G = (rng.normal(size=64) + 1j * rng.normal(size=64)).astype(np.complex64)
    g = api.scatter_bwd(cube, None, torch.from_numpy(S).cuda(), torch.from_numpy(G).cuda())
    idx = np.unique(np.concatenate([[0, 1, MAX // 2, MAX - 2, MAX - 1],
                                    rng.integers(0, MAX, size=2043)]))
    g_s = g[torch.from_numpy(idx).cuda()].cpu().numpy()
    del g
    g_ref = oracle.adjoint(cube_sites_host(idx), None, S, G)
    en, em = M.t3(g_s, g_ref)
    print(f"max atoms adjoint sampled: T3 norm={en:.3e} max={em:.3e}", flush=True)
    assert en <= M.T3_NORM_TOL and em <= M.T3_MAX_TOL


def test_forward_max_points_sampled():
    """2^30 points (dyadic coordinates) x 3 atoms: sampled amplitudes against the oracle."""
    xyz = np.array([[0.25, 1.5, -3.0], [7.0, 0.125, 2.5], [-1.75, 4.0, 0.5]], dtype=np.float32)
    k = torch.arange(MAX, dtype=torch.int64, device="cuda")
    S = torch.stack([((k & 1023).float() / 256.0), (((k >> 10) & 1023).float() / 512.0),
                     ((k >> 20).float() / 1024.0)], dim=1).contiguous()
    del k
    print(f"case max points: 3 atoms x {MAX} points", flush=True)
    A = api.scatter_fwd(torch.from_numpy(xyz).cuda(), None, S)
    del S
    rng = np.random.default_rng(92)
    idx = np.unique(np.concatenate([[0, 1, MAX - 1], rng.integers(0, MAX, size=4093)]))
    A_s = A[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.complex128)
    del A
    torch.cuda.empty_cache()
    S_h = np.stack([(idx & 1023) / 256.0, ((idx >> 10) & 1023) / 512.0, (idx >> 20) / 1024.0], axis=1)
    A_ref = oracle.forward(xyz, None, S_h)
    err = float(np.max(np.abs(A_s - A_ref)))
    print(f"max points sampled: max |dA| = {err:.3e}", flush=True)
    assert err <= 3 * M.INC_TOL * np.sqrt(3)


def max_grid():
    """1024^3 = 2^30 points with dyadic steps around (0, 0, 4): the grid kernels' 32-bit
    index arithmetic, row and plane decomposition and 2 x 2 x 2 blocks at the largest
    count."""
    from paper_1010_2641_amd import workloads as wl
    h = 1.0 / 1024.0
    return wl.RegularGrid((-0.5, -0.5, 3.5), (h, 0.0, 0.0), (0.0, h, 0.0), (0.0, 0.0, h), 1024, 1024, 1024)


def test_grid_forward_max_points_sampled(monkeypatch):
    """The grid forward over 2^30 points (64 atoms, 16-atom groups forced so that the
    2 x 2 x 2 blocks run): sampled amplitudes, the corners included, against the oracle."""
    from paper_1010_2641_amd import workloads as wl
    grid = max_grid()
    assert grid.size == MAX
    xyz, f, _ = wl.random_problem(64, 1, seed=93, extent=20.0, s_range=1.0)
    monkeypatch.setenv("NX_TUNE_GRP", "16")
    print(f"case grid max points: 64 atoms x {MAX} points", flush=True)
    A = api.scatter_fwd_grid(torch.from_numpy(xyz).cuda(), torch.from_numpy(f).cuda(), grid)
    rng = np.random.default_rng(94)
    idx = np.unique(np.concatenate([[0, 1, 1023, 1024, MAX // 2, MAX - 1025, MAX - 2, MAX - 1],
                                    rng.integers(0, MAX, size=4088)]))
    A_s = A[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.complex128)
    del A
    torch.cuda.empty_cache()
    e = M.incoherent(A_s, oracle.forward(xyz, f, grid.points(idx)), f, 64)
    print(f"grid max points sampled: pointwise/sqrt(sum|f|^2) = {e:.3e}", flush=True)
    assert e <= M.INC_TOL


def test_grid_adjoint_max_points_sampled():
    """The grid adjoint over 2^30 points (256 atoms, the stepped 64-point runs): the seed is
    zero except at 4,096 seeded points, whose contributions the oracle sums."""
    from paper_1010_2641_amd import workloads as wl
    grid = max_grid()
    xyz, f, _ = wl.random_problem(256, 1, seed=95, extent=20.0, s_range=1.0)
    rng = np.random.default_rng(96)
    idx = np.unique(np.concatenate([[0, 63, 64, MAX - 64, MAX - 1], rng.integers(0, MAX, size=4091)]))
    Gs = (rng.normal(size=len(idx)) + 1j * rng.normal(size=len(idx))).astype(np.complex64)
    G = torch.zeros(MAX, dtype=torch.complex64, device="cuda")
    G[torch.from_numpy(idx).cuda()] = torch.from_numpy(Gs).cuda()
    print(f"case grid max points adjoint: 256 atoms x {MAX} points", flush=True)
    g = api.scatter_bwd_grid(torch.from_numpy(xyz).cuda(), torch.from_numpy(f).cuda(), grid, G)
    del G
    g_np = g.cpu().numpy().astype(np.float64)
    del g
    torch.cuda.empty_cache()
    en, em = M.t3(g_np, oracle.adjoint(xyz, f, grid.points(idx), Gs))
    print(f"grid max points adjoint: T3 norm={en:.3e} max={em:.3e}", flush=True)
    assert en <= M.T3_NORM_TOL and em <= M.T3_MAX_TOL


def test_counts_above_the_maximum_are_rejected():
    x = torch.zeros((4, 3), dtype=torch.float32, device="cuda")
    assert _lib.nx_scatter_fwd(x.data_ptr(), None, MAX + 1, x.data_ptr(), 4, x.data_ptr(), 1, None, 0,
                               None) == _lib.NX_ERR_ARG
    assert "NX_MAX_COUNT" in _lib.last_error()
