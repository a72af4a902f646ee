"""Unstructured reciprocal-space points: an area detector's pixels projected on Ewald's
sphere during a rocking scan (curved sheets, no grid), and the invariance of the GPU
sums under any reordering of the points (the kernels exploit no grid structure)."""
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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_ewald_scan_forward_against_oracle_and_f64_path():
    w = wl.ewald(n_pix=64, n_frames=16)
    print(f"case ewald: {w.n_atoms} atoms x {w.n_points} detector points", flush=True)
    A = host(api.scatter_fwd(dev(w.xyz), dev(w.f), dev(w.S))).astype(np.complex128)
    A64 = host(api.scatter_fwd_f64(dev(w.xyz.astype(np.float64)), dev(w.f.astype(np.complex128)),
                                   dev(w.S.astype(np.float64))))
    rng = np.random.default_rng(61)
    strongest = np.argsort(-np.abs(A64))[:64]
    idx = np.unique(np.concatenate([rng.choice(w.n_points, 448, replace=False), strongest]))
    A_ref = oracle.forward(w.xyz, w.f, w.S[idx])
    e1, e2 = M.t1(A[idx], A_ref), M.t2(A[idx], A_ref)
    print(f"ewald sampled: T1={e1:.3e} T2={e2:.3e}", flush=True)
    assert e1 <= M.T1_TOL and e2 <= M.T2_TOL
    f1, f2 = M.t1(A64[idx], A_ref), M.t2(A64[idx], A_ref)
    assert f1 <= M.F64_T1_TOL and f2 <= M.F64_T2_TOL
    g1, g2 = M.t1(A, A64), M.t2(A, A64)
    print(f"ewald every point vs f64 path: T1={g1:.3e} T2={g2:.3e}", flush=True)
    assert g1 <= M.T1_TOL and g2 <= M.T2_TOL


def test_ewald_fit_step_as_benchmarked():
    """The benchmark's ewald step: forward, misfit against the strain x1.1 target and
    adjoint on 2,097,152 detector points; the adjoint against the all-FP64 adjoint fed the
    same seed on sampled atoms, and sampled amplitudes against the oracle."""
    w = wl.ewald()
    tx, tf, tS = dev(w.xyz), dev(w.f), dev(w.S)
    I = (api.scatter_fwd(dev(w.target_xyz), tf, tS).abs() ** 2).float()
    L, A, g = api.fit_step(tx, tf, tS, I)
    A_np = host(A)
    rng = np.random.default_rng(62)
    idx = np.unique(np.concatenate([rng.choice(w.n_points, 192, replace=False),
                                    np.argsort(-np.abs(A_np))[:64]]))
    A_ref = oracle.forward(w.xyz, w.f, w.S[idx])
    e1, e2 = M.t1(A_np[idx], A_ref), M.t2(A_np[idx], A_ref)
    print(f"ewald fit-step sampled: T1={e1:.3e} T2={e2:.3e}", flush=True)
    assert e1 <= M.T1_TOL and e2 <= M.T2_TOL
    _, G = api.loss_grad(A, I)
    atoms = np.sort(rng.choice(w.n_atoms, size=2048, replace=False))
    g64 = api.scatter_bwd_f64(dev(w.xyz[atoms].astype(np.float64)),
                              dev(w.f[atoms].astype(np.complex128)), tS.double(),
                              G.to(torch.complex128))
    en, em = M.t3(host(g)[atoms], host(g64))
    print(f"ewald fit-step adjoint vs f64 path: T3 norm={en:.3e} max={em:.3e}", flush=True)
    assert en <= M.T3_NORM_TOL and em <= M.T3_MAX_TOL


@pytest.mark.parametrize("mode", ["ph64", "f32"])
def test_point_order_is_irrelevant(mode):
    """Permuting the points permutes the forward bitwise (every point is computed
    independently of the others) and leaves the adjoint unchanged up to the order of
    its sums over points."""
    w = wl.ewald(n_pix=32, n_frames=8)
    xyz, f = w.xyz[:20000], w.f[:20000]
    rng = np.random.default_rng(63)
    perm = rng.permutation(w.n_points)
    A = host(api.scatter_fwd(dev(xyz), dev(f), dev(w.S), mode))
    Ap = host(api.scatter_fwd(dev(xyz), dev(f), dev(w.S[perm]), mode))
    assert np.array_equal(Ap, A[perm])
    G = wl.random_seed_field(w.n_points, seed=64)
    g = host(api.scatter_bwd(dev(xyz), dev(f), dev(w.S), dev(G), mode))
    gp = host(api.scatter_bwd(dev(xyz), dev(f), dev(w.S[perm]), dev(G[perm]), mode))
    en, em = M.t3(gp, g)
    assert en <= (2e-6 if mode == "ph64" else 2e-4)


def test_random_points_wide_range_against_oracle():
    """Fig. 1's input kind: random atoms and random points over a wide S range."""
    xyz, _, S = wl.random_problem(6000, 7001, seed=65, extent=100.0, s_range=4.0, complex_f=False)
    A = host(api.scatter_fwd(dev(xyz), None, dev(S))).astype(np.complex128)
    e = M.incoherent(A, oracle.forward(xyz, None, S), None, len(xyz))
    print(f"random wide: pointwise/sqrt(N)={e:.3e}", flush=True)
    assert e <= M.INC_TOL
