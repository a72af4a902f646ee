"""Eq. 4 (block form) and Eq. 5 (FFT approximation) on the GPU: the block form through
the species kernels against the oracle, its exactness for rigid blocks, the FFT form
against its definition, and the accuracy comparison with the atom-by-atom sum."""
import numpy as np
import pytest
import torch

import oracle
from paper_1010_2641_amd import api, approx, workloads as wl
from tests import metrics as M

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def cells(n, amp, seed):
    r = np.arange(n, dtype=np.float64)
    X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
    r0 = np.stack([X, Y, Z], -1)
    return r0, amp * np.random.default_rng(seed).normal(size=r0.shape)


def test_block_form_against_oracle_and_rigid_blocks():
    r0, u = cells(14, 0.03, 81)
    blocks = wl._f32((r0 + u).reshape(-1, 3))
    H = (2.0, 2.0, 0.0)
    Sg = approx.fft_grid((14, 14, 14), 2, H)
    S = wl._f32(Sg[np.random.default_rng(82).choice(len(Sg), 3000, replace=False)])
    tS = dev(S)
    A = approx.block_form(dev(blocks), wl.FCC_BASIS, tS).cpu().numpy().astype(np.complex128)
    F = oracle.forward(wl.FCC_BASIS, None, S)
    A_ref, _ = oracle.forward_species(blocks, [0, len(blocks)], F[None, :], S)
    e1, e2 = M.t1(A, A_ref), M.t2(A, A_ref)
    print(f"block form vs oracle: T1={e1:.3e} T2={e2:.3e}", flush=True)
    assert e1 <= M.T1_TOL and e2 <= M.T2_TOL
    # rigid blocks: the atom-by-atom GPU sum over the same atoms agrees
    atoms = wl._f32((blocks.astype(np.float64)[:, None, :] + wl.FCC_BASIS[None]).reshape(-1, 3))
    A_at = api.scatter_fwd(dev(atoms), None, tS).cpu().numpy().astype(np.complex128)
    assert M.t2(A, A_at) <= 2 * M.T2_TOL


def test_fft_form_against_definition_on_gpu():
    r0, u = cells(11, 0.05, 83)
    H = (2.0, 0.0, 2.0)
    FT = approx.fft_approximation(dev(u), H, 3).cpu().numpy()
    Sg = approx.fft_grid((11, 11, 11), 3, H)
    idx = np.random.default_rng(84).choice(len(Sg), 200, replace=False)
    f = np.exp(2j * np.pi * (u.reshape(-1, 3) @ np.asarray(H)))
    ref = oracle.forward(r0.reshape(-1, 3), f, Sg[idx] - np.asarray(H))
    assert np.max(np.abs(FT[idx] - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_accuracy_comparison_small():
    """The comparison report at a small size: the FP64-phase direct sum and the species
    kernel's block form stay at their rounding level (their inputs are the FP32-rounded
    positions and points: ~1e-6 of a cycle at |S| ~ 3 and |r| ~ 12), and the FFT form's
    own error (Eq. 5 against the exact block form) grows with the Eq. 7 quantity."""
    text, res = approx.compare(cells=12, pad=3, window=0.25)
    print(text, flush=True)
    assert res["t2"]["FP64-phase sum vs exact"] <= 2e-5
    assert res["t2"]["Eq. 4 (species kernel) vs Eq. 4"] <= 2e-5
    eq5 = [b[3][3] for b in res["bins"]]
    assert len(eq5) >= 3 and eq5[-1] > 3 * eq5[0]
    assert res["t2"]["Eq. 4 vs exact"] < 0.05 and res["t2"]["Eq. 5 vs exact"] < 0.2


def test_eq7_bound_on_gpu():
    """|A_Eq4 - A_Eq5| <= |F| sum_j |exp(2 i pi q.u_j) - 1| at every point (all-FP64 GPU
    sums for Eq. 4, the FFT for Eq. 5)."""
    r0, u = cells(9, 0.04, 85)
    H = np.array([2.0, 2.0, 0.0])
    Sg = approx.fft_grid((9, 9, 9), 2, H)
    tS = dev(Sg)
    F = api.scatter_fwd_f64(dev(wl.FCC_BASIS), None, tS).cpu().numpy()
    Ab = F * api.scatter_fwd_f64(dev((r0 + u).reshape(-1, 3)), None, tS).cpu().numpy()
    Af = F * approx.fft_approximation(dev(u), H, 2).cpu().numpy()
    q = Sg - H[None, :]
    bound = np.abs(F) * np.sum(np.abs(np.exp(2j * np.pi * (q @ u.reshape(-1, 3).T)) - 1), axis=1)
    assert np.all(np.abs(Ab - Af) <= bound * (1 + 1e-9) + 1e-9)
