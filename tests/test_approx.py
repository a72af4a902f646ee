"""The comparison forms of Eq. 4 and Eq. 5 on the CPU: the FFT evaluation of Eq. 5's
transform equals its definition (a direct sum, by the oracle), and the block form of
Eq. 4 equals the atom-by-atom sum exactly when every atom of a block shares the block's
displacement; the gap between the block form and the FFT form obeys the bound that
follows from dropping exp(2 i pi q.u) (the condition of Eq. 7)."""
import numpy as np
import torch

import oracle
from paper_1010_2641_amd import approx, workloads as wl


def lattice(n, amp, seed):
    r = np.arange(n, dtype=np.float64)
    X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
    r0 = np.stack([X, Y, Z], -1)
    u = amp * np.random.default_rng(seed).normal(size=r0.shape)
    return r0, u


def test_fft_transform_equals_its_definition():
    r0, u = lattice(7, 0.05, 0)
    H = (2.0, 2.0, 0.0)
    for origin in ((0.0, 0.0, 0.0), (1.0, -3.0, 2.0)):
        FT = approx.fft_approximation(torch.from_numpy(u), H, 3, origin=origin).numpy()
        Sg = approx.fft_grid((7, 7, 7), 3, H)
        idx = np.random.default_rng(1).choice(len(Sg), 60, replace=False)
        q = Sg[idx] - np.asarray(H)
        f = np.exp(2j * np.pi * (u.reshape(-1, 3) @ np.asarray(H)))
        ref = oracle.forward(r0.reshape(-1, 3) + np.asarray(origin), f, q)
        assert np.max(np.abs(FT[idx] - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_block_form_identity_and_eq7_bound():
    r0, u = lattice(5, 0.04, 2)
    H = np.array([2.0, 2.0, 0.0])
    Sg = approx.fft_grid((5, 5, 5), 2, H)
    S = Sg[np.random.default_rng(3).choice(len(Sg), 40, replace=False)]
    blocks = (r0 + u).reshape(-1, 3)
    # every atom of a cell carries the cell's displacement: Eq. 4 is then exact
    atoms = (blocks[:, None, :] + wl.FCC_BASIS[None, :, :]).reshape(-1, 3)
    F = oracle.forward(wl.FCC_BASIS, None, S)
    A_atoms = oracle.forward(atoms, None, S)
    A_block, _ = oracle.forward_species(blocks, [0, len(blocks)], F[None, :], S)
    assert np.max(np.abs(A_block - A_atoms)) <= 1e-12 * np.max(np.abs(A_atoms))
    # Eq. 5 drops exp(2 i pi q.u_j): |A_block - F FT| <= |F| sum_j |exp(2 i pi q.u_j) - 1|
    FT_all = approx.fft_approximation(torch.from_numpy(u), H, 2).numpy()
    key = {tuple(np.round(s, 9)): i for i, s in enumerate(Sg)}
    FT = FT_all[[key[tuple(np.round(s, 9))] for s in S]]
    q = S - H[None, :]
    bound = np.abs(F) * np.sum(np.abs(np.exp(2j * np.pi * (q @ u.reshape(-1, 3).T)) - 1), axis=1)
    gap = np.abs(A_block - F * FT)
    assert np.all(gap <= bound * (1 + 1e-9) + 1e-12)
    assert np.max(gap / bound) > 0.01          # the bound is not vacuous
