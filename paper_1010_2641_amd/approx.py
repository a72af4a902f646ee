"""The paper's two alternatives to the atom-by-atom sum, built for an accuracy
comparison against it (Section 1):

* the block form (Eq. 4): A(S) = sum_j F_j(S) exp(2 i pi S.(r0_j + u_j)) over blocks of
  atoms (here unit cells) with structure factor F_j(S) and one displacement u_j per block.
  With identical blocks F_j = F it is the species-factorised sum with one species, so it
  runs in libnx's species kernels; F(S) itself is the direct sum over the block's basis;
* the FFT approximation (Eq. 5): A(H + q) ~ F(H + q) FT[exp(2 i pi H.u_j)](q) on the
  triperiodic grid of block origins, valid while |q.u| << 1 (Eq. 7).  It is evaluated
  with torch.fft (complex128) on the GPU, zero-padded `pad` times per axis so that q is
  sampled every 1/(n pad) r.l.u.

Neither is a product path: the block form drops the displacement differences inside a
block and the FFT form drops exp(2 i pi q.u) - 1; `compare` measures both against the
direct sum over every atom.

    python -m paper_1010_2641_amd.approx [--cells 29] [--pad 4] [--window 0.2] [--out FILE]
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np
import torch

from . import api, workloads as wl


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t if dtype is None else t.to(dtype)


def cell_structure_factor(basis, S, f_basis=None, mode="ph64"):
    """F(S) = sum_b f_b exp(2 i pi S.b) over the atoms b of one block (GPU direct sum);
    basis (B, 3), S (K, 3) torch float32 on the GPU -> (K,) complex64."""
    b = torch.as_tensor(np.asarray(basis, dtype=np.float32)).cuda()
    f = None if f_basis is None else torch.as_tensor(np.asarray(f_basis, dtype=np.complex64)).cuda()
    return api.scatter_fwd(b, f, S, mode)


def block_form(block_xyz, basis, S, f_basis=None, mode="ph64"):
    """Eq. 4 with identical blocks at positions block_xyz = r0_j + u_j (torch (M, 3)
    float32): the per-point factor F(S) is the structure factor of the basis, and the
    sum over blocks runs as a one-species factorised sum.  Returns (K,) complex64."""
    F = cell_structure_factor(basis, S, f_basis, mode)
    return api.scatter_fwd_species(block_xyz, [0, block_xyz.shape[0]], F[None, :].contiguous(), S, mode)


def fft_grid(shape, pad, H):
    """The points S = H + q of the padded FFT, q_a = i_a / (n_a pad) for i_a in
    [-n_a pad / 2, n_a pad / 2), listed with the last axis fastest (float64 (K, 3))."""
    axes = [np.fft.fftshift(np.fft.fftfreq(n * pad)) for n in shape]
    Q = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    return Q + np.asarray(H, dtype=np.float64)[None, :]


def fft_approximation(u_cells, H, pad, origin=(0.0, 0.0, 0.0)):
    """FT[exp(2 i pi H.u_j)](q) of Eq. 5 for blocks at origin + (i, j, k), i < n_a, with
    displacements u_cells (n1, n2, n3, 3) (torch float64 on the GPU), on the padded grid
    of `fft_grid`: sum_j exp(2 i pi H.u_j) exp(2 i pi q.r0_j), complex128, flattened in
    the grid's order.  (The structure factor F(S) multiplies this outside.)"""
    n = tuple(u_cells.shape[:3])
    Hd = torch.tensor(np.asarray(H, dtype=np.float64), device=u_cells.device)
    field = torch.exp(2j * np.pi * (u_cells @ Hd))
    m = tuple(a * pad for a in n)
    # e^{+2 i pi q.r}: the inverse DFT times the grid size, centred with fftshift
    A = torch.fft.ifftn(field, s=m) * float(np.prod(m))
    A = torch.fft.fftshift(A)
    q = fft_grid(n, pad, (0.0, 0.0, 0.0))
    ramp = np.exp(2j * np.pi * (q @ np.asarray(origin, dtype=np.float64)))
    return A.reshape(-1) * torch.from_numpy(ramp).to(A.device)


def _timed(fn):
    """fn's result and the wall time of a second call (the first one pays for
    allocations and, for the FFT, the plan)."""
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def compare(cells=29, pad=4, window=0.2, amp=0.03, wavelength=20.0, H=(2.0, 2.0, 0.0),
            floor=1e-4):
    """Atom-by-atom sum vs block form vs FFT approximation for an fcc cube of
    cells^3 unit cells with the displacement field u = amp sin(2 pi (z, x, y)/wavelength)
    evaluated at each atom (exact sum) or at each cell origin (block and FFT forms), on
    the FFT grid points within `window` r.l.u. of H.  Returns (markdown text, dict)."""
    rng_cells = np.arange(cells, dtype=np.float64)
    X, Y, Z = np.meshgrid(rng_cells, rng_cells, rng_cells, indexing="ij")
    r0 = np.stack([X, Y, Z], axis=-1)                                   # (n, n, n, 3)
    w = 2 * np.pi / wavelength

    def field(p):
        return amp * np.stack([np.sin(w * p[..., 2]), np.sin(w * p[..., 0]), np.sin(w * p[..., 1])], -1)

    u_cell = field(r0)
    atoms0 = (r0.reshape(-1, 1, 3) + wl.FCC_BASIS[None, :, :]).reshape(-1, 3)
    atoms64 = atoms0 + field(atoms0)
    blocks64 = r0.reshape(-1, 3) + u_cell.reshape(-1, 3)
    Sg = fft_grid((cells,) * 3, pad, H)
    sel = np.all(np.abs(Sg - np.asarray(H)) <= window + 1e-12, axis=1)
    S64 = Sg[sel]
    tS, tS64 = _dev(wl._f32(S64)), _dev(S64)
    basis64 = _dev(wl.FCC_BASIS)
    res = {}
    # the exact sum and the exact block form, both on the all-FP64 path
    A_exact, res["t_exact_f64"] = _timed(lambda: api.scatter_fwd_f64(_dev(atoms64), None, tS64))
    A_b64 = api.scatter_fwd_f64(basis64, None, tS64) * api.scatter_fwd_f64(_dev(blocks64), None, tS64)
    # the FP32 forms the library runs
    A_ph, res["t_atoms_ph64"] = _timed(lambda: api.scatter_fwd(_dev(wl._f32(atoms64)), None, tS))
    A_blk, res["t_block_ph64"] = _timed(lambda: block_form(_dev(wl._f32(blocks64)), wl.FCC_BASIS, tS))

    def fft_form():
        FT = fft_approximation(_dev(u_cell), H, pad)
        F = api.scatter_fwd_f64(basis64, None, _dev(Sg))
        return F * FT

    A_fft_all, res["t_fft"] = _timed(fft_form)
    A_fft = A_fft_all[torch.from_numpy(np.nonzero(sel)[0]).cuda()]
    ex = A_exact.cpu().numpy()
    b64 = A_b64.cpu().numpy()
    cols = {"FP64-phase sum vs exact": (A_ph.cpu().numpy().astype(np.complex128), ex),
            "Eq. 4 vs exact": (b64, ex),
            "Eq. 4 (species kernel) vs Eq. 4": (A_blk.cpu().numpy().astype(np.complex128), b64),
            "Eq. 5 vs Eq. 4": (A_fft.cpu().numpy(), b64),
            "Eq. 5 vs exact": (A_fft.cpu().numpy(), ex)}
    # Eq. 7's quantity, bounded per point by sum_a |q_a| max_j |u_j,a|
    q = S64 - np.asarray(H)[None, :]
    qu = np.abs(q) @ np.abs(u_cell.reshape(-1, 3)).max(axis=0)
    Ir = np.abs(ex) ** 2
    strong = Ir >= floor * Ir.max()
    bins = [0.0, 0.002, 0.004, 0.006, 0.008, 0.012, 0.016, np.inf]
    lines = ["## Eq. 4 block form and Eq. 5 FFT approximation against the atom-by-atom sum", "",
             f"fcc cube of {cells}^3 cells ({atoms64.shape[0]} atoms, {blocks64.shape[0]} blocks "
             f"= unit cells), u = {amp} sin(2 pi (z, x, y)/{wavelength:g}); points: the FFT grid "
             f"(padding x{pad}, q step {1 / (cells * pad):.4f} r.l.u.) within {window} r.l.u. of "
             f"H = {tuple(H)}, {S64.shape[0]} points.", "",
             "- exact: the all-FP64 direct sum over every atom (FP64 positions and points);",
             "- Eq. 4: every cell displaced rigidly by u at its origin, with the fcc structure "
             "factor F(S) (all-FP64 path; the species-kernel column runs it in the FP32 product "
             "path on FP32 inputs);",
             "- Eq. 5: F(S) times the zero-padded FFT of exp(2 i pi H.u) over the cell grid "
             "(torch.fft, complex128).", "",
             f"Entries: max over the points of a bin with I >= {floor:g} max I of "
             "|A - A_ref| / |A_ref|.  Bins: sum_a |q_a| max_j |u_j,a| (an upper bound of Eq. 7's "
             "max_j |(S - H).u_j|).", "",
             "| Eq. 7 bound | points | " + " | ".join(cols) + " |",
             "|---|---:|" + "---:|" * len(cols)]
    res["bins"] = []
    for lo, hi in zip(bins[:-1], bins[1:]):
        m = (qu >= lo) & (qu < hi) & strong
        if not np.any(m):
            continue
        errs = [float(np.max(np.abs(a[m] - r[m]) / np.abs(r[m]))) for a, r in cols.values()]
        res["bins"].append((lo, hi, int(m.sum()), errs))
        lines.append(f"| [{lo:g}, {hi:g}) | {int(m.sum())} | " + " | ".join(f"{e:.2e}" for e in errs) + " |")
    res["t2"] = {k: float(np.linalg.norm(a - r) / np.linalg.norm(r)) for k, (a, r) in cols.items()}
    lines += ["", "| form | pairs or grid size | time of a second call (ms, incl. host sync) |",
              "|---|---:|---:|",
              f"| atom-by-atom, all-FP64 path | {atoms64.shape[0] * S64.shape[0]:.2e} pairs | "
              f"{res['t_exact_f64'] * 1e3:.2f} |",
              f"| atom-by-atom, FP64-phase | {atoms64.shape[0] * S64.shape[0]:.2e} pairs | "
              f"{res['t_atoms_ph64'] * 1e3:.2f} |",
              f"| Eq. 4, species kernel | {blocks64.shape[0] * S64.shape[0]:.2e} pairs | "
              f"{res['t_block_ph64'] * 1e3:.2f} |",
              f"| Eq. 5, FFT over the whole padded grid | {Sg.shape[0]} points | "
              f"{res['t_fft'] * 1e3:.2f} |", "",
              "Normwise (T2) over all points: " + ", ".join(f"{k}: {v:.2e}" for k, v in res["t2"].items())]
    return "\n".join(lines) + "\n", res


def main(argv=None):
    p = argparse.ArgumentParser(description="Eq. 4 / Eq. 5 accuracy comparison")
    p.add_argument("--cells", type=int, default=29)
    p.add_argument("--pad", type=int, default=4)
    p.add_argument("--window", type=float, default=0.2)
    p.add_argument("--out", default=None)
    a = p.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("approx: needs a GPU (libnx has no CPU path)")
    text, _ = compare(a.cells, a.pad, a.window)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text)
    print(text, flush=True)


if __name__ == "__main__":
    main()
