"""PyTorch-facing wrappers of libnx.  Torch supplies device memory and the current
stream only: each wrapper checks shapes, dtypes and devices, allocates the outputs
and the workspace with the caching allocator, and makes one call into the HIP
library (include/nx.h), which does all the arithmetic.

* ``scatter_fwd`` / ``scatter_bwd``         -- Eq. 2 of Favre-Nicolin et al. (2010)
  and its adjoint in FP32 with FP64 phase reduction (``mode="ph64"``, default) or the
  paper's plain FP32 arithmetic (``mode="f32"``);
* ``scatter_fwd_f64`` / ``scatter_bwd_f64`` -- the all-FP64 path;
* ``loss_grad``                             -- misfit L = sum (|A|^2 - I)^2 and seed G;
* ``scatter``                               -- differentiable forward (autograd.Function);
* ``fit_step``                              -- forward, misfit and adjoint in one call.
"""
from __future__ import annotations

from typing import Optional, Tuple

import torch

from . import _lib

MODES = {"f32": _lib.NX_F32, "ph64": _lib.NX_F32_PH64}


def _mode(mode) -> int:
    if isinstance(mode, int):
        return mode
    try:
        return MODES[mode]
    except KeyError:
        raise ValueError(f"unknown mode {mode!r}; expected one of {sorted(MODES)}") from None


def _need_gpu(t: torch.Tensor, name: str, dtype, shape_tail=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU (got {t.device}); libnx has no CPU path")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if shape_tail is not None and (t.dim() != 2 or t.shape[1] != shape_tail):
        raise ValueError(f"{name} must have shape (n, {shape_tail}) (got {tuple(t.shape)})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _workspace(nbytes: int, device) -> Tuple[Optional[torch.Tensor], int]:
    if nbytes == 0:
        return None, 0
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


def _f_arg(f: Optional[torch.Tensor], n: int, dtype):
    if f is None:
        return None
    _need_gpu(f, "f", dtype)
    if f.dim() != 1 or f.shape[0] != n:
        raise ValueError(f"f must have shape ({n},) (got {tuple(f.shape)})")
    return torch.view_as_real(f)


def workspace_bytes(n_atoms: int, n_points: int, mode="ph64", op=_lib.NX_OP_FWD,
                    f_is_null: bool = False) -> int:
    n = _lib.nx_workspace_bytes(n_atoms, n_points, _mode(mode), op, int(bool(f_is_null)))
    msg = _lib.last_error()
    if msg:
        raise _lib.NxError(_lib.NX_ERR_ARG, msg)
    return int(n)


def scatter_fwd(xyz: torch.Tensor, f: Optional[torch.Tensor], S: torch.Tensor, mode="ph64",
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """A_k = sum_j f_j exp(2 i pi S_k . r_j) (Eq. 2).  xyz (N,3) float32, f (N,)
    complex64 or None (f_j = 1), S (K,3) float32 -> A (K,) complex64."""
    _need_gpu(xyz, "xyz", torch.float32, 3)
    _need_gpu(S, "S", torch.float32, 3)
    n, k = xyz.shape[0], S.shape[0]
    fr = _f_arg(f, n, torch.complex64)
    m = _mode(mode)
    if out is None:
        out = torch.empty(k, dtype=torch.complex64, device=S.device)
    ws, wsb = _workspace(workspace_bytes(n, k, m, _lib.NX_OP_FWD, f is None), S.device)
    _lib.check(_lib.nx_scatter_fwd(_ptr(xyz), _ptr(fr), n, _ptr(S), k,
                                   _ptr(torch.view_as_real(out)), m, _ptr(ws), wsb,
                                   _stream(S.device)))
    return out


def scatter_bwd(xyz: torch.Tensor, f: Optional[torch.Tensor], S: torch.Tensor, G: torch.Tensor,
                mode="ph64") -> torch.Tensor:
    """dL/dr_j = Re sum_k conj(G_k) f_j (2 i pi S_k) exp(2 i pi S_k . r_j) for the seed
    G = dL/dRe A + i dL/dIm A (K,) complex64 -> (N,3) float32."""
    _need_gpu(xyz, "xyz", torch.float32, 3)
    _need_gpu(S, "S", torch.float32, 3)
    _need_gpu(G, "G", torch.complex64)
    n, k = xyz.shape[0], S.shape[0]
    if G.dim() != 1 or G.shape[0] != k:
        raise ValueError(f"G must have shape ({k},)")
    fr = _f_arg(f, n, torch.complex64)
    m = _mode(mode)
    grad = torch.empty((n, 3), dtype=torch.float32, device=xyz.device)
    ws, wsb = _workspace(workspace_bytes(n, k, m, _lib.NX_OP_BWD, f is None), xyz.device)
    _lib.check(_lib.nx_scatter_bwd(_ptr(xyz), _ptr(fr), n, _ptr(S), k,
                                   _ptr(torch.view_as_real(G)), _ptr(grad), m, _ptr(ws), wsb,
                                   _stream(xyz.device)))
    return grad


def scatter_fwd_f64(xyz: torch.Tensor, f: Optional[torch.Tensor], S: torch.Tensor) -> torch.Tensor:
    """All-FP64 Eq. 2: xyz (N,3) float64, f (N,) complex128 or None, S (K,3) float64
    -> (K,) complex128."""
    _need_gpu(xyz, "xyz", torch.float64, 3)
    _need_gpu(S, "S", torch.float64, 3)
    n, k = xyz.shape[0], S.shape[0]
    fr = _f_arg(f, n, torch.complex128)
    out = torch.empty(k, dtype=torch.complex128, device=S.device)
    ws, wsb = _workspace(workspace_bytes(n, k, 0, _lib.NX_OP_FWD_F64, f is None), S.device)
    _lib.check(_lib.nx_scatter_fwd_f64(_ptr(xyz), _ptr(fr), n, _ptr(S), k,
                                       _ptr(torch.view_as_real(out)), _ptr(ws), wsb,
                                       _stream(S.device)))
    return out


def scatter_bwd_f64(xyz: torch.Tensor, f: Optional[torch.Tensor], S: torch.Tensor,
                    G: torch.Tensor) -> torch.Tensor:
    """All-FP64 adjoint: G (K,) complex128 -> (N,3) float64."""
    _need_gpu(xyz, "xyz", torch.float64, 3)
    _need_gpu(S, "S", torch.float64, 3)
    _need_gpu(G, "G", torch.complex128)
    n, k = xyz.shape[0], S.shape[0]
    if G.dim() != 1 or G.shape[0] != k:
        raise ValueError(f"G must have shape ({k},)")
    fr = _f_arg(f, n, torch.complex128)
    grad = torch.empty((n, 3), dtype=torch.float64, device=xyz.device)
    ws, wsb = _workspace(workspace_bytes(n, k, 0, _lib.NX_OP_BWD_F64, f is None), xyz.device)
    _lib.check(_lib.nx_scatter_bwd_f64(_ptr(xyz), _ptr(fr), n, _ptr(S), k,
                                       _ptr(torch.view_as_real(G)), _ptr(grad), _ptr(ws), wsb,
                                       _stream(xyz.device)))
    return grad


def loss_grad(A: torch.Tensor, I: torch.Tensor, want_grad: bool = True):
    """L = sum_k (|A_k|^2 - I_k)^2 (float64 scalar tensor on the device) and the seed
    G = 4 (|A|^2 - I) A (complex64) or None."""
    _need_gpu(A, "A", torch.complex64)
    _need_gpu(I, "I", torch.float32)
    k = A.shape[0]
    if A.dim() != 1 or I.dim() != 1 or I.shape[0] != k:
        raise ValueError("A and I must be 1-D of the same length")
    L = torch.empty((), dtype=torch.float64, device=A.device)
    G = torch.empty(k, dtype=torch.complex64, device=A.device) if want_grad else None
    ws, wsb = _workspace(workspace_bytes(0, k, 0, _lib.NX_OP_LOSS, True), A.device)
    _lib.check(_lib.nx_loss_grad(_ptr(torch.view_as_real(A)), _ptr(I), k, _ptr(L),
                                 None if G is None else _ptr(torch.view_as_real(G)),
                                 _ptr(ws), wsb, _stream(A.device)))
    return L, G


class ScatterFn(torch.autograd.Function):
    """Differentiable Eq. 2 with respect to the positions (f and S are constants).
    Backward receives torch's complex gradient dL/dRe A + i dL/dIm A and calls the
    hand-written adjoint kernel; the phases are recomputed, never stored."""

    @staticmethod
    def forward(ctx, xyz, f, S, mode):
        ctx.save_for_backward(xyz, f, S) if f is not None else ctx.save_for_backward(xyz, S)
        ctx.has_f = f is not None
        ctx.mode = mode
        if xyz.dtype == torch.float64:
            return scatter_fwd_f64(xyz, f, S)
        return scatter_fwd(xyz, f, S, mode)

    @staticmethod
    def backward(ctx, gA):
        if ctx.has_f:
            xyz, f, S = ctx.saved_tensors
        else:
            (xyz, S), f = ctx.saved_tensors, None
        if not ctx.needs_input_grad[0]:
            return None, None, None, None
        if xyz.dtype == torch.float64:
            g = scatter_bwd_f64(xyz, f, S, gA.to(torch.complex128).contiguous())
        else:
            g = scatter_bwd(xyz, f, S, gA.to(torch.complex64).contiguous(), ctx.mode)
        return g, None, None, None


def scatter(xyz: torch.Tensor, f: Optional[torch.Tensor], S: torch.Tensor, mode="ph64"):
    """Differentiable forward sum; float64 xyz/S select the all-FP64 path."""
    return ScatterFn.apply(xyz, f, S, mode)


def fit_step(xyz: torch.Tensor, f: Optional[torch.Tensor], S: torch.Tensor, I: torch.Tensor,
             mode="ph64"):
    """One fitting step's hot path on the current stream: A = Eq. 2, misfit L and seed
    G, then dL/dxyz by the adjoint.  Returns (L, A, grad_xyz)."""
    A = scatter_fwd(xyz, f, S, mode)
    L, G = loss_grad(A, I)
    grad = scatter_bwd(xyz, f, S, G, mode)
    return L, A, grad
