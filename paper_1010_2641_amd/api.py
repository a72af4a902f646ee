"""PyTorch-facing wrappers of libnx.  Torch supplies device memory and the current
stream only: each wrapper checks shapes, dtypes and devices, allocates the outputs
and the workspace with the caching allocator, and makes one call into the HIP
library (include/nx.h), which does all the arithmetic.

* ``scatter_fwd`` / ``scatter_bwd``         -- Eq. 2 of Favre-Nicolin et al. (2010)
  and its adjoint in FP32 with FP64 phase reduction (``mode="ph64"``, default) or the
  paper's plain FP32 arithmetic (``mode="f32"``);
* ``scatter_fwd_f64`` / ``scatter_bwd_f64`` -- the all-FP64 path;
* ``loss_grad``                             -- misfit L = sum (|A|^2 - I)^2 and seed G;
* ``scatter_bwd_ex`` / ``scatter_bwd_ex_f64`` -- the adjoint with dL/df as well;
* ``scatter_fwd_species`` / ``scatter_bwd_species`` -- the species-factorised sum of
  Section 4.2 (unit-factor sums per species times S-dependent species factors);
* ``scatter``, ``scatter_species``          -- differentiable forwards (autograd.Function);
* ``fit_step``, ``fit_step_species``        -- forward, misfit and adjoint in one call;
* ``Grid``, ``scatter_fwd_grid``, ``scatter_bwd_grid``, ``fit_step_grid`` -- the same sums
  over a regular grid of points given exactly (FP64 origin and steps), walked by rows;
  ``scatter_grid`` is differentiable with respect to the positions;
  ``scatter_fwd_species_grid`` / ``scatter_bwd_species_grid`` the species-factorised sum
  over such a grid.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

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


def _need(t: torch.Tensor, name: str, dtype, shape=None):
    """Type, dtype, shape and layout of one tensor argument (no device check, so that
    these checks also run, and can be tested, on CPU tensors).  ``shape`` is a tuple
    whose None entries match any size."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if shape is not None and (t.dim() != len(shape) or any(
            want is not None and got != want for got, want in zip(t.shape, shape))):
        want = ", ".join("n" if v is None else str(v) for v in shape)
        raise ValueError(f"{name} must have shape ({want}{',' if len(shape) == 1 else ''}) "
                         f"(got {tuple(t.shape)})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.is_conj():
        raise ValueError(f"{name} is an unresolved conjugate view; call resolve_conj() first")


def _on_gpu(**tensors):
    """Every given tensor (None entries skipped) on one and the same GPU: the library
    takes device pointers only and has no CPU path."""
    dev = None
    for name, t in tensors.items():
        if t is None:
            continue
        if t.device.type != "cuda":
            raise ValueError(f"{name} must be on the GPU (got {t.device}); libnx has no CPU path")
        if dev is None:
            dev = t.device
        elif t.device != dev:
            raise ValueError(f"{name} is on {t.device}, the other arguments on {dev}")


def _seed_arg(gA: torch.Tensor, dtype) -> torch.Tensor:
    """An adjoint seed as a plain contiguous tensor of `dtype`: autograd may hand
    backward a lazy conjugate view (e.g. after A.conj()), which view_as_real refuses."""
    return gA.resolve_conj().to(dtype).contiguous()


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
    _need(f, "f", dtype, (n,))
    return f


def _real(t: Optional[torch.Tensor]) -> Optional[torch.Tensor]:
    """A complex tensor for the C ABI's interleaved (re, im) arrays: a contiguous complex
    tensor already is that array (its data pointer is the first real part), so it is
    passed as it is, without building a view."""
    return t


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
    complex64 or None (f_j = 1), S (K,3) float32 -> A (K,) complex64 (written into
    ``out`` when given: a contiguous (K,) complex64 tensor on the same GPU)."""
    _need(xyz, "xyz", torch.float32, (None, 3))
    _need(S, "S", torch.float32, (None, 3))
    n, k = xyz.shape[0], S.shape[0]
    _f_arg(f, n, torch.complex64)
    if out is not None:
        _need(out, "out", torch.complex64, (k,))
    m = _mode(mode)
    _on_gpu(xyz=xyz, S=S, f=f, out=out)
    if out is None:
        out = torch.empty(k, dtype=torch.complex64, device=S.device)
    ws, wsb = _workspace(workspace_bytes(n, k, m, _lib.NX_OP_FWD, f is None), S.device)
    _lib.check(_lib.nx_scatter_fwd(_ptr(xyz), _ptr(_real(f)), n, _ptr(S), k,
                                   _ptr(_real(out)), m, _ptr(ws), wsb, _stream(S.device)))
    return out


def scatter_bwd(xyz: torch.Tensor, f: Optional[torch.Tensor], S: torch.Tensor, G: torch.Tensor,
                mode="ph64") -> torch.Tensor:
    """dL/dr_j = Re sum_k conj(G_k) f_j (2 i pi S_k) exp(2 i pi S_k . r_j) for the seed
    G = dL/dRe A + i dL/dIm A (K,) complex64 -> (N,3) float32."""
    _need(xyz, "xyz", torch.float32, (None, 3))
    _need(S, "S", torch.float32, (None, 3))
    n, k = xyz.shape[0], S.shape[0]
    _need(G, "G", torch.complex64, (k,))
    _f_arg(f, n, torch.complex64)
    m = _mode(mode)
    _on_gpu(xyz=xyz, S=S, G=G, f=f)
    grad = torch.empty((n, 3), dtype=torch.float32, device=xyz.device)
    ws, wsb = _workspace(workspace_bytes(n, k, m, _lib.NX_OP_BWD, f is None), xyz.device)
    _lib.check(_lib.nx_scatter_bwd(_ptr(xyz), _ptr(_real(f)), n, _ptr(S), k, _ptr(_real(G)),
                                   _ptr(grad), m, _ptr(ws), wsb, _stream(xyz.device)))
    return grad


def scatter_fwd_f64(xyz: torch.Tensor, f: Optional[torch.Tensor], S: torch.Tensor) -> torch.Tensor:
    """All-FP64 Eq. 2: xyz (N,3) float64, f (N,) complex128 or None, S (K,3) float64
    -> (K,) complex128."""
    _need(xyz, "xyz", torch.float64, (None, 3))
    _need(S, "S", torch.float64, (None, 3))
    n, k = xyz.shape[0], S.shape[0]
    _f_arg(f, n, torch.complex128)
    _on_gpu(xyz=xyz, S=S, f=f)
    out = torch.empty(k, dtype=torch.complex128, device=S.device)
    ws, wsb = _workspace(workspace_bytes(n, k, 0, _lib.NX_OP_FWD_F64, f is None), S.device)
    _lib.check(_lib.nx_scatter_fwd_f64(_ptr(xyz), _ptr(_real(f)), n, _ptr(S), k, _ptr(_real(out)),
                                       _ptr(ws), wsb, _stream(S.device)))
    return out


def scatter_bwd_f64(xyz: torch.Tensor, f: Optional[torch.Tensor], S: torch.Tensor,
                    G: torch.Tensor) -> torch.Tensor:
    """All-FP64 adjoint: G (K,) complex128 -> (N,3) float64."""
    _need(xyz, "xyz", torch.float64, (None, 3))
    _need(S, "S", torch.float64, (None, 3))
    n, k = xyz.shape[0], S.shape[0]
    _need(G, "G", torch.complex128, (k,))
    _f_arg(f, n, torch.complex128)
    _on_gpu(xyz=xyz, S=S, G=G, f=f)
    grad = torch.empty((n, 3), dtype=torch.float64, device=xyz.device)
    ws, wsb = _workspace(workspace_bytes(n, k, 0, _lib.NX_OP_BWD_F64, f is None), xyz.device)
    _lib.check(_lib.nx_scatter_bwd_f64(_ptr(xyz), _ptr(_real(f)), n, _ptr(S), k, _ptr(_real(G)),
                                       _ptr(grad), _ptr(ws), wsb, _stream(xyz.device)))
    return grad


def scatter_bwd_ex(xyz: torch.Tensor, f: Optional[torch.Tensor], S: torch.Tensor, G: torch.Tensor,
                   mode="ph64", want_xyz: bool = True, want_f: bool = True):
    """The adjoint with the factor gradient: returns (dL/dxyz (N,3) float32 or None,
    dL/df (N,) complex64 or None)."""
    _need(xyz, "xyz", torch.float32, (None, 3))
    _need(S, "S", torch.float32, (None, 3))
    n, k = xyz.shape[0], S.shape[0]
    _need(G, "G", torch.complex64, (k,))
    _f_arg(f, n, torch.complex64)
    m = _mode(mode)
    _on_gpu(xyz=xyz, S=S, G=G, f=f)
    grad = torch.empty((n, 3), dtype=torch.float32, device=xyz.device) if want_xyz else None
    gradf = torch.empty(n, dtype=torch.complex64, device=xyz.device) if want_f else None
    op = _lib.NX_OP_BWD_GF if want_f else _lib.NX_OP_BWD
    ws, wsb = _workspace(workspace_bytes(n, k, m, op, f is None), xyz.device)
    _lib.check(_lib.nx_scatter_bwd_ex(_ptr(xyz), _ptr(_real(f)), n, _ptr(S), k, _ptr(_real(G)),
                                      _ptr(grad), _ptr(_real(gradf)), m, _ptr(ws), wsb,
                                      _stream(xyz.device)))
    return grad, gradf


def scatter_bwd_ex_f64(xyz: torch.Tensor, f: Optional[torch.Tensor], S: torch.Tensor,
                       G: torch.Tensor, want_xyz: bool = True, want_f: bool = True):
    """All-FP64 adjoint with the factor gradient: (dL/dxyz float64 or None, dL/df complex128
    or None)."""
    _need(xyz, "xyz", torch.float64, (None, 3))
    _need(S, "S", torch.float64, (None, 3))
    n, k = xyz.shape[0], S.shape[0]
    _need(G, "G", torch.complex128, (k,))
    _f_arg(f, n, torch.complex128)
    _on_gpu(xyz=xyz, S=S, G=G, f=f)
    grad = torch.empty((n, 3), dtype=torch.float64, device=xyz.device) if want_xyz else None
    gradf = torch.empty(n, dtype=torch.complex128, device=xyz.device) if want_f else None
    op = _lib.NX_OP_BWD_GF_F64 if want_f else _lib.NX_OP_BWD_F64
    ws, wsb = _workspace(workspace_bytes(n, k, 0, op, f is None), xyz.device)
    _lib.check(_lib.nx_scatter_bwd_ex_f64(_ptr(xyz), _ptr(_real(f)), n, _ptr(S), k, _ptr(_real(G)),
                                          _ptr(grad), _ptr(_real(gradf)), _ptr(ws), wsb,
                                          _stream(xyz.device)))
    return grad, gradf


def _species_array(species_start: Sequence[int], n_atoms: int):
    start = [int(v) for v in species_start]
    if len(start) < 2 or start[0] != 0 or start[-1] != n_atoms or any(
            b < a for a, b in zip(start, start[1:])):
        raise ValueError("species_start must run from 0 to n_atoms without decreasing")
    if len(start) - 1 > _lib.NX_MAX_SPECIES:
        raise ValueError(f"at most {_lib.NX_MAX_SPECIES} species")
    return (ctypes.c_int64 * len(start))(*start), len(start) - 1


def _fs_arg(fs: Optional[torch.Tensor], ns: int, k: int):
    if fs is None:
        return None
    _need(fs, "fs", torch.complex64, (ns, k))
    return fs


def scatter_fwd_species(xyz: torch.Tensor, species_start: Sequence[int], fs: Optional[torch.Tensor],
                        S: torch.Tensor, mode="ph64", return_species: bool = False):
    """A_k = sum_s fs[s, k] sum_{j in species s} exp(2 i pi S_k . r_j) (Section 4.2): atoms
    listed species by species, species s = atoms [species_start[s], species_start[s+1]);
    fs (n_species, K) complex64 or None.  Returns A (K,) complex64, and the per-species
    sums (n_species, K) when return_species."""
    _need(xyz, "xyz", torch.float32, (None, 3))
    _need(S, "S", torch.float32, (None, 3))
    n, k = xyz.shape[0], S.shape[0]
    start, ns = _species_array(species_start, n)
    _fs_arg(fs, ns, k)
    m = _mode(mode)
    _on_gpu(xyz=xyz, S=S, fs=fs)
    A = torch.empty(k, dtype=torch.complex64, device=S.device)
    As = torch.empty((ns, k), dtype=torch.complex64, device=S.device) if return_species else None
    nb = _lib.nx_workspace_bytes_species(start, ns, k, m, 0)
    if _lib.last_error():
        raise _lib.NxError(_lib.NX_ERR_ARG, _lib.last_error())
    ws, wsb = _workspace(int(nb), S.device)
    _lib.check(_lib.nx_scatter_fwd_species(_ptr(xyz), n, start, ns, _ptr(_real(fs)), _ptr(S), k,
                                           _ptr(_real(A)), _ptr(_real(As)), m, _ptr(ws), wsb,
                                           _stream(S.device)))
    return (A, As) if return_species else A


def scatter_bwd_species(xyz: torch.Tensor, species_start: Sequence[int], fs: Optional[torch.Tensor],
                        S: torch.Tensor, G: torch.Tensor, A_species: Optional[torch.Tensor] = None,
                        mode="ph64", want_xyz: bool = True):
    """Adjoint of ``scatter_fwd_species``: (dL/dxyz (N,3) float32 or None, dL/dfs
    (n_species, K) complex64 or None -- the latter when A_species, the per-species sums
    (n_species, K) complex64 of the forward, is given)."""
    _need(xyz, "xyz", torch.float32, (None, 3))
    _need(S, "S", torch.float32, (None, 3))
    n, k = xyz.shape[0], S.shape[0]
    _need(G, "G", torch.complex64, (k,))
    start, ns = _species_array(species_start, n)
    _fs_arg(fs, ns, k)
    if A_species is not None:
        _need(A_species, "A_species", torch.complex64, (ns, k))
    m = _mode(mode)
    _on_gpu(xyz=xyz, S=S, G=G, fs=fs, A_species=A_species)
    grad = torch.empty((n, 3), dtype=torch.float32, device=xyz.device) if want_xyz else None
    gfs = torch.empty((ns, k), dtype=torch.complex64, device=xyz.device) if A_species is not None else None
    nb = _lib.nx_workspace_bytes_species(start, ns, k, m, 1)
    if _lib.last_error():
        raise _lib.NxError(_lib.NX_ERR_ARG, _lib.last_error())
    ws, wsb = _workspace(int(nb), xyz.device)
    _lib.check(_lib.nx_scatter_bwd_species(_ptr(xyz), n, start, ns, _ptr(_real(fs)), _ptr(S), k,
                                           _ptr(_real(G)), _ptr(_real(A_species)), _ptr(grad),
                                           _ptr(_real(gfs)), m, _ptr(ws), wsb, _stream(xyz.device)))
    return grad, gfs


def loss_grad(A: torch.Tensor, I: torch.Tensor, want_grad: bool = True):
    """L = sum_k (|A_k|^2 - I_k)^2 (float64 scalar tensor on the device) and the seed
    G = 4 (|A|^2 - I) A (complex64) or None."""
    _need(A, "A", torch.complex64, (None,))
    k = A.shape[0]
    _need(I, "I", torch.float32, (k,))
    _on_gpu(A=A, I=I)
    L = torch.empty((), dtype=torch.float64, device=A.device)
    G = torch.empty(k, dtype=torch.complex64, device=A.device) if want_grad else None
    ws, wsb = _workspace(workspace_bytes(0, k, 0, _lib.NX_OP_LOSS, True), A.device)
    _lib.check(_lib.nx_loss_grad(_ptr(_real(A)), _ptr(I), k, _ptr(L), _ptr(_real(G)),
                                 _ptr(ws), wsb, _stream(A.device)))
    return L, G


class ScatterFn(torch.autograd.Function):
    """Differentiable Eq. 2 with respect to the positions and the factors (S is a
    constant).  Backward receives torch's complex gradient dL/dRe A + i dL/dIm A and calls
    the hand-written adjoint kernel; the phases are recomputed, never stored."""

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
        want_x = ctx.needs_input_grad[0]
        want_f = ctx.has_f and ctx.needs_input_grad[1]
        if not (want_x or want_f):
            return None, None, None, None
        if xyz.dtype == torch.float64:
            gx, gf = scatter_bwd_ex_f64(xyz, f, S, _seed_arg(gA, torch.complex128), want_x, want_f)
        else:
            gx, gf = scatter_bwd_ex(xyz, f, S, _seed_arg(gA, torch.complex64), ctx.mode,
                                    want_x, want_f)
        return gx, gf, None, None


class ScatterSpeciesFn(torch.autograd.Function):
    """Differentiable species-factorised sum with respect to the positions and the
    per-species factors fs (n_species, K)."""

    @staticmethod
    def forward(ctx, xyz, fs, S, species_start, mode):
        A, As = scatter_fwd_species(xyz, species_start, fs, S, mode, return_species=True)
        ctx.save_for_backward(xyz, S, As, fs) if fs is not None else ctx.save_for_backward(xyz, S, As)
        ctx.has_fs = fs is not None
        ctx.species_start = list(species_start)
        ctx.mode = mode
        return A

    @staticmethod
    def backward(ctx, gA):
        if ctx.has_fs:
            xyz, S, As, fs = ctx.saved_tensors
        else:
            (xyz, S, As), fs = ctx.saved_tensors, None
        want_x = ctx.needs_input_grad[0]
        want_fs = ctx.has_fs and ctx.needs_input_grad[1]
        gx, gfs = scatter_bwd_species(xyz, ctx.species_start, fs, S, _seed_arg(gA, torch.complex64),
                                      As if want_fs else None, ctx.mode, want_x)
        return gx, gfs, None, None, None


def scatter_species(xyz: torch.Tensor, species_start: Sequence[int], fs: Optional[torch.Tensor],
                    S: torch.Tensor, mode="ph64"):
    """Differentiable species-factorised forward."""
    return ScatterSpeciesFn.apply(xyz, fs, S, list(species_start), mode)


def scatter(xyz: torch.Tensor, f: Optional[torch.Tensor], S: torch.Tensor, mode="ph64"):
    """Differentiable forward sum; float64 xyz/S select the all-FP64 path."""
    return ScatterFn.apply(xyz, f, S, mode)


def fit_step_species(xyz: torch.Tensor, species_start: Sequence[int], fs: Optional[torch.Tensor],
                     S: torch.Tensor, I: torch.Tensor, mode="ph64"):
    """The fit step with the species-factorised sum: (L, A, dL/dxyz)."""
    A = scatter_fwd_species(xyz, species_start, fs, S, mode)
    L, G = loss_grad(A, I)
    grad, _ = scatter_bwd_species(xyz, species_start, fs, S, G, None, mode)
    return L, A, grad


def fit_step(xyz: torch.Tensor, f: Optional[torch.Tensor], S: torch.Tensor, I: torch.Tensor,
             mode="ph64", return_seed: bool = False):
    """One fitting step's hot path on the current stream, queued by one call into the
    library (nx_fit_step): A = Eq. 2, misfit L and seed G, then dL/dxyz by the adjoint.
    Returns (L, A, grad_xyz), and G as well when return_seed."""
    _need(xyz, "xyz", torch.float32, (None, 3))
    _need(S, "S", torch.float32, (None, 3))
    n, k = xyz.shape[0], S.shape[0]
    _f_arg(f, n, torch.complex64)
    _need(I, "I", torch.float32, (k,))
    m = _mode(mode)
    _on_gpu(xyz=xyz, S=S, f=f, I=I)
    dev = S.device
    A = torch.empty(k, dtype=torch.complex64, device=dev)
    G = torch.empty(k, dtype=torch.complex64, device=dev)
    L = torch.empty((), dtype=torch.float64, device=dev)
    grad = torch.empty((n, 3), dtype=torch.float32, device=dev)
    ws, wsb = _workspace(workspace_bytes(n, k, m, _lib.NX_OP_FIT, f is None), dev)
    _lib.check(_lib.nx_fit_step(_ptr(xyz), _ptr(f), n, _ptr(S), k, _ptr(I), _ptr(A), _ptr(L),
                                _ptr(G), _ptr(grad), m, _ptr(ws), wsb, _stream(dev)))
    return (L, A, grad, G) if return_seed else (L, A, grad)


@dataclass(frozen=True)
class Grid:
    """A regular grid of reciprocal-space points (r.l.u., FP64): point (i1, i2, i3) is
    origin + i1 step1 + i2 step2 + i3 step3, 0 <= i_a < n_a, listed with i1 fastest
    (k = i1 + n1 (i2 + n2 i3)), the order of A, G and I in the grid calls."""
    origin: Tuple[float, float, float]
    step1: Tuple[float, float, float]
    step2: Tuple[float, float, float]
    step3: Tuple[float, float, float]
    n1: int
    n2: int = 1
    n3: int = 1

    @property
    def size(self) -> int:
        return int(self.n1) * int(self.n2) * int(self.n3)



def _grid_arg(grid) -> Tuple[_lib.nx_grid, int]:
    """The nx_grid struct and point count of a Grid (or of any object with the same
    fields, such as a workload's grid)."""
    try:
        parts = {name: tuple(float(x) for x in getattr(grid, name))
                 for name in ("origin", "step1", "step2", "step3")}
        counts = tuple(int(getattr(grid, name)) for name in ("n1", "n2", "n3"))
    except (AttributeError, TypeError):
        raise TypeError("grid must be a Grid (origin, step1, step2, step3, n1, n2, n3)") from None
    g = _lib.nx_grid()
    for name, v in parts.items():
        if len(v) != 3:
            raise ValueError(f"grid {name} must have 3 components (got {len(v)})")
        getattr(g, name)[:] = v
    if min(counts) < 0:
        raise ValueError(f"grid counts must be >= 0 (got {counts})")
    g.n1, g.n2, g.n3 = counts
    return g, counts[0] * counts[1] * counts[2]


def workspace_bytes_grid(n_atoms: int, grid: Grid, op=_lib.NX_OP_FWD, f_is_null: bool = False) -> int:
    g, _ = _grid_arg(grid)
    n = _lib.nx_workspace_bytes_grid(n_atoms, ctypes.byref(g), op, int(bool(f_is_null)))
    msg = _lib.last_error()
    if msg:
        raise _lib.NxError(_lib.NX_ERR_ARG, msg)
    return int(n)


def scatter_fwd_grid(xyz: torch.Tensor, f: Optional[torch.Tensor], grid: Grid,
                     out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Eq. 2 over the points of ``grid`` (FP64-phase mode): xyz (N,3) float32, f (N,)
    complex64 or None -> A (grid.size,) complex64, in the grid's order."""
    _need(xyz, "xyz", torch.float32, (None, 3))
    g, k = _grid_arg(grid)
    n = xyz.shape[0]
    _f_arg(f, n, torch.complex64)
    if out is not None:
        _need(out, "out", torch.complex64, (k,))
    _on_gpu(xyz=xyz, f=f, out=out)
    nbytes = workspace_bytes_grid(n, grid, _lib.NX_OP_FWD, f is None)    # validates the grid
    if out is None:
        out = torch.empty(k, dtype=torch.complex64, device=xyz.device)
    ws, wsb = _workspace(nbytes, xyz.device)
    _lib.check(_lib.nx_scatter_fwd_grid(_ptr(xyz), _ptr(f), n, ctypes.byref(g), _ptr(out),
                                        _lib.NX_F32_PH64, _ptr(ws), wsb, _stream(xyz.device)))
    return out


def scatter_bwd_grid(xyz: torch.Tensor, f: Optional[torch.Tensor], grid: Grid,
                     G: torch.Tensor) -> torch.Tensor:
    """The position adjoint over the points of ``grid``: seed G (grid.size,) complex64 ->
    dL/dxyz (N,3) float32 (as scatter_bwd)."""
    _need(xyz, "xyz", torch.float32, (None, 3))
    g, k = _grid_arg(grid)
    n = xyz.shape[0]
    _need(G, "G", torch.complex64, (k,))
    _f_arg(f, n, torch.complex64)
    _on_gpu(xyz=xyz, G=G, f=f)
    nbytes = workspace_bytes_grid(n, grid, _lib.NX_OP_BWD, f is None)
    grad = torch.empty((n, 3), dtype=torch.float32, device=xyz.device)
    ws, wsb = _workspace(nbytes, xyz.device)
    _lib.check(_lib.nx_scatter_bwd_grid(_ptr(xyz), _ptr(f), n, ctypes.byref(g), _ptr(G), _ptr(grad),
                                        _lib.NX_F32_PH64, _ptr(ws), wsb, _stream(xyz.device)))
    return grad


def fit_step_grid(xyz: torch.Tensor, f: Optional[torch.Tensor], grid: Grid, I: torch.Tensor,
                  return_seed: bool = False):
    """fit_step over the points of ``grid`` (nx_fit_step_grid): I (grid.size,) float32.
    Returns (L, A, grad_xyz), and G as well when return_seed."""
    _need(xyz, "xyz", torch.float32, (None, 3))
    g, k = _grid_arg(grid)
    n = xyz.shape[0]
    _f_arg(f, n, torch.complex64)
    _need(I, "I", torch.float32, (k,))
    _on_gpu(xyz=xyz, f=f, I=I)
    dev = xyz.device
    nbytes = workspace_bytes_grid(n, grid, _lib.NX_OP_FIT, f is None)
    A = torch.empty(k, dtype=torch.complex64, device=dev)
    G = torch.empty(k, dtype=torch.complex64, device=dev)
    L = torch.empty((), dtype=torch.float64, device=dev)
    grad = torch.empty((n, 3), dtype=torch.float32, device=dev)
    ws, wsb = _workspace(nbytes, dev)
    _lib.check(_lib.nx_fit_step_grid(_ptr(xyz), _ptr(f), n, ctypes.byref(g), _ptr(I), _ptr(A), _ptr(L),
                                     _ptr(G), _ptr(grad), _lib.NX_F32_PH64, _ptr(ws), wsb, _stream(dev)))
    return (L, A, grad, G) if return_seed else (L, A, grad)


def workspace_bytes_species_grid(species_start: Sequence[int], grid: Grid, op: int = 0) -> int:
    """Workspace bytes of the species-factorised calls over a grid (op 0 forward, 1 adjoint)."""
    g, _ = _grid_arg(grid)
    start, ns = _species_array(species_start, int(species_start[-1]) if len(species_start) else -1)
    n = _lib.nx_workspace_bytes_species_grid(start, ns, ctypes.byref(g), op)
    msg = _lib.last_error()
    if msg:
        raise _lib.NxError(_lib.NX_ERR_ARG, msg)
    return int(n)


def scatter_fwd_species_grid(xyz: torch.Tensor, species_start: Sequence[int], fs: Optional[torch.Tensor],
                             grid: Grid, return_species: bool = False):
    """``scatter_fwd_species`` over the points of ``grid`` (FP64-phase mode): fs
    (n_species, grid.size) complex64 or None.  Returns A (grid.size,) complex64, and the
    per-species sums (n_species, grid.size) when return_species."""
    _need(xyz, "xyz", torch.float32, (None, 3))
    g, k = _grid_arg(grid)
    n = xyz.shape[0]
    start, ns = _species_array(species_start, n)
    _fs_arg(fs, ns, k)
    _on_gpu(xyz=xyz, fs=fs)
    nbytes = workspace_bytes_species_grid(species_start, grid, 0)
    A = torch.empty(k, dtype=torch.complex64, device=xyz.device)
    As = torch.empty((ns, k), dtype=torch.complex64, device=xyz.device) if return_species else None
    ws, wsb = _workspace(nbytes, xyz.device)
    _lib.check(_lib.nx_scatter_fwd_species_grid(_ptr(xyz), n, start, ns, _ptr(_real(fs)), ctypes.byref(g),
                                                _ptr(_real(A)), _ptr(_real(As)), _lib.NX_F32_PH64,
                                                _ptr(ws), wsb, _stream(xyz.device)))
    return (A, As) if return_species else A


def scatter_bwd_species_grid(xyz: torch.Tensor, species_start: Sequence[int], fs: Optional[torch.Tensor],
                             grid: Grid, G: torch.Tensor, A_species: Optional[torch.Tensor] = None,
                             want_xyz: bool = True):
    """Adjoint of ``scatter_fwd_species_grid``: (dL/dxyz (N,3) float32 or None, dL/dfs
    (n_species, grid.size) complex64 or None -- the latter when A_species is given)."""
    _need(xyz, "xyz", torch.float32, (None, 3))
    g, k = _grid_arg(grid)
    n = xyz.shape[0]
    _need(G, "G", torch.complex64, (k,))
    start, ns = _species_array(species_start, n)
    _fs_arg(fs, ns, k)
    if A_species is not None:
        _need(A_species, "A_species", torch.complex64, (ns, k))
    _on_gpu(xyz=xyz, G=G, fs=fs, A_species=A_species)
    nbytes = workspace_bytes_species_grid(species_start, grid, 1)
    grad = torch.empty((n, 3), dtype=torch.float32, device=xyz.device) if want_xyz else None
    gfs = torch.empty((ns, k), dtype=torch.complex64, device=xyz.device) if A_species is not None else None
    ws, wsb = _workspace(nbytes, xyz.device)
    _lib.check(_lib.nx_scatter_bwd_species_grid(_ptr(xyz), n, start, ns, _ptr(_real(fs)), ctypes.byref(g),
                                                _ptr(_real(G)), _ptr(_real(A_species)), _ptr(grad),
                                                _ptr(_real(gfs)), _lib.NX_F32_PH64, _ptr(ws), wsb,
                                                _stream(xyz.device)))
    return grad, gfs


class ScatterGridFn(torch.autograd.Function):
    """Differentiable Eq. 2 over a grid with respect to the positions (the grid and f are
    constants).  Backward receives torch's complex gradient dL/dRe A + i dL/dIm A and calls
    the grid adjoint kernel."""

    @staticmethod
    def forward(ctx, xyz, f, grid):
        ctx.save_for_backward(xyz, f) if f is not None else ctx.save_for_backward(xyz)
        ctx.has_f = f is not None
        ctx.grid = grid
        return scatter_fwd_grid(xyz, f, grid)

    @staticmethod
    def backward(ctx, gA):
        if ctx.has_f:
            xyz, f = ctx.saved_tensors
        else:
            (xyz,), f = ctx.saved_tensors, None
        if not ctx.needs_input_grad[0]:
            return None, None, None
        return scatter_bwd_grid(xyz, f, ctx.grid, _seed_arg(gA, torch.complex64)), None, None


def scatter_grid(xyz: torch.Tensor, f: Optional[torch.Tensor], grid: Grid):
    """Differentiable forward sum over the points of ``grid`` (gradients with respect to
    xyz; the grid adjoint has no factor gradient: take dL/df through ``scatter`` with the
    grid's points as a list)."""
    if f is not None and f.requires_grad:
        raise NotImplementedError("scatter_grid: no gradient with respect to f over a grid; use "
                                  "scatter() with the grid's points for dL/df")
    return ScatterGridFn.apply(xyz, f, grid)
