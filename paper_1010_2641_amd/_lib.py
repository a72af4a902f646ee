"""ctypes binding of libnx (include/nx.h): the same entry points with the same names
and arguments.  Argument marshalling only -- every step of the sum runs in the HIP
library.  Importing this module loads libnx.so and fails loudly if it is missing;
there is no CPU fallback."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnx.so")

NX_OK, NX_ERR_ARG, NX_ERR_MODE, NX_ERR_WORKSPACE, NX_ERR_DEVICE = 0, -1, -2, -3, -4
NX_F32, NX_F32_PH64 = 0, 1
NX_OP_FWD, NX_OP_BWD, NX_OP_FWD_F64, NX_OP_BWD_F64, NX_OP_LOSS = 0, 1, 2, 3, 4
NX_OP_BWD_GF, NX_OP_BWD_GF_F64, NX_OP_FIT = 5, 6, 7
NX_MAX_COUNT = 1 << 30
NX_MAX_SPECIES = 16
NX_NOALLOC_SCRATCH_BYTES = 128 << 20



class nx_grid(ctypes.Structure):
    """struct nx_grid: point (i1, i2, i3) is origin + i1 step1 + i2 step2 + i3 step3 (FP64),
    listed with i1 fastest."""
    _fields_ = [("origin", ctypes.c_double * 3), ("step1", ctypes.c_double * 3),
                ("step2", ctypes.c_double * 3), ("step3", ctypes.c_double * 3),
                ("n1", ctypes.c_int64), ("n2", ctypes.c_int64), ("n3", ctypes.c_int64)]


# every symbol include/nx.h declares, with its ctypes signature
_VP, _I64, _SZ, _I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t, ctypes.c_int
_GP = ctypes.POINTER(nx_grid)
SIGNATURES = {
    "nx_version": ([], _I),
    "nx_last_error": ([], ctypes.c_char_p),
    "nx_workspace_bytes": ([_I64, _I64, _I, _I, _I], _SZ),
    "nx_scatter_fwd": ([_VP, _VP, _I64, _VP, _I64, _VP, _I, _VP, _SZ, _VP], _I),
    "nx_scatter_fwd_noalloc": ([_VP, _VP, _I64, _VP, _I64, _VP, _I, _VP], _I),
    "nx_scatter_bwd": ([_VP, _VP, _I64, _VP, _I64, _VP, _VP, _I, _VP, _SZ, _VP], _I),
    "nx_scatter_fwd_f64": ([_VP, _VP, _I64, _VP, _I64, _VP, _VP, _SZ, _VP], _I),
    "nx_scatter_bwd_f64": ([_VP, _VP, _I64, _VP, _I64, _VP, _VP, _VP, _SZ, _VP], _I),
    "nx_loss_grad": ([_VP, _VP, _I64, _VP, _VP, _VP, _SZ, _VP], _I),
    "nx_fit_step": ([_VP, _VP, _I64, _VP, _I64, _VP, _VP, _VP, _VP, _VP, _I, _VP, _SZ, _VP], _I),
    "nx_scatter_bwd_ex": ([_VP, _VP, _I64, _VP, _I64, _VP, _VP, _VP, _I, _VP, _SZ, _VP], _I),
    "nx_scatter_bwd_ex_f64": ([_VP, _VP, _I64, _VP, _I64, _VP, _VP, _VP, _VP, _SZ, _VP], _I),
    "nx_scatter_fwd_species": ([_VP, _I64, _VP, _I, _VP, _VP, _I64, _VP, _VP, _I, _VP, _SZ, _VP], _I),
    "nx_scatter_bwd_species": ([_VP, _I64, _VP, _I, _VP, _VP, _I64, _VP, _VP, _VP, _VP, _I, _VP, _SZ,
                                _VP], _I),
    "nx_workspace_bytes_species": ([_VP, _I, _I64, _I, _I], _SZ),
    "nx_workspace_bytes_grid": ([_I64, _GP, _I, _I], _SZ),
    "nx_scatter_fwd_grid": ([_VP, _VP, _I64, _GP, _VP, _I, _VP, _SZ, _VP], _I),
    "nx_scatter_bwd_grid": ([_VP, _VP, _I64, _GP, _VP, _VP, _I, _VP, _SZ, _VP], _I),
    "nx_fit_step_grid": ([_VP, _VP, _I64, _GP, _VP, _VP, _VP, _VP, _VP, _I, _VP, _SZ, _VP], _I),
    "nx_scatter_fwd_species_grid": ([_VP, _I64, _VP, _I, _VP, _GP, _VP, _VP, _I, _VP, _SZ, _VP], _I),
    "nx_scatter_bwd_species_grid": ([_VP, _I64, _VP, _I, _VP, _GP, _VP, _VP, _VP, _VP, _I, _VP, _SZ,
                                     _VP], _I),
    "nx_workspace_bytes_species_grid": ([_VP, _I, _GP, _I], _SZ),
}


class NxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libnx error {code}: {msg}")
        self.code = code


def _hip_runtimes():
    """Paths of the HIP runtime libraries mapped into this process (Linux)."""
    try:
        with open("/proc/self/maps") as fh:
            return sorted({l.split()[-1] for l in fh if "libamdhip64" in l})
    except OSError:
        return []


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1010_2641_amd.build` "
                           "(the HIP library is required; there is no CPU fallback)")
    # PyTorch ships its own HIP runtime.  It must be the one libnx binds to: if libnx were
    # loaded first, the dynamic linker would map the system runtime as well, and two HIP
    # (and HSA) runtimes in one process do not share devices, streams or memory.
    import torch  # noqa: F401  (loads torch's libamdhip64 before libnx resolves its own)
    lib = ctypes.CDLL(LIB_PATH)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise RuntimeError("more than one HIP runtime is loaded in this process "
                           f"({runtimes}); import torch before loading libnx")
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def last_error() -> str:
    return lib.nx_last_error().decode()


def check(code: int) -> None:
    if code != NX_OK:
        raise NxError(code, last_error())


# The entry points under their C names.
nx_version = lib.nx_version
nx_last_error = lib.nx_last_error
nx_workspace_bytes = lib.nx_workspace_bytes
nx_scatter_fwd = lib.nx_scatter_fwd
nx_scatter_fwd_noalloc = lib.nx_scatter_fwd_noalloc
nx_scatter_bwd = lib.nx_scatter_bwd
nx_scatter_fwd_f64 = lib.nx_scatter_fwd_f64
nx_scatter_bwd_f64 = lib.nx_scatter_bwd_f64
nx_loss_grad = lib.nx_loss_grad
nx_fit_step = lib.nx_fit_step
nx_scatter_bwd_ex = lib.nx_scatter_bwd_ex
nx_scatter_bwd_ex_f64 = lib.nx_scatter_bwd_ex_f64
nx_scatter_fwd_species = lib.nx_scatter_fwd_species
nx_scatter_bwd_species = lib.nx_scatter_bwd_species
nx_workspace_bytes_species = lib.nx_workspace_bytes_species
nx_workspace_bytes_grid = lib.nx_workspace_bytes_grid
nx_scatter_fwd_grid = lib.nx_scatter_fwd_grid
nx_scatter_bwd_grid = lib.nx_scatter_bwd_grid
nx_fit_step_grid = lib.nx_fit_step_grid
nx_scatter_fwd_species_grid = lib.nx_scatter_fwd_species_grid
nx_scatter_bwd_species_grid = lib.nx_scatter_bwd_species_grid
nx_workspace_bytes_species_grid = lib.nx_workspace_bytes_species_grid
