"""ctypes binding of libnx_micro (include/nx_micro.h) and the issue ceilings it measures.

Each microbenchmark kernel repeats the per-pair instruction sequence of one of libnx's
sums on register operands only; its rate in pairs per second is the VALU issue ceiling
of that instruction mix on the chip, at the clock the chip runs under such a load.  The
benchmark divides a sum's measured pairs per second by the ceiling of its own mix (the
fraction of the issue rate the sum reaches for its necessary work), beside the paper's
flop count of 8 per pair (Section 2.2) against the FP32 peak."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnx_micro.so")

# (mode, sum, factor kind) -> mix id of include/nx_micro.h
MIXES = {
    ("ph64", "fwd", "complex"): 0, ("ph64", "fwd", "unit"): 1,
    ("ph64", "bwd", "complex"): 2, ("ph64", "bwd", "unit"): 3,
    ("f32", "fwd", "complex"): 4, ("f32", "fwd", "unit"): 5,
    ("f32", "bwd", "complex"): 6, ("f32", "bwd", "unit"): 7,
}

SIGNATURES = {
    "nxm_pairs_per_lane_iter": ([ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "nxm_threads_per_block": ([], ctypes.c_int),
    "nxm_run": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p],
                ctypes.c_int),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1010_2641_amd.build`")
    import torch  # noqa: F401  (torch's HIP runtime first, as for libnx)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()

nxm_pairs_per_lane_iter = lib.nxm_pairs_per_lane_iter
nxm_threads_per_block = lib.nxm_threads_per_block
nxm_run = lib.nxm_run


def mix_rate(mode: str, op: str, fkind: str, n_blocks: int = 8192, iters: int = 2048,
             reps: int = 3) -> float:
    """Pairs per second of the (mode, op, fkind) instruction mix: the best of `reps` timed
    launches of each of the two kernel shapes after one warm-up each, timed with events on
    the current stream."""
    import torch
    mix = MIXES[(mode, op, fkind)]
    threads = nxm_threads_per_block()
    out = torch.empty(n_blocks * threads, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    best = 0.0
    for wide in (0, 1):
        it = iters if not wide else iters // 2
        pairs = float(n_blocks) * threads * it * nxm_pairs_per_lane_iter(mix, wide)
        for r in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rc = nxm_run(mix, wide, n_blocks, it, out.data_ptr(), stream.cuda_stream)
            e1.record(stream)
            if rc != 0:
                raise RuntimeError(f"nxm_run({mix}, {wide}) returned {rc}")
            e1.synchronize()
            if r > 0:
                best = max(best, pairs / (e0.elapsed_time(e1) / 1e3))
    return best
