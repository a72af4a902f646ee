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

# single instruction kinds of include/nx_micro.h
OPS = {"fma_f32": 8, "fma_f64": 9, "sin_f32": 10, "fmac_f32": 11, "fmac_f64": 12,
       "add_f64": 13, "rndne_f64": 14, "fract_f64": 15, "cvt_f32_i32": 16, "cos_f32": 17,
       "mul_f32": 18, "fma_f32_v": 19, "add_f32": 20}

# (mode, sum, factor kind) -> mix id of include/nx_micro.h
MIXES = {
    ("ph64", "fwd", "complex"): 0, ("ph64", "fwd", "unit"): 1,
    ("ph64", "bwd", "complex"): 2, ("ph64", "bwd", "unit"): 3,
    ("f32", "fwd", "complex"): 4, ("f32", "fwd", "unit"): 5,
    ("f32", "bwd", "complex"): 6, ("f32", "bwd", "unit"): 7,
    ("grid", "fwd", "complex"): 21, ("grid", "fwd", "unit"): 22,
    ("grid", "bwd", "complex"): 23, ("grid", "bwd", "unit"): 24,
}

SIGNATURES = {
    "nxm_pairs_per_lane_iter": ([ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "nxm_threads_per_block": ([], ctypes.c_int),
    "nxm_wallclock_khz": ([], ctypes.c_int),
    "nxm_run": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                 ctypes.c_void_p], ctypes.c_int),
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
nxm_wallclock_khz = lib.nxm_wallclock_khz
nxm_run = lib.nxm_run


def _rate(mix: int, n_blocks: int, iters: int, reps: int):
    """(best items per second over the kernel shapes, clock in GHz of that launch): `reps`
    timed launches of each shape the mix has after one warm-up, events on the current
    stream; every shape runs about the same number of items per lane."""
    import torch
    threads = nxm_threads_per_block()
    out = torch.empty(n_blocks * threads, dtype=torch.float32, device="cuda")
    clk = torch.zeros(2 * n_blocks, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    khz = nxm_wallclock_khz()
    best, ghz = 0.0, None
    # the pairs per lane of the mix's first shape set the work of every shape
    base = next((b for b in (nxm_pairs_per_lane_iter(mix, w) for w in (0, 1, 2)) if b > 0), 0)
    if base <= 0:
        raise ValueError(f"mix {mix} has no kernel shape")
    for wide in (0, 1, 2):
        per = nxm_pairs_per_lane_iter(mix, wide)
        if per <= 0:
            continue
        it = max(1, iters * base // per)
        items = float(n_blocks) * threads * it * per
        for r in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rc = nxm_run(mix, wide, n_blocks, it, out.data_ptr(), clk.data_ptr(), stream.cuda_stream)
            e1.record(stream)
            if rc != 0:
                raise RuntimeError(f"nxm_run({mix}, {wide}) returned {rc}")
            e1.synchronize()
            rate = items / (e0.elapsed_time(e1) / 1e3)
            if r > 0 and rate > best:
                best = rate
                c = clk.view(-1, 2).double().sum(0)
                ghz = float(c[0] / c[1]) * khz / 1e6 if khz > 0 and c[1] > 0 else None
    return best, ghz


def mix_rate(mode: str, op: str, fkind: str, n_blocks: int = 8192, iters: int = 2048,
             reps: int = 3):
    """(pairs per second, clock in GHz) of the (mode, op, fkind) instruction mix: the
    issue ceiling of that mix, the better of the two kernel shapes."""
    return _rate(MIXES[(mode, op, fkind)], n_blocks, iters, reps)


def op_rate(kind: str, n_blocks: int = 8192, iters: int = 1024, reps: int = 3):
    """(wave64 instructions per second per SIMD, clock in GHz) of one instruction kind
    (see OPS) issued alone; cycles per instruction = clock / that rate."""
    rate, ghz = _rate(OPS[kind], n_blocks, iters, reps)
    return rate / 64.0 / (256 * 4), ghz
