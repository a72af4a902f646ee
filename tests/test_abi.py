"""The C ABI on the CPU: the library loads without a GPU, exports every entry point
include/nx.h declares, and rejects invalid arguments on the host, before any HIP
call, with the documented status codes and a message.  No compute call is made here
(the pointers below are never dereferenced: validation fails first)."""
import ctypes
import os
import re

import pytest

from paper_1010_2641_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nx.h")

FAKE = 0x10000          # a non-NULL, well-aligned address that validation never reaches


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nx_\w+)\s*\(", text)))


def test_header_symbols_exported():
    names = declared_functions()
    assert "nx_scatter_fwd" in names and "nx_scatter_bwd" in names
    for name in names:
        assert hasattr(_lib.lib, name), f"libnx.so does not export {name}"
        assert name in _lib.SIGNATURES, f"binding has no signature for {name}"
    assert sorted(_lib.SIGNATURES) == names


def test_micro_header_symbols_exported():
    """libnx_micro (the issue-ceiling microbenchmarks) exports what nx_micro.h declares and
    refuses bad arguments before launching anything."""
    from paper_1010_2641_amd import micro
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "nx_micro.h")).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(nxm_\w+)\s*\(", text)))
    assert names == sorted(micro.SIGNATURES)
    for name in names:
        assert hasattr(micro.lib, name)
    assert micro.nxm_threads_per_block() == 256
    assert micro.nxm_pairs_per_lane_iter(0, 0) == 4 and micro.nxm_pairs_per_lane_iter(4, 0) == 8
    assert micro.nxm_pairs_per_lane_iter(0, 1) == 8 and micro.nxm_pairs_per_lane_iter(4, 1) == 16
    assert micro.nxm_pairs_per_lane_iter(8, 0) == 32 and micro.nxm_pairs_per_lane_iter(10, 1) == 64
    assert micro.nxm_run(99, 0, 1, 1, FAKE, None, None) == -2
    assert micro.nxm_run(0, 0, 0, 1, FAKE, None, None) == -1
    assert micro.nxm_run(0, 0, 1, 1, None, None, None) == -1
    assert micro.nxm_run(0, 3, 1, 1, FAKE, None, None) == -1
    # the sums' shape exists for the FP64-phase mixes only: refused before any launch
    assert micro.nxm_pairs_per_lane_iter(0, 2) == 16 and micro.nxm_pairs_per_lane_iter(2, 2) == 32
    assert micro.nxm_pairs_per_lane_iter(4, 2) == 0 and micro.nxm_pairs_per_lane_iter(8, 2) == 0
    assert micro.nxm_pairs_per_lane_iter(0, 3) == 0
    assert micro.nxm_run(4, 2, 1, 1, FAKE, None, None) == -1
    assert micro.nxm_run(8, 2, 1, 1, FAKE, None, None) == -1
    # the mixes of the sums over grid rows: the sums' shape only
    assert micro.nxm_pairs_per_lane_iter(21, 2) == 16 and micro.nxm_pairs_per_lane_iter(24, 2) == 128
    assert micro.nxm_pairs_per_lane_iter(21, 0) == 0 and micro.nxm_pairs_per_lane_iter(23, 1) == 0
    assert micro.nxm_run(22, 0, 1, 1, FAKE, None, None) == -1
    assert micro.nxm_run(25, 2, 1, 1, FAKE, None, None) == -2
    assert micro.nxm_pairs_per_lane_iter(25, 2) == 0


def test_version():
    assert _lib.nx_version() == 104


def fwd(n_atoms=8, n_points=8, xyz=FAKE, f=None, S=FAKE, A=FAKE, mode=1, ws=FAKE, wsb=1 << 40):
    return _lib.nx_scatter_fwd(xyz, f, n_atoms, S, n_points, A, mode, ws, wsb, None)


def bwd(n_atoms=8, n_points=8, xyz=FAKE, f=None, S=FAKE, G=FAKE, g=FAKE, mode=1, ws=FAKE, wsb=1 << 40):
    return _lib.nx_scatter_bwd(xyz, f, n_atoms, S, n_points, G, g, mode, ws, wsb, None)


def test_negative_and_oversized_counts():
    assert fwd(n_atoms=-1) == _lib.NX_ERR_ARG
    assert "negative" in _lib.last_error()
    assert fwd(n_points=-5) == _lib.NX_ERR_ARG
    assert fwd(n_points=_lib.NX_MAX_COUNT + 1) == _lib.NX_ERR_ARG
    assert "NX_MAX_COUNT" in _lib.last_error()
    assert bwd(n_atoms=-1) == _lib.NX_ERR_ARG
    assert _lib.nx_scatter_fwd_f64(FAKE, None, -1, FAKE, 4, FAKE, FAKE, 1 << 40, None) == _lib.NX_ERR_ARG
    assert _lib.nx_scatter_bwd_f64(FAKE, None, 4, FAKE, -1, FAKE, FAKE, FAKE, 1 << 40, None) == _lib.NX_ERR_ARG
    assert _lib.nx_loss_grad(FAKE, FAKE, -3, FAKE, FAKE, FAKE, 1 << 40, None) == _lib.NX_ERR_ARG


def test_null_pointers():
    assert fwd(S=None) == _lib.NX_ERR_ARG
    assert "NULL" in _lib.last_error()
    assert fwd(A=None) == _lib.NX_ERR_ARG
    assert fwd(xyz=None) == _lib.NX_ERR_ARG
    assert bwd(G=None) == _lib.NX_ERR_ARG
    assert bwd(g=None) == _lib.NX_ERR_ARG
    assert _lib.nx_loss_grad(FAKE, None, 4, FAKE, FAKE, FAKE, 1 << 40, None) == _lib.NX_ERR_ARG
    assert _lib.nx_loss_grad(FAKE, FAKE, 4, None, FAKE, FAKE, 1 << 40, None) == _lib.NX_ERR_ARG


def test_unknown_mode():
    assert fwd(mode=7) == _lib.NX_ERR_MODE
    assert "mode" in _lib.last_error()
    assert bwd(mode=-1) == _lib.NX_ERR_MODE
    assert _lib.nx_workspace_bytes(4, 4, 3, _lib.NX_OP_FWD, 0) == 0
    assert "mode" in _lib.last_error()
    assert _lib.nx_workspace_bytes(4, 4, 1, 9, 0) == 0
    assert "op" in _lib.last_error()


def test_misaligned():
    assert fwd(A=FAKE + 4) == _lib.NX_ERR_ARG
    assert fwd(f=FAKE + 2) == _lib.NX_ERR_ARG
    assert _lib.nx_scatter_fwd_f64(FAKE, None, 4, FAKE, 4, FAKE + 8, FAKE, 1 << 40, None) == _lib.NX_ERR_ARG


def test_workspace_checks():
    need = _lib.nx_workspace_bytes(4096, 4096, 1, _lib.NX_OP_FWD, 1)
    assert need >= 4096 * 32          # packed FP64-phase atom records
    assert fwd(n_atoms=4096, n_points=4096, wsb=need - 1) == _lib.NX_ERR_WORKSPACE
    assert "workspace" in _lib.last_error()
    assert fwd(n_atoms=4096, n_points=4096, ws=None, wsb=need) == _lib.NX_ERR_WORKSPACE
    assert fwd(n_atoms=4096, n_points=4096, ws=FAKE + 8, wsb=need) == _lib.NX_ERR_WORKSPACE
    # loss workspace is a fixed small scratch
    lw = _lib.nx_workspace_bytes(0, 10, 0, _lib.NX_OP_LOSS, 1)
    assert 0 < lw <= 1 << 16
    assert _lib.nx_loss_grad(FAKE, FAKE, 10, FAKE, FAKE, FAKE, lw - 8, None) == _lib.NX_ERR_WORKSPACE


def test_workspace_sizes_scale():
    # split partials appear when there are few points; packed records always
    small_k = _lib.nx_workspace_bytes(1_000_000, 65_536, 1, _lib.NX_OP_FWD, 1)
    assert small_k > 1_000_000 * 32
    big_k = _lib.nx_workspace_bytes(203_557, 2_097_152, 1, _lib.NX_OP_FWD, 0)
    assert big_k >= 203_557 * 32
    f64 = _lib.nx_workspace_bytes(1000, 1000, 0, _lib.NX_OP_FWD_F64, 0)
    assert f64 >= 1000 * 48
    b = _lib.nx_workspace_bytes(97_556, 262_144, 1, _lib.NX_OP_BWD, 1)
    assert b >= 262_144 * 48


def test_empty_calls_queue_nothing():
    # n_points == 0 forward and n_atoms == 0 adjoint return OK before any HIP call
    assert fwd(n_points=0, xyz=None, S=None, A=None, ws=None, wsb=0) == _lib.NX_OK
    assert _lib.last_error() == ""
    assert bwd(n_atoms=0, xyz=None, S=None, G=None, g=None, ws=None, wsb=0) == _lib.NX_OK
    assert _lib.nx_scatter_fwd_f64(None, None, 5, None, 0, None, None, 0, None) == _lib.NX_OK
    assert _lib.nx_scatter_bwd_f64(None, None, 0, None, 5, None, None, None, 0, None) == _lib.NX_OK


def test_python_wrappers_refuse_cpu_tensors():
    torch = pytest.importorskip("torch")
    from paper_1010_2641_amd import api
    x = torch.zeros((4, 3), dtype=torch.float32)
    with pytest.raises(ValueError, match="GPU"):
        api.scatter_fwd(x, None, x)
    with pytest.raises(ValueError, match="unknown mode"):
        api._mode("fp16")


def test_fit_step_checks_before_queueing():
    """nx_fit_step checks what its three stages check before queueing any of them."""
    fit = lambda n=8, k=8, xyz=FAKE, S=FAKE, I=FAKE, A=FAKE, L=FAKE, G=FAKE, g=FAKE, mode=1, ws=FAKE, \
        wsb=1 << 40: _lib.nx_fit_step(xyz, None, n, S, k, I, A, L, G, g, mode, ws, wsb, None)
    assert fit(n=-1) == _lib.NX_ERR_ARG
    assert fit(mode=9) == _lib.NX_ERR_MODE
    for kw in ("S", "I", "A", "L", "G", "g", "xyz"):
        assert fit(**{kw: None}) == _lib.NX_ERR_ARG, kw
        assert "nx_fit_step" in _lib.last_error()
    assert fit(A=FAKE + 4) == _lib.NX_ERR_ARG
    need = _lib.nx_workspace_bytes(1000, 3000, 1, _lib.NX_OP_FIT, 1)
    assert need >= max(_lib.nx_workspace_bytes(1000, 3000, 1, op, 1)
                       for op in (_lib.NX_OP_FWD, _lib.NX_OP_BWD, _lib.NX_OP_LOSS))
    assert fit(n=1000, k=3000, wsb=need - 1) == _lib.NX_ERR_WORKSPACE
    assert fit(n=1000, k=3000, ws=None) == _lib.NX_ERR_WORKSPACE


def test_single_hip_runtime():
    """libnx must bind to the HIP runtime torch brought in, never a second copy."""
    assert len(_lib._hip_runtimes()) == 1


def starts(*v):
    return (ctypes.c_int64 * len(v))(*v)


def fwd_sp(start, ns, n_atoms=8, n_points=8, xyz=FAKE, fs=None, S=FAKE, A=FAKE, As=None, mode=1,
           ws=FAKE, wsb=1 << 40):
    return _lib.nx_scatter_fwd_species(xyz, n_atoms, start, ns, fs, S, n_points, A, As, mode, ws, wsb,
                                       None)


def test_species_partition_checks():
    assert fwd_sp(starts(0, 3, 8), 2, wsb=0) == _lib.NX_ERR_WORKSPACE   # valid partition
    assert fwd_sp(None, 2) == _lib.NX_ERR_ARG
    assert "species_start" in _lib.last_error()
    assert fwd_sp(starts(1, 3, 8), 2) == _lib.NX_ERR_ARG           # must start at 0
    assert fwd_sp(starts(0, 3, 7), 2) == _lib.NX_ERR_ARG           # must end at n_atoms
    assert fwd_sp(starts(0, 5, 3, 8), 3) == _lib.NX_ERR_ARG        # decreasing
    assert "decreases" in _lib.last_error()
    assert fwd_sp(starts(0, 8), 0) == _lib.NX_ERR_ARG
    assert fwd_sp(starts(*range(0, 18)), 17, n_atoms=17) == _lib.NX_ERR_ARG
    assert "n_species" in _lib.last_error()
    assert fwd_sp(starts(0, 8), 1, mode=5) == _lib.NX_ERR_MODE
    g = _lib.nx_scatter_bwd_species
    assert g(FAKE, 8, starts(0, 9), 1, None, FAKE, 8, FAKE, None, FAKE, None, 1, FAKE, 1 << 40,
             None) == _lib.NX_ERR_ARG
    # the factor gradient needs the per-species sums
    assert g(FAKE, 8, starts(0, 8), 1, None, FAKE, 8, FAKE, None, None, FAKE, 1, FAKE, 1 << 40,
             None) == _lib.NX_ERR_ARG
    assert "A_species" in _lib.last_error()
    # neither gradient asked for: nothing to do
    assert g(FAKE, 8, starts(0, 8), 1, None, FAKE, 8, FAKE, None, None, None, 1, None, 0,
             None) == _lib.NX_OK


def test_species_workspace():
    ws1 = _lib.nx_workspace_bytes_species(starts(0, 100_000, 203_557), 2, 2_097_152, 1, 0)
    # all atom records, then one (sum, comp) state of 16 bytes per point and species
    assert ws1 >= 203_557 * 32 + 2 * 2_097_152 * 16
    ws0 = _lib.nx_workspace_bytes_species(starts(0, 100_000, 203_557), 2, 2_097_152, 1, 1)
    assert ws0 >= 2_097_152 * (8 + 48)       # per-species seed and the point records
    assert _lib.nx_workspace_bytes_species(starts(0, 4), 1, 8, 1, 2) == 0
    assert "op" in _lib.last_error()
    assert _lib.nx_workspace_bytes_species(starts(0, 4), 1, 8, 9, 0) == 0
    assert "mode" in _lib.last_error()
    assert fwd_sp(starts(0, 4096), 1, n_atoms=4096, n_points=4096, wsb=100) == _lib.NX_ERR_WORKSPACE


def test_species_and_factor_gradient_empty_calls():
    assert fwd_sp(starts(0, 8), 1, n_points=0, xyz=None, S=None, A=None, ws=None, wsb=0) == _lib.NX_OK
    assert _lib.nx_scatter_bwd_ex(None, None, 0, None, 5, None, None, FAKE, 1, None, 0, None) == _lib.NX_OK
    assert _lib.nx_scatter_bwd_ex(FAKE, None, 4, FAKE, 5, FAKE, None, FAKE + 4, 1, FAKE, 1 << 40,
                                  None) == _lib.NX_ERR_ARG
    assert _lib.nx_scatter_bwd_ex(FAKE, None, 4, FAKE, 5, FAKE, None, FAKE, 6, FAKE, 1 << 40,
                                  None) == _lib.NX_ERR_MODE
    need = _lib.nx_workspace_bytes(1000, 1000, 1, _lib.NX_OP_BWD_GF, 0)
    assert need > _lib.nx_workspace_bytes(1000, 1000, 1, _lib.NX_OP_BWD, 0)   # two more sums
    assert _lib.nx_scatter_bwd_ex(FAKE, FAKE, 1000, FAKE, 1000, FAKE, FAKE, FAKE, 1, FAKE, need - 1,
                                  None) == _lib.NX_ERR_WORKSPACE


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/libnx.so")
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _lib._load()


def test_plan_l2_sized_forward_chunks(monkeypatch):
    """The forward cuts its launches when a split's slice of atom records exceeds an
    XCD's L2: the carried running sums then appear in the workspace (host-side plan)."""
    monkeypatch.setenv("NX_TUNE_TARGET_BLOCKS", "4096")   # one split at this size
    n, k = 203_557, 2_097_152                                 # 48-byte FP64-phase records
    rec = -(-n * 48 // 256) * 256
    for f_is_null in (0, 1):
        with_chunks = _lib.nx_workspace_bytes(n, k, 1, _lib.NX_OP_FWD, f_is_null)
        assert with_chunks == rec + k * 16         # one (sum, comp) state per point
    monkeypatch.setenv("NX_TUNE_L2_CHUNK", "0")
    assert _lib.nx_workspace_bytes(n, k, 1, _lib.NX_OP_FWD, 0) == rec
    monkeypatch.delenv("NX_TUNE_L2_CHUNK")
    # slices that fit the L2 are not cut: 80,000 records of 48 bytes
    assert _lib.nx_workspace_bytes(80_000, k, 1, _lib.NX_OP_FWD, 0) == -(-80_000 * 48 // 256) * 256
    # the FP32 mode's records are 32 bytes: 120,000 of them fit
    assert _lib.nx_workspace_bytes(120_000, k, 0, _lib.NX_OP_FWD, 1) == -(-120_000 * 32 // 256) * 256


def test_plan_launch_chunks_and_splits(monkeypatch):
    # few points: the atoms are split across work-groups, with one state per split
    few = _lib.nx_workspace_bytes(1_000_000, 65_536, 1, _lib.NX_OP_FWD, 1)
    assert few > 1_000_000 * 32 + 65_536 * 16
    # enough points for the target number of work-groups: no split, no carried state ...
    monkeypatch.setenv("NX_TUNE_TARGET_BLOCKS", "4096")
    n, k = 5000, 1 << 20
    rec = -(-n * 48 // 256) * 256
    assert _lib.nx_workspace_bytes(n, k, 1, _lib.NX_OP_FWD, 1) == rec
    # ... until a small launch size forces chunks, which carry one state per point
    monkeypatch.setenv("NX_TUNE_LAUNCH_PAIRS", str(1 << 24))
    assert _lib.nx_workspace_bytes(n, k, 1, _lib.NX_OP_FWD, 1) == rec + k * 16


def test_plan_stream_splits_for_the_target_block_count(monkeypatch):
    """The adjoint of a 203,557-atom, 2,097,152-point fit: 398 work-groups of 512 atoms are
    too few, so the points are cut into ceil(32768 / 398) = 83 slices, each with its own
    (sum, comp) state of the 3 position sums per atom (24 bytes).  The 48-byte point records
    are followed by one float per 256 points (the tiles' bound of the fixed-point phase
    reduction)."""
    n, k = 203_557, 2_097_152
    rec = -(-k * 48 // 256) * 256 + -(-(-(-k // 256)) * 4 // 256) * 256
    part = -(-83 * n * 24 // 256) * 256
    assert _lib.nx_workspace_bytes(n, k, 1, _lib.NX_OP_BWD, 0) == rec + part
    monkeypatch.setenv("NX_TUNE_TARGET_BLOCKS", "4096")              # ceil(4096 / 398) = 11
    assert _lib.nx_workspace_bytes(n, k, 1, _lib.NX_OP_BWD, 0) == rec + -(-11 * n * 24 // 256) * 256


def test_plan_stream_slices_are_at_least_256_items(monkeypatch):
    """Splits stop at slices of 256 stream items: a 100,000-atom forward over 10,000 points
    (40 work-groups) would want ceil(32768 / 40) = 820 slices, and gets 100000 // 256 =
    390, each with one (sum, comp) float4 per point.  Only when such slices leave fewer
    than 1,024 work-groups (4 waves per SIMD) may they shrink to 32 items: 1,000 atoms over
    1,000 points (4 work-groups of points) get 1000 // 32 = 31 slices instead of 3, and the
    4,096 x 4,096 block (16 work-groups) 64 slices of 64 atoms instead of 16."""
    monkeypatch.delenv("NX_TUNE_TARGET_BLOCKS", raising=False)
    rec = 100_000 * 48
    assert _lib.nx_workspace_bytes(100_000, 10_000, 1, _lib.NX_OP_FWD, 1) == rec + 390 * 10_000 * 16
    a256 = lambda b: -(-b // 256) * 256
    assert _lib.nx_workspace_bytes(1000, 1000, 1, _lib.NX_OP_FWD, 1) == a256(1000 * 48) + a256(31 * 1000 * 16)
    # the FP32 mode's 32-byte records, same slices
    assert _lib.nx_workspace_bytes(1000, 1000, 0, _lib.NX_OP_FWD, 1) == a256(1000 * 32) + a256(31 * 1000 * 16)
    assert _lib.nx_workspace_bytes(4096, 4096, 1, _lib.NX_OP_FWD, 1) == a256(4096 * 48) + a256(64 * 4096 * 16)
    # a small target keeps the small grid (the knob the launch-shape tests use)
    monkeypatch.setenv("NX_TUNE_TARGET_BLOCKS", "12")
    assert _lib.nx_workspace_bytes(1000, 1000, 1, _lib.NX_OP_FWD, 1) == a256(1000 * 48) + a256(3 * 1000 * 16)


def grid_struct(n1=64, n2=2, n3=3, origin=(3.95, -0.05, 3.95), step=1e-3):
    g = _lib.nx_grid()
    g.origin[:] = origin
    g.step1[:] = (step, 0.0, 0.0)
    g.step2[:] = (0.0, step, 0.0)
    g.step3[:] = (0.0, 0.0, step)
    g.n1, g.n2, g.n3 = n1, n2, n3
    return g


def fwd_grid(g, n_atoms=8, xyz=FAKE, f=None, A=FAKE, mode=1, ws=FAKE, wsb=1 << 40):
    return _lib.nx_scatter_fwd_grid(xyz, f, n_atoms, ctypes.byref(g) if g is not None else None, A,
                                    mode, ws, wsb, None)


def bwd_grid(g, n_atoms=8, xyz=FAKE, f=None, G=FAKE, grad=FAKE, mode=1, ws=FAKE, wsb=1 << 40):
    return _lib.nx_scatter_bwd_grid(xyz, f, n_atoms, ctypes.byref(g) if g is not None else None, G,
                                    grad, mode, ws, wsb, None)


def test_grid_struct_layout():
    """struct nx_grid: 12 doubles, then three int64 counts (120 bytes)."""
    assert ctypes.sizeof(_lib.nx_grid) == 120
    assert _lib.nx_grid.n1.offset == 96 and _lib.nx_grid.n3.offset == 112


def test_grid_argument_checks():
    assert fwd_grid(None) == _lib.NX_ERR_ARG and "NULL grid" in _lib.last_error()
    assert bwd_grid(None) == _lib.NX_ERR_ARG
    assert fwd_grid(grid_struct(n2=-1)) == _lib.NX_ERR_ARG and "n2" in _lib.last_error()
    assert fwd_grid(grid_struct(n1=1 << 11, n2=1 << 10, n3=1 << 10)) == _lib.NX_ERR_ARG
    assert "exceeds" in _lib.last_error()
    assert fwd_grid(grid_struct(n1=1 << 40)) == _lib.NX_ERR_ARG
    assert fwd_grid(grid_struct(origin=(float("nan"), 0.0, 0.0))) == _lib.NX_ERR_ARG
    assert "finite" in _lib.last_error()
    g = grid_struct()
    g.step3[2] = float("inf")
    assert bwd_grid(g) == _lib.NX_ERR_ARG
    # FP64-phase mode only
    assert fwd_grid(grid_struct(), mode=0) == _lib.NX_ERR_MODE and "NX_F32_PH64" in _lib.last_error()
    assert bwd_grid(grid_struct(), mode=0) == _lib.NX_ERR_MODE
    # NULL pointers and alignment
    assert fwd_grid(grid_struct(), A=None) == _lib.NX_ERR_ARG
    assert fwd_grid(grid_struct(), xyz=None) == _lib.NX_ERR_ARG
    assert bwd_grid(grid_struct(), G=None) == _lib.NX_ERR_ARG
    assert bwd_grid(grid_struct(), grad=None) == _lib.NX_ERR_ARG
    assert fwd_grid(grid_struct(), A=FAKE + 4) == _lib.NX_ERR_ARG
    assert fwd_grid(grid_struct(), f=FAKE + 4) == _lib.NX_ERR_ARG
    # workspace too small or missing
    assert fwd_grid(grid_struct(), ws=None, wsb=0) == _lib.NX_ERR_WORKSPACE
    assert bwd_grid(grid_struct(), wsb=16) == _lib.NX_ERR_WORKSPACE
    assert fwd_grid(grid_struct(), n_atoms=-1) == _lib.NX_ERR_ARG


def test_grid_empty_calls_queue_nothing():
    """An empty grid forward and a zero-atom adjoint return before any launch."""
    assert fwd_grid(grid_struct(n3=0), A=None, xyz=None, ws=None, wsb=0) == _lib.NX_OK
    assert bwd_grid(grid_struct(), n_atoms=0, xyz=None, grad=None, G=None, ws=None, wsb=0) == _lib.NX_OK


def test_grid_fit_step_checks_before_queueing():
    g = grid_struct()
    args = lambda **kw: [kw.get("xyz", FAKE), None, 8, ctypes.byref(g), kw.get("I", FAKE), kw.get("A", FAKE),
                         kw.get("L", FAKE), kw.get("G", FAKE), kw.get("grad", FAKE), kw.get("mode", 1),
                         kw.get("ws", FAKE), kw.get("wsb", 1 << 40), None]
    assert _lib.nx_fit_step_grid(*args(L=None)) == _lib.NX_ERR_ARG
    assert _lib.nx_fit_step_grid(*args(I=None)) == _lib.NX_ERR_ARG
    assert _lib.nx_fit_step_grid(*args(mode=0)) == _lib.NX_ERR_MODE
    assert _lib.nx_fit_step_grid(*args(L=FAKE + 4)) == _lib.NX_ERR_ARG
    assert _lib.nx_fit_step_grid(*args(ws=None, wsb=0)) == _lib.NX_ERR_WORKSPACE
    # the step's workspace covers its three stages
    fit = _lib.nx_workspace_bytes_grid(8, ctypes.byref(g), _lib.NX_OP_FIT, 1)
    stages = [_lib.nx_workspace_bytes_grid(8, ctypes.byref(g), op, 1) for op in (_lib.NX_OP_FWD, _lib.NX_OP_BWD)]
    stages.append(_lib.nx_workspace_bytes(0, 384, 1, _lib.NX_OP_LOSS, 1))
    assert fit == max(stages)


def test_grid_workspace(monkeypatch):
    """Rows of a multiple of 64 points: 80-byte atom records (forward); 16-byte point
    records (the seed and the point's place in its 64-point group) and one 16-byte record
    per group (its first point; adjoint), followed as in the point-list calls by the
    tiles' bounds; other grids take the point-list records (48 B).  Unknown ops are
    refused."""
    monkeypatch.delenv("NX_TUNE_GRID", raising=False)
    a256 = lambda b: -(-b // 256) * 256
    g = grid_struct(n1=128, n2=128, n3=128)          # 2,097,152 points
    n, k = 203_557, 128 ** 3
    bwd_rows = _lib.nx_workspace_bytes_grid(n, ctypes.byref(g), _lib.NX_OP_BWD, 0)
    bwd_list = _lib.nx_workspace_bytes(n, k, 1, _lib.NX_OP_BWD, 0)
    assert bwd_list - bwd_rows == a256(k * 48) - a256(k * 16) - a256(k // 64 * 16)
    # the forward: 2 x 2 x 2 blocks of points per lane
    fw = _lib.nx_workspace_bytes_grid(n, ctypes.byref(g), _lib.NX_OP_FWD, 0)
    assert fw % 256 == 0 and fw >= a256(n * 80)
    # a row of 50 points takes the general kernels and their records
    g50 = grid_struct(n1=50, n2=40, n3=3)
    assert (_lib.nx_workspace_bytes_grid(1000, ctypes.byref(g50), _lib.NX_OP_BWD, 1)
            == _lib.nx_workspace_bytes(1000, 6000, 1, _lib.NX_OP_BWD, 1))
    # the forward over rows takes 80-byte atom records (with the three steps), also for few
    # atoms (8-atom groups), against 48 bytes for the point-list kernels
    small = grid_struct(n1=256, n2=3, n3=2)
    rows_fw = _lib.nx_workspace_bytes_grid(5000, ctypes.byref(small), _lib.NX_OP_FWD, 0)
    # and every grid takes the point-list kernels under NX_TUNE_GRID=1
    monkeypatch.setenv("NX_TUNE_GRID", "1")
    list_fw = _lib.nx_workspace_bytes_grid(5000, ctypes.byref(small), _lib.NX_OP_FWD, 0)
    assert rows_fw - list_fw == a256(5000 * 80) - a256(5000 * 48)
    assert _lib.nx_workspace_bytes_grid(n, ctypes.byref(g), _lib.NX_OP_BWD, 0) == bwd_list
    assert _lib.nx_workspace_bytes_grid(8, ctypes.byref(g), 3, 1) == 0
    assert "op must be" in _lib.last_error()
    assert _lib.nx_workspace_bytes_grid(8, None, _lib.NX_OP_FWD, 1) == 0


def fwd_sp_grid(g, start, ns, n_atoms=8, xyz=FAKE, fs=None, A=FAKE, As=None, mode=1, ws=FAKE,
                wsb=1 << 40):
    return _lib.nx_scatter_fwd_species_grid(xyz, n_atoms, start, ns, fs,
                                            ctypes.byref(g) if g is not None else None, A, As, mode,
                                            ws, wsb, None)


def bwd_sp_grid(g, start, ns, n_atoms=8, xyz=FAKE, fs=None, G=FAKE, As=None, grad=FAKE, gfs=None,
                mode=1, ws=FAKE, wsb=1 << 40):
    return _lib.nx_scatter_bwd_species_grid(xyz, n_atoms, start, ns, fs,
                                            ctypes.byref(g) if g is not None else None, G, As, grad,
                                            gfs, mode, ws, wsb, None)


def test_species_grid_argument_checks():
    """The species-factorised calls over a grid check the grid, the partition, the mode,
    pointers, alignment and workspace before queueing anything."""
    g = grid_struct()
    assert fwd_sp_grid(None, starts(0, 8), 1) == _lib.NX_ERR_ARG and "NULL grid" in _lib.last_error()
    assert bwd_sp_grid(None, starts(0, 8), 1) == _lib.NX_ERR_ARG
    assert fwd_sp_grid(grid_struct(n1=-2), starts(0, 8), 1) == _lib.NX_ERR_ARG
    assert fwd_sp_grid(g, starts(0, 3, 7), 2) == _lib.NX_ERR_ARG            # must end at n_atoms
    assert fwd_sp_grid(g, starts(0, 5, 3, 8), 3) == _lib.NX_ERR_ARG         # decreasing
    assert "decreases" in _lib.last_error()
    assert fwd_sp_grid(g, starts(*range(0, 18)), 17, n_atoms=17) == _lib.NX_ERR_ARG
    assert fwd_sp_grid(g, starts(0, 8), 1, mode=0) == _lib.NX_ERR_MODE
    assert "NX_F32_PH64" in _lib.last_error()
    assert bwd_sp_grid(g, starts(0, 8), 1, mode=0) == _lib.NX_ERR_MODE
    assert fwd_sp_grid(g, starts(0, 8), 1, A=None) == _lib.NX_ERR_ARG
    assert fwd_sp_grid(g, starts(0, 8), 1, xyz=None) == _lib.NX_ERR_ARG
    assert fwd_sp_grid(g, starts(0, 8), 1, A=FAKE + 4) == _lib.NX_ERR_ARG
    assert fwd_sp_grid(g, starts(0, 8), 1, As=FAKE + 4) == _lib.NX_ERR_ARG
    assert fwd_sp_grid(g, starts(0, 3, 8), 2, wsb=0) == _lib.NX_ERR_WORKSPACE
    assert bwd_sp_grid(g, starts(0, 8), 1, G=None) == _lib.NX_ERR_ARG
    assert bwd_sp_grid(g, starts(0, 8), 1, xyz=None) == _lib.NX_ERR_ARG
    assert bwd_sp_grid(g, starts(0, 8), 1, grad=None, gfs=FAKE) == _lib.NX_ERR_ARG   # needs A_species
    assert "A_species" in _lib.last_error()
    assert bwd_sp_grid(g, starts(0, 8), 1, wsb=16) == _lib.NX_ERR_WORKSPACE
    # nothing asked for; an empty grid forward; no atoms
    assert bwd_sp_grid(g, starts(0, 8), 1, grad=None, gfs=None, ws=None, wsb=0) == _lib.NX_OK
    assert fwd_sp_grid(grid_struct(n2=0), starts(0, 8), 1, A=None, xyz=None, ws=None, wsb=0) == _lib.NX_OK
    assert bwd_sp_grid(g, starts(0, 0), 1, n_atoms=0, xyz=None, grad=FAKE, ws=None, wsb=0) == _lib.NX_OK


def test_species_grid_workspace(monkeypatch):
    """Forward: every atom's grid record (80 B over rows), then one 16-byte (sum, comp) state
    per point, split and species; adjoint: the per-species seed (8 B per point), then the
    largest species' grid adjoint workspace."""
    monkeypatch.delenv("NX_TUNE_GRID", raising=False)
    a256 = lambda b: -(-b // 256) * 256
    g = grid_struct(n1=128, n2=128, n3=128)
    k, st = 128 ** 3, starts(0, 100_000, 203_557)
    fw = _lib.nx_workspace_bytes_species_grid(st, 2, ctypes.byref(g), 0)
    assert fw >= a256(203_557 * 80) + 2 * k * 16
    bw = _lib.nx_workspace_bytes_species_grid(st, 2, ctypes.byref(g), 1)
    most = max(_lib.nx_workspace_bytes_grid(n, ctypes.byref(g), _lib.NX_OP_BWD, 1) for n in (100_000, 103_557))
    assert bw == a256(k * 8) + most
    # the point-list species call over the same points needs 48-byte point records
    assert bw < _lib.nx_workspace_bytes_species(st, 2, k, 1, 1)
    assert _lib.nx_workspace_bytes_species_grid(st, 2, ctypes.byref(g), 2) == 0
    assert "op must be" in _lib.last_error()
    assert _lib.nx_workspace_bytes_species_grid(st, 2, None, 0) == 0
    assert _lib.nx_workspace_bytes_species_grid(None, 2, ctypes.byref(g), 0) == 0
    assert fwd_sp_grid(grid_struct(n1=128, n2=2, n3=2), starts(0, 4096), 1, n_atoms=4096,
                       wsb=100) == _lib.NX_ERR_WORKSPACE
