"""nx_scatter_fwd_noalloc: the forward for callers that cannot allocate, with its workspace
in the library's static per-GPU scratch, checked through the C ABI against nx_scatter_fwd
(the entry point with a caller-supplied workspace) on two calls in a row, the second one
smaller than the first, and against the references that bound both.  The size check runs
on the host before any HIP call (tested on the CPU)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1010_2641_amd import _lib, api, workloads as wl
from tests import metrics as M


def noalloc(xyz, f, S, mode):
    A = torch.empty(S.shape[0], dtype=torch.complex64, device=S.device)
    stream = torch.cuda.current_stream(S.device).cuda_stream
    rc = _lib.nx_scatter_fwd_noalloc(xyz.data_ptr(), None if f is None else f.data_ptr(), xyz.shape[0],
                                     S.data_ptr(), S.shape[0], torch.view_as_real(A).data_ptr(),
                                     api.MODES[mode], stream)
    _lib.check(rc)
    torch.cuda.synchronize()
    return A


def test_oversized_calls_are_refused_on_the_host():
    fake = 0x10000
    # 2^30 atoms need 48 GiB of atom records: far beyond the 128 MiB scratch
    rc = _lib.nx_scatter_fwd_noalloc(fake, None, 1 << 30, fake, 1000, fake, 1, None)
    assert rc == _lib.NX_ERR_WORKSPACE
    msg = _lib.last_error()
    assert "nx_scatter_fwd_noalloc" in msg and str(_lib.NX_NOALLOC_SCRATCH_BYTES) in msg
    assert _lib.nx_scatter_fwd_noalloc(fake, None, -1, fake, 10, fake, 1, None) == _lib.NX_ERR_ARG
    assert _lib.nx_scatter_fwd_noalloc(fake, None, 10, fake, 10, fake, 5, None) == _lib.NX_ERR_MODE
    assert _lib.nx_scatter_fwd_noalloc(fake, None, 10, None, 10, fake, 1, None) == _lib.NX_ERR_ARG
    assert _lib.nx_scatter_fwd_noalloc(None, None, 10, None, 0, None, 1, None) == _lib.NX_OK


@pytest.mark.gpu
def test_two_calls_against_the_workspace_forward():
    dev = torch.device("cuda:0")
    # first call: the 1e6-atom cube over 65,536 points, whose usual plan (256 stream
    # slices, 316 MB of workspace) does not fit the scratch, so the call runs with fewer
    # slices; held to T1/T2 against the all-FP64 path on every point, like the usual plan
    w = wl.c3()
    print(f"no-alloc call 1: {w.n_atoms} atoms x {w.n_points} points (fewer slices)", flush=True)
    tx, tS = torch.from_numpy(w.xyz).to(dev), torch.from_numpy(w.S).to(dev)
    A_na = noalloc(tx, None, tS, "ph64").cpu().numpy().astype(np.complex128)
    A_ws = api.scatter_fwd(tx, None, tS, "ph64").cpu().numpy().astype(np.complex128)
    A64 = api.scatter_fwd_f64(tx.double(), None, tS.double()).cpu().numpy()
    e_na, e_ws = (M.t1(A_na, A64), M.t2(A_na, A64)), (M.t1(A_ws, A64), M.t2(A_ws, A64))
    print(f"  no-alloc vs f64 path: T1={e_na[0]:.3e} T2={e_na[1]:.3e}; "
          f"workspace forward: T1={e_ws[0]:.3e} T2={e_ws[1]:.3e}", flush=True)
    assert e_na[0] <= M.T1_TOL and e_na[1] <= M.T2_TOL
    assert M.t1(A_na, A_ws) <= 2 * M.T1_TOL and M.t2(A_na, A_ws) <= 2 * M.T2_TOL
    del tx, tS
    # second call, smaller, complex f: the usual plan fits, so the result is bitwise that
    # of nx_scatter_fwd, and within the random-position tolerance of the oracle
    xyz, f, S = wl.random_problem(3001, 5003, seed=77, extent=30.0, s_range=3.0)
    print("no-alloc call 2: 3001 atoms x 5003 points, complex f", flush=True)
    tx, tf, tS = (torch.from_numpy(a).to(dev) for a in (xyz, f, S))
    for mode in ("ph64", "f32"):
        a_na = noalloc(tx, tf, tS, mode)
        a_ws = api.scatter_fwd(tx, tf, tS, mode)
        torch.cuda.synchronize()
        assert torch.equal(a_na, a_ws), mode
    A_ref = oracle.forward(xyz, f, S)
    a = noalloc(tx, tf, tS, "ph64").cpu().numpy()
    inc = M.incoherent(a, A_ref, f, xyz.shape[0])
    print(f"  no-alloc vs oracle: pointwise/sqrt(sum|f|^2)={inc:.3e} T2={M.t2(a, A_ref):.3e}", flush=True)
    assert inc <= M.INC_TOL and M.t2(a, A_ref) <= M.T2_TOL
