"""The paper's own experiments replayed on the GPU (synthetic inputs): the Section 4.1
cube against its closed form and the oracle, the Fig. 2 chains against the analytic
chain amplitude, and a small run of the Fig. 1 sweep code."""
import numpy as np
import pytest
import torch

import oracle
from paper_1010_2641_amd import api, replay, workloads as wl
from tests import metrics as M

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def test_cube41_plain_against_closed_form():
    w = wl.cube41()
    ref = replay.laue_cube41(w.S)
    A = api.scatter_fwd(dev(w.xyz), None, dev(w.S)).cpu().numpy().astype(np.complex128)
    e1, e2 = M.t1(A, ref), M.t2(A, ref)
    e1b = M.t1(A, ref, floor=1e-5)
    print(f"cube41 plain vs closed form: T1={e1:.3e} (floor 1e-5: {e1b:.3e}) T2={e2:.3e}", flush=True)
    # a perfect lattice is where the hardware sin/cos error would add up coherently
    # (each harmonic of that periodic error like an amplitude at a multiple of S); the
    # groups' eighth turns make it add up incoherently, so the usual bound holds
    assert e1 <= M.T1_TOL and e2 <= M.T2_TOL
    # the closed form itself against the oracle on a few points (the (004) node included)
    node = int(np.argmin(np.abs(w.S[:, 0]) + np.abs(w.S[:, 2] - 4.0)))
    idx = np.array([0, 7777, node, 39999])
    assert M.t2(ref[idx], oracle.forward(w.xyz, None, w.S[idx])) <= 1e-10


def test_cube41_strained_against_oracle():
    w = wl.cube41(True)
    A = api.scatter_fwd(dev(w.xyz), None, dev(w.S)).cpu().numpy().astype(np.complex128)
    rng = np.random.default_rng(71)
    idx = np.unique(np.concatenate([rng.choice(w.n_points, 200, replace=False),
                                    np.argsort(-np.abs(A))[:56]]))
    A_ref = oracle.forward(w.xyz, None, w.S[idx])
    e1, e2 = M.t1(A[idx], A_ref), M.t2(A[idx], A_ref)
    print(f"cube41 strained sampled: T1={e1:.3e} T2={e2:.3e}", flush=True)
    assert e1 <= M.T1_TOL and e2 <= M.T2_TOL


@pytest.mark.parametrize("n", [1000, 100000])
def test_chain_against_analytic_formula(n):
    """The paper's chain formula is the reference: the FP64-phase mode keeps a reliable
    intensity range far beyond the paper's single-precision 1e8."""
    xyz, S = wl.chain(n)
    ref = replay.chain_amplitude(S[:, 0].astype(np.float64), n)
    A = api.scatter_fwd(dev(xyz), None, dev(S)).cpu().numpy().astype(np.complex128)
    dr = replay.reliable_range(A, ref)
    print(f"chain N={n} ph64 reliable range {dr:.2e}", flush=True)
    assert dr >= 1e10
    # the analytic formula agrees with the oracle
    assert M.t2(ref, oracle.forward(xyz, None, S)) <= 1e-12


def test_fig1_sweep_code_runs_small():
    text = replay.fig1(max_pairs=1e8, sizes=(100, 1000, 10000))
    rows = [ln for ln in text.splitlines() if ln.startswith("| 1e+0")]
    assert len(rows) == 6 and all(ln.count("e+") == 4 for ln in rows)


def test_cube_and_chain_reports_run():
    """The replay reports themselves (timing loops included) on the GPU."""
    cube = replay.cube()
    rows = [ln for ln in cube.splitlines() if ln.startswith("| plain") or ln.startswith("| strained")]
    assert len(rows) == 7
    chain = replay.chain()
    ph64 = [ln for ln in chain.splitlines() if "| ph64 |" in ln]
    assert len(ph64) == 3
    for ln in ph64:
        assert float(ln.split("|")[3]) >= 1e10      # reliable range of the FP64-phase mode
