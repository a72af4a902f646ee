"""Seeded random shapes and launch plans against the oracle: atom and point counts drawn
log-uniformly (with at most 2e8 pairs per case), factor kind, precision mode and the
plan knobs (items per lane, record staging, launch size, group size, reduction variant)
drawn at random, so that the
combinations of splits, chunks, ragged tails and kernel forms are exercised beyond the
hand-picked cases.  The draws are fixed by the seed; every case prints its parameters."""
import numpy as np
import pytest
import torch

import oracle
from paper_1010_2641_amd import api, workloads as wl
from tests import metrics as M

pytestmark = pytest.mark.gpu


def draw(case):
    rng = np.random.default_rng(7000 + case)
    while True:
        n = int(np.exp(rng.uniform(0, np.log(60000))))
        k = int(np.exp(rng.uniform(0, np.log(60000))))
        if n * k <= 2e8:
            break
    c = dict(n=n, k=k, fkind=str(rng.choice(["none", "real", "complex"])),
             mode=str(rng.choice(["ph64", "ph64", "f64", "f32"])),
             P=str(rng.choice(["", "1", "2", "4"])), lds=str(rng.choice(["", "0", "1"])),
             pairs=str(rng.choice(["", str(1 << 22), str(1 << 26)])), seed=int(rng.integers(1 << 30)))
    # drawn last, so that the draws above are those of the cases without these knobs
    c.update(grp=str(rng.choice(["", "8", "16", "32"])), red=str(rng.choice(["", "0", "1"])))
    return c


@pytest.mark.parametrize("case", range(48))
def test_random_shape(case, monkeypatch):
    c = draw(case)
    print(f"case {case}: {c}", flush=True)
    for var, val in (("NX_TUNE_P", c["P"]), ("NX_TUNE_LDS", c["lds"]), ("NX_TUNE_LAUNCH_PAIRS", c["pairs"]),
                     ("NX_TUNE_GRP", c["grp"]), ("NX_TUNE_RED", c["red"])):
        if val and not (var == "NX_TUNE_P" and val == "4" and c["mode"] == "f64"):
            monkeypatch.setenv(var, val)
    n, k = c["n"], c["k"]
    xyz, f, S = wl.random_problem(n, k, seed=c["seed"], extent=30.0, s_range=3.0,
                                  complex_f=(c["fkind"] == "complex"))
    if c["fkind"] == "real":
        f = np.random.default_rng(c["seed"]).uniform(0.5, 2.0, n).astype(np.complex64)
    G = wl.random_seed_field(k, seed=c["seed"] + 1)
    dev = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()
    if c["mode"] == "f64":
        A = api.scatter_fwd_f64(dev(xyz.astype(np.float64)), None if f is None else dev(f.astype(np.complex128)),
                                dev(S.astype(np.float64)))
        g = api.scatter_bwd_f64(dev(xyz.astype(np.float64)), None if f is None else dev(f.astype(np.complex128)),
                                dev(S.astype(np.float64)), dev(G.astype(np.complex128)))
    else:
        A = api.scatter_fwd(dev(xyz), dev(f), dev(S), c["mode"])
        g = api.scatter_bwd(dev(xyz), dev(f), dev(S), dev(G), c["mode"])
    torch.cuda.synchronize()
    A = A.cpu().numpy().astype(np.complex128)
    g = g.cpu().numpy().astype(np.float64)
    e = M.incoherent(A, oracle.forward(xyz, f, S), f, n)
    en, _ = M.t3(g, oracle.adjoint(xyz, f, S, G))
    print(f"  pointwise/scale={e:.2e} adjoint T3={en:.2e}", flush=True)
    lim_f = {"ph64": M.INC_TOL, "f64": M.F64_INC_TOL, "f32": 2e-3}[c["mode"]]
    lim_b = {"ph64": M.T3_NORM_TOL, "f64": M.F64_T3_TOL, "f32": 5e-3}[c["mode"]]
    # a single point or atom: normwise adjoint errors of one term
    if min(n, k) < 4:
        lim_b = max(lim_b, {"ph64": 1e-4, "f64": 1e-10, "f32": 2e-2}[c["mode"]])
    assert e <= lim_f and en <= lim_b
