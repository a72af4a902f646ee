"""The gradient with respect to the scattering factors and the species-factorised sum
(Section 4.2: one unit-factor sum per species, multiplied by that species' factor at
each S), against the FP64 oracle, element by element, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_1010_2641_amd import api, workloads as wl
from tests import metrics as M
from tests.test_gpu_configs import central_lines, sample_points

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return None if t is None else t.cpu().numpy()


def cplx_t3(g, g_ref):
    """T3 on a complex gradient, taken over its real and imaginary parts."""
    return M.t3(np.stack([np.real(g), np.imag(g)]), np.stack([np.real(g_ref), np.imag(g_ref)]))


def run_bwd_ex(xyz, f, S, G, mode, want_xyz=True):
    if mode == "f64":
        gx, gf = api.scatter_bwd_ex_f64(dev(xyz.astype(np.float64)),
                                        None if f is None else dev(f.astype(np.complex128)),
                                        dev(S.astype(np.float64)), dev(G.astype(np.complex128)),
                                        want_xyz, True)
    else:
        gx, gf = api.scatter_bwd_ex(dev(xyz), dev(f), dev(S), dev(G.astype(np.complex64)), mode,
                                    want_xyz, True)
    return host(gx), host(gf)


# ----------------------------------------------------------------------------- dL/df

GF_TOL = {"ph64": (M.T3_NORM_TOL, M.T3_MAX_TOL), "f64": (M.F64_T3_TOL, M.F64_T3_TOL),
          "f32": (5e-3, 5e-2)}


@pytest.mark.parametrize("n,k,cplx", [(2999, 4001, True), (1000, 2500, False), (300, 9000, True)])
@pytest.mark.parametrize("mode", ["ph64", "f64", "f32"])
def test_grad_f_random_ragged(n, k, cplx, mode):
    xyz, f, S = wl.random_problem(n, k, seed=n + 7 * k, extent=40.0, s_range=3.0, complex_f=cplx)
    G = wl.random_seed_field(k, seed=n + k)
    print(f"case grad_f N={n} K={k} complex={cplx} mode={mode}", flush=True)
    gx, gf = run_bwd_ex(xyz, f, S, G, mode)
    gf_ref = oracle.adjoint_f(xyz, S, G)
    en, em = cplx_t3(gf, gf_ref)
    print(f"  dL/df T3 norm={en:.3e} max={em:.3e}", flush=True)
    tn, tm = GF_TOL[mode]
    assert en <= tn and em <= tm
    # the position gradient of the same call is the plain adjoint's
    xn, xm = M.t3(gx, oracle.adjoint(xyz, f, S, G))
    assert xn <= GF_TOL[mode][0] and xm <= GF_TOL[mode][1]


def test_grad_f_matches_plain_adjoint_positions_bitwise():
    """Adding the two factor sums changes nothing in the position sums."""
    xyz, f, S = wl.random_problem(5000, 3000, seed=41, extent=30.0, s_range=2.0)
    G = wl.random_seed_field(3000, seed=42)
    gx, _ = run_bwd_ex(xyz, f, S, G, "ph64")
    g0 = host(api.scatter_bwd(dev(xyz), dev(f), dev(S), dev(G), "ph64"))
    assert np.array_equal(gx, g0)


@pytest.mark.parametrize("mode", ["ph64", "f64", "f32"])
@pytest.mark.parametrize("n,k", [(1, 1), (100, 0), (1, 333), (257, 15), (33, 17)])
def test_grad_f_edge_sizes(n, k, mode):
    xyz, f, S = wl.random_problem(n, k, seed=43 + n + k, extent=10.0, s_range=2.0)
    G = wl.random_seed_field(k, seed=44)
    print(f"case grad_f edge N={n} K={k} mode={mode}", flush=True)
    _, gf = run_bwd_ex(xyz, f, S, G, mode, want_xyz=False)
    gf_ref = oracle.adjoint_f(xyz, S, G)
    if k == 0:
        assert np.all(gf == 0)
        return
    en, em = cplx_t3(gf, gf_ref)
    assert en <= GF_TOL[mode][0] and em <= GF_TOL[mode][1]


@pytest.mark.parametrize("mode", ["ph64", "f64"])
def test_grad_f_chunked_launches(mode, monkeypatch):
    monkeypatch.setenv("NX_TUNE_LAUNCH_PAIRS", str(1 << 20))
    xyz, f, S = wl.random_problem(1500, 7000, seed=45, extent=25.0, s_range=3.0)
    G = wl.random_seed_field(7000, seed=46)
    gx, gf = run_bwd_ex(xyz, f, S, G, mode)
    en, em = cplx_t3(gf, oracle.adjoint_f(xyz, S, G))
    assert en <= GF_TOL[mode][0] and em <= GF_TOL[mode][1]
    xn, xm = M.t3(gx, oracle.adjoint(xyz, f, S, G))
    assert xn <= GF_TOL[mode][0] and xm <= GF_TOL[mode][1]


def test_autograd_factor_gradient():
    """ScatterFn with f requiring a gradient: torch's complex gradient of a real loss
    (dL/dRe f + i dL/dIm f) from the hand-written kernel, against the oracle."""
    xyz, f, S = wl.random_problem(800, 1500, seed=47, extent=15.0, s_range=2.0)
    I = np.abs(wl.random_seed_field(1500, seed=48, scale=30.0)).astype(np.float32) ** 2
    A_ref = oracle.forward(xyz, f, S)
    _, G_ref = oracle.loss(A_ref, I)
    x = dev(xyz).requires_grad_(True)
    ff = dev(f).requires_grad_(True)
    A = api.scatter(x, ff, dev(S), "ph64")
    L = ((A.abs() ** 2 - dev(I)) ** 2).sum()
    L.backward()
    en, em = cplx_t3(host(ff.grad), oracle.adjoint_f(xyz, S, G_ref))
    print(f"autograd dL/df T3 norm={en:.3e} max={em:.3e}", flush=True)
    assert en <= M.T3_NORM_TOL and em <= M.T3_MAX_TOL
    xn, xm = M.t3(host(x.grad), oracle.adjoint(xyz, f, S, G_ref))
    assert xn <= M.T3_NORM_TOL and xm <= M.T3_MAX_TOL


def test_gradcheck_f64_factors():
    """torch.autograd.gradcheck over positions and complex factors (FP64 kernels)."""
    xyz, f, S = wl.random_problem(10, 16, seed=49, extent=4.0, s_range=1.0)
    x = dev(xyz.astype(np.float64)).requires_grad_(True)
    ff = dev(f.astype(np.complex128)).requires_grad_(True)
    SS = dev(S.astype(np.float64))
    assert torch.autograd.gradcheck(lambda a, b: api.scatter(a, b, SS), (x, ff), eps=1e-6, atol=1e-7,
                                    rtol=1e-5)


# ----------------------------------------------------------------------------- species

def species_problem(counts, k, seed, extent=30.0, s_range=3.0):
    rng = np.random.default_rng(seed)
    n = int(sum(counts))
    xyz = (rng.random((n, 3)) * extent).astype(np.float32)
    S = ((rng.random((k, 3)) * 2 - 1) * s_range).astype(np.float32)
    start = [0] + np.cumsum(counts).astype(int).tolist()
    base = [complex(31, 1), complex(22, 3.5), complex(8, 0.2), complex(14, -0.5)]
    fs = wl.species_factor_table(S, [base[s % 4] for s in range(len(counts))],
                                 b_iso=(1.2, 0.6, 0.3, 0.9))
    return xyz, start, fs, S


def species_scale(fs, start):
    n_s = np.diff(start).astype(np.float64)
    return np.sqrt(np.sum(n_s[:, None] * np.abs(fs.astype(np.complex128)) ** 2, axis=0))


@pytest.mark.parametrize("counts,k", [((1200, 1801), 2500), ((0, 700, 1, 333), 1031),
                                      ((4097,), 300), ((5, 9, 1000, 0, 17), 64),
                                      # species above and below 65,536 atoms (16- and 8-atom
                                      # groups) starting at offsets that are not multiples of
                                      # either: each species' records are packed with its plan
                                      ((70001, 333, 66001), 300)])
@pytest.mark.parametrize("mode", ["ph64", "f32"])
def test_species_forward_random(counts, k, mode):
    xyz, start, fs, S = species_problem(counts, k, seed=sum(counts) + k)
    print(f"case species fwd counts={counts} K={k} mode={mode}", flush=True)
    A, As = api.scatter_fwd_species(dev(xyz), start, dev(fs), dev(S), mode, return_species=True)
    A, As = host(A), host(As)
    A_ref, As_ref = oracle.forward_species(xyz, start, fs, S)
    e = float(np.max(np.abs(A - A_ref) / species_scale(fs, start)))
    es = max((float(np.max(np.abs(As[s] - As_ref[s]))) / np.sqrt(max(start[s + 1] - start[s], 1))
              for s in range(len(counts))), default=0.0)
    print(f"  pointwise/scale={e:.3e} per-species={es:.3e}", flush=True)
    lim = M.INC_TOL if mode == "ph64" else 2e-3
    assert e <= lim and es <= lim


def test_species_forward_unit_factors():
    """fs = None: every species factor is 1, so the sum is the unit-factor Eq. 2."""
    xyz, start, _, S = species_problem((300, 0, 901), 777, seed=51)
    A = host(api.scatter_fwd_species(dev(xyz), start, None, dev(S)))
    assert M.incoherent(A, oracle.forward(xyz, None, S), None, len(xyz)) <= M.INC_TOL


@pytest.mark.parametrize("counts,k", [((1200, 1801), 2500), ((0, 700, 1, 333), 1031), ((64,), 0),
                                      ((3, 0), 17)])
@pytest.mark.parametrize("mode", ["ph64", "f32"])
def test_species_adjoint_random(counts, k, mode):
    xyz, start, fs, S = species_problem(counts, k, seed=2 * sum(counts) + k)
    G = wl.random_seed_field(k, seed=52)
    print(f"case species bwd counts={counts} K={k} mode={mode}", flush=True)
    _, As = api.scatter_fwd_species(dev(xyz), start, dev(fs), dev(S), mode, return_species=True)
    gx, gfs = api.scatter_bwd_species(dev(xyz), start, dev(fs), dev(S), dev(G), As, mode)
    gx, gfs = host(gx), host(gfs)
    _, As_ref = oracle.forward_species(xyz, start, fs, S)
    gx_ref, gfs_ref = oracle.adjoint_species(xyz, start, fs, S, G, As_ref)
    if k == 0:
        assert np.all(gx == 0) and gfs.size == 0
        return
    tn, tm = (M.T3_NORM_TOL, M.T3_MAX_TOL) if mode == "ph64" else (5e-3, 5e-2)
    en, em = M.t3(gx, gx_ref)
    fn_, fm = cplx_t3(gfs, gfs_ref)
    print(f"  grad_xyz T3 {en:.3e}/{em:.3e}  grad_fs T3 {fn_:.3e}/{fm:.3e}", flush=True)
    assert en <= tn and em <= tm
    assert fn_ <= tn and fm <= tm


def test_species_autograd():
    """ScatterSpeciesFn: gradients with respect to positions and to the S-dependent
    species factors, from a torch-side loss, against the oracle."""
    xyz, start, fs, S = species_problem((500, 400), 1200, seed=53, extent=12.0, s_range=1.5)
    I = np.abs(wl.random_seed_field(1200, seed=54, scale=300.0)).astype(np.float32) ** 2
    A_ref, As_ref = oracle.forward_species(xyz, start, fs, S)
    _, G_ref = oracle.loss(A_ref, I)
    gx_ref, gfs_ref = oracle.adjoint_species(xyz, start, fs, S, G_ref, As_ref)
    x = dev(xyz).requires_grad_(True)
    f = dev(fs).requires_grad_(True)
    A = api.scatter_species(x, start, f, dev(S))
    L = ((A.abs() ** 2 - dev(I)) ** 2).sum()
    L.backward()
    en, em = M.t3(host(x.grad), gx_ref)
    fn_, fm = cplx_t3(host(f.grad), gfs_ref)
    print(f"species autograd: grad_xyz {en:.3e}/{em:.3e} grad_fs {fn_:.3e}/{fm:.3e}", flush=True)
    assert en <= M.T3_NORM_TOL and em <= M.T3_MAX_TOL
    assert fn_ <= M.T3_NORM_TOL and fm <= M.T3_MAX_TOL


def test_species_bitwise_deterministic():
    xyz, start, fs, S = species_problem((2000, 3000), 4000, seed=55)
    a = host(api.scatter_fwd_species(dev(xyz), start, dev(fs), dev(S)))
    b = host(api.scatter_fwd_species(dev(xyz), start, dev(fs), dev(S)))
    assert np.array_equal(a, b)


def test_species_python_validation():
    x = torch.zeros((4, 3), dtype=torch.float32, device=DEV)
    with pytest.raises(ValueError, match="species_start"):
        api.scatter_fwd_species(x, [0, 5], None, x)
    with pytest.raises(ValueError, match="fs must have shape"):
        api.scatter_fwd_species(x, [0, 2, 4], torch.zeros((3, 4), dtype=torch.complex64, device=DEV), x)


def test_c2_species_forward_and_fit_step():
    """C2 with its two species factored out: the species-factorised forward against the
    oracle on sampled points (per-atom factors, the original atom order), against the
    all-FP64 path on every point at T1 <= 1e-5 (both the same Eq. 2 amplitude), and
    against the per-atom-factor kernel on every point (two single-precision results, each
    within T1 of the truth); the species adjoint against the per-atom adjoint on sampled
    atoms."""
    w = wl.c2()
    xs, start, vals, order = wl.group_by_species(w.xyz, w.f)
    fs = np.repeat(vals[:, None], w.n_points, axis=1)
    tS = dev(w.S)
    A_sp = host(api.scatter_fwd_species(dev(xs), start, dev(fs), tS))
    A_pa = host(api.scatter_fwd(dev(w.xyz), dev(w.f), tS))
    A64 = host(api.scatter_fwd_f64(dev(w.xyz.astype(np.float64)), dev(w.f.astype(np.complex128)),
                                   tS.double()))
    idx = sample_points(w.n_points, 256, central_lines(128, 3), seed=7)
    A_ref = oracle.forward(w.xyz, w.f, w.S[idx])
    e1, e2 = M.t1(A_sp[idx], A_ref), M.t2(A_sp[idx], A_ref)
    print(f"c2 species sampled: T1={e1:.3e} T2={e2:.3e}", flush=True)
    assert e1 <= M.T1_TOL and e2 <= M.T2_TOL
    assert M.t1(A64[idx], A_ref) <= M.F64_T1_TOL
    f1, f2 = M.t1(A_sp, A64), M.t2(A_sp, A64)
    print(f"c2 species vs f64 path, full grid: T1={f1:.3e} T2={f2:.3e}", flush=True)
    assert f1 <= M.T1_TOL and f2 <= M.T2_TOL
    g1, g2 = M.t1(A_sp, A_pa), M.t2(A_sp, A_pa)
    print(f"c2 species vs per-atom kernel, full grid: T1={g1:.3e} T2={g2:.3e}", flush=True)
    assert g1 <= 2 * M.T1_TOL and g2 <= 2 * M.T2_TOL
    # fit step: species adjoint vs per-atom adjoint on the same seed
    I = (api.scatter_fwd(dev(w.target_xyz), dev(w.f), tS).abs() ** 2).float()
    L, A, gs = api.fit_step_species(dev(xs), start, dev(fs), tS, I)
    G = api.loss_grad(A, I)[1]
    gp = api.scatter_bwd(dev(xs), dev(w.f[order]), tS, G)
    rng = np.random.default_rng(8)
    atoms = np.sort(rng.choice(w.n_atoms, size=4096, replace=False))
    g64 = api.scatter_bwd_f64(dev(xs[atoms].astype(np.float64)),
                              dev(w.f[order][atoms].astype(np.complex128)),
                              tS.double(), G.to(torch.complex128))
    en, em = M.t3(host(gs)[atoms], host(g64))
    print(f"c2 species adjoint vs f64 path: T3 norm={en:.3e} max={em:.3e}", flush=True)
    assert en <= M.T3_NORM_TOL and em <= M.T3_MAX_TOL
    pn, pm = M.t3(host(gs), host(gp))
    assert pn <= 2 * M.T3_NORM_TOL and pm <= 2 * M.T3_MAX_TOL


@pytest.mark.parametrize("mode", ["ph64", "f32"])
def test_species_chunked_launches(mode, monkeypatch):
    """Species sums carried across launch chunks (forward) and across chunks of points
    (adjoint), with an empty species among them."""
    monkeypatch.setenv("NX_TUNE_LAUNCH_PAIRS", str(1 << 20))
    xyz, start, fs, S = species_problem((1500, 0, 2100), 3000, seed=56)
    G = wl.random_seed_field(3000, seed=57)
    A, As = api.scatter_fwd_species(dev(xyz), start, dev(fs), dev(S), mode, return_species=True)
    gx, gfs = api.scatter_bwd_species(dev(xyz), start, dev(fs), dev(S), dev(G), As, mode)
    A, As, gx, gfs = host(A), host(As), host(gx), host(gfs)
    A_ref, As_ref = oracle.forward_species(xyz, start, fs, S)
    gx_ref, gfs_ref = oracle.adjoint_species(xyz, start, fs, S, G, As_ref)
    lim = M.INC_TOL if mode == "ph64" else 2e-3
    assert float(np.max(np.abs(A - A_ref) / species_scale(fs, start))) <= lim
    tn = M.T3_NORM_TOL if mode == "ph64" else 5e-3
    assert M.t3(gx, gx_ref)[0] <= tn and cplx_t3(gfs, gfs_ref)[0] <= tn
