"""Accuracy of the hardware sin and cos of gfx950 (v_sin_f32 / v_cos_f32, which take the
angle in turns), measured through the public forward: the error budget of the FP64-phase
mode rests on these figures (Section 2.2 notes that the GPU's sin/cos are hardware
approximations; Section 2.3 discusses the single-precision error they feed).

* Raw instructions.  One atom at r = (1, 0, 0) with f = 1 and points S = (t, 0, 0), t on
  a 2^-20 grid of [-1/2, 1/2].  In the plain FP32 mode the phase S.r = t is exact, the
  reduction fract(t) is exact on that grid, and a one-term sum stores the instructions'
  results unchanged: A = (v_cos(u), v_sin(u)) with u = fract(t).  Compared with
  cos 2 pi t and sin 2 pi t in FP64.
* One term of the FP64-phase mode.  The same atom and f = 1 at seeded random t in
  [-1/2, 1/2] and at t plus integers up to 2^10 (the FP64 phase is exact; its reduced
  value is rounded once to FP32): the error of a single term as the forward computes
  it (phase rounding, the instructions, the group's turn-back factor), per component,
  against the FP64 oracle.

The bounds are the figures the tolerance derivation uses (max 1.25e-7, rms 3.5e-8 for the
instructions; about 5e-8 rms per FP64-phase term), with the margin stated at each."""
import numpy as np
import pytest
import torch

import oracle
from paper_1010_2641_amd import api

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")

# the instructions' measured error (per component, against FP64)
RAW_MAX, RAW_RMS = 1.3e-7, 3.6e-8
# one FP64-phase term, per component: the phase rounding (at most 2^-26 cycles, 9.4e-8 rad;
# about 3e-8 rms per component), the instructions (1.24e-7 max, 3.5e-8 rms) and the
# rounded turn-back factor of the group's eighth turn with its two fma (about 3e-8 rms,
# at most 9e-8 for odd turns): about 5e-8 rms, at most 3.1e-7
TERM_RMS, TERM_MAX = 6e-8, 3.2e-7


def one_atom_forward(t, mode):
    xyz = torch.tensor([[1.0, 0.0, 0.0]], dtype=torch.float32, device=DEV)
    S = torch.zeros((t.size, 3), dtype=torch.float32, device=DEV)
    S[:, 0] = torch.from_numpy(t.astype(np.float32)).to(DEV)
    A = api.scatter_fwd(xyz, None, S, mode)
    torch.cuda.synchronize()
    return A.cpu().numpy().astype(np.complex128)


def component_errors(A, t):
    ref_c = np.cos(2 * np.pi * (t - np.rint(t)))
    ref_s = np.sin(2 * np.pi * (t - np.rint(t)))
    return np.concatenate([A.real - ref_c, A.imag - ref_s])


def test_raw_sin_cos_error():
    t = -0.5 + np.arange((1 << 20) + 1, dtype=np.float64) * 2.0 ** -20
    assert np.array_equal(t.astype(np.float32).astype(np.float64), t)
    A = one_atom_forward(t, "f32")
    e = component_errors(A, t)
    emax, erms = float(np.max(np.abs(e))), float(np.sqrt(np.mean(e * e)))
    ec = A.real - np.cos(2 * np.pi * t)
    es = A.imag - np.sin(2 * np.pi * t)
    print(f"v_cos/v_sin on {t.size} grid turns: max {emax:.3e} rms {erms:.3e} "
          f"(cos max {np.max(np.abs(ec)):.3e}, sin max {np.max(np.abs(es)):.3e})", flush=True)
    assert emax <= RAW_MAX and erms <= RAW_RMS


def test_ph64_term_error():
    rng = np.random.default_rng(31)
    t = rng.uniform(-0.5, 0.5, 1 << 20).astype(np.float32).astype(np.float64)
    t_far = (t[: 1 << 16] + rng.integers(-1024, 1025, 1 << 16)).astype(np.float32).astype(np.float64)
    for name, tt in (("|t| <= 1/2", t), ("t + n, |n| <= 1024", t_far)):
        A = one_atom_forward(tt, "ph64")
        ref = oracle.forward(np.array([[1.0, 0.0, 0.0]]), None, np.stack(
            [tt, np.zeros_like(tt), np.zeros_like(tt)], axis=1))
        d = np.concatenate([A.real - ref.real, A.imag - ref.imag])
        emax, erms = float(np.max(np.abs(d))), float(np.sqrt(np.mean(d * d)))
        print(f"FP64-phase term error per component, {name}: max {emax:.3e} rms {erms:.3e} "
              f"(complex: rms {np.sqrt(2) * erms:.3e})", flush=True)
        assert erms <= TERM_RMS and emax <= TERM_MAX
