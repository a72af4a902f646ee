"""Property tests of the oracle on hypothesis-drawn shapes and values (N and K from 0).

Each property is fixed by Eq. 2 itself, not by re-typing it: superposition over any
split of the atoms, linearity in f, the phase factor of an integer translation, Friedel
symmetry for real f, f = NULL as f_j = 1, and the adjoints as the exact derivatives of
the forward (central differences in the positions; the factor adjoint as the linear
map it is).  Coordinates and points are dyadic, so translated coordinates stay exact in
FP32 and S.t is exact in FP64."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle

SETTINGS = settings(max_examples=40, deadline=None)


@st.composite
def problems(draw, min_n=0, min_k=0, real_f=False):
    n = draw(st.integers(min_n, 12))
    k = draw(st.integers(min_k, 12))
    seed = draw(st.integers(0, 2 ** 32 - 1))
    rng = np.random.default_rng(seed)
    xyz = (rng.integers(-2560, 2561, size=(n, 3)) / 64.0).astype(np.float32)    # |x| <= 40
    S = (rng.integers(-1024, 1025, size=(k, 3)) / 256.0).astype(np.float32)     # |S| <= 4
    fr = rng.uniform(-3, 3, n)
    fi = np.zeros(n) if real_f else rng.uniform(-3, 3, n)
    f = (fr + 1j * fi).astype(np.complex64)
    return xyz, f, S


def scale(f):
    return float(np.sum(np.abs(f.astype(np.complex128)))) + 1.0


@SETTINGS
@given(problems())
def test_shapes_and_empty_sums(p):
    xyz, f, S = p
    A = oracle.forward(xyz, f, S)
    assert A.shape == (len(S),)
    if len(xyz) == 0:
        assert np.all(A == 0)
    G = np.ones(len(S), dtype=np.complex128)
    g = oracle.adjoint(xyz, f, S, G)
    assert g.shape == (len(xyz), 3)
    if len(S) == 0:
        assert np.all(g == 0)


@SETTINGS
@given(problems(), st.integers(0, 12))
def test_superposition(p, m):
    xyz, f, S = p
    m = min(m, len(xyz))
    A = oracle.forward(xyz, f, S)
    A1 = oracle.forward(xyz[:m], f[:m], S)
    A2 = oracle.forward(xyz[m:], f[m:], S)
    assert np.max(np.abs(A - (A1 + A2)), initial=0.0) <= 1e-12 * scale(f)


@SETTINGS
@given(problems(), st.complex_numbers(max_magnitude=4.0, allow_nan=False, allow_infinity=False))
def test_linearity_in_f(p, c):
    xyz, f, S = p
    c = complex(np.complex64(c))
    cf = (f.astype(np.complex128) * c)
    A = oracle.forward(xyz, f, S)
    Ac = oracle.forward(xyz, cf, S)
    assert np.max(np.abs(Ac - c * A), initial=0.0) <= 1e-12 * (abs(c) + 1) * scale(f)


@SETTINGS
@given(problems(), st.tuples(*[st.integers(-3, 3)] * 3))
def test_integer_translation_phase(p, t):
    xyz, f, S = p
    t = np.array(t, dtype=np.float32)
    A = oracle.forward(xyz, f, S)
    At = oracle.forward(xyz + t, f, S)
    phase = np.exp(2j * np.pi * (S.astype(np.float64) @ t.astype(np.float64)))
    assert np.max(np.abs(At - phase * A), initial=0.0) <= 1e-12 * scale(f)


@SETTINGS
@given(problems(real_f=True))
def test_friedel_real_f(p):
    xyz, f, S = p
    A = oracle.forward(xyz, f, S)
    Am = oracle.forward(xyz, f, -S)
    assert np.max(np.abs(Am - np.conj(A)), initial=0.0) <= 1e-12 * scale(f)


@SETTINGS
@given(problems())
def test_null_f_is_unit_f(p):
    xyz, _, S = p
    A0 = oracle.forward(xyz, None, S)
    A1 = oracle.forward(xyz, np.ones(len(xyz), dtype=np.complex64), S)
    assert np.max(np.abs(A0 - A1), initial=0.0) <= 1e-13 * (len(xyz) + 1)


@SETTINGS
@given(problems(min_n=1, min_k=1), st.integers(0, 2 ** 32 - 1))
def test_position_adjoint_is_the_derivative(p, seed):
    """grad = d/dr Re sum_k conj(G_k) A_k(r): central differences along a random
    direction of all positions at once (h = 1e-6 in FP64 positions)."""
    xyz, f, S = p
    rng = np.random.default_rng(seed)
    G = rng.normal(size=len(S)) + 1j * rng.normal(size=len(S))
    d = rng.normal(size=xyz.shape)
    h = 1e-6
    x64 = xyz.astype(np.float64)

    def L(x):
        return float(np.real(np.sum(np.conj(G) * oracle.forward(x, f, S))))

    fd = (L(x64 + h * d) - L(x64 - h * d)) / (2 * h)
    g = oracle.adjoint(xyz, f, S, G)
    an = float(np.sum(g * d))
    bound = (2 * np.pi * 4 * np.sqrt(3)) * float(np.sum(np.abs(G))) * scale(f) * float(np.max(np.abs(d)))
    assert abs(fd - an) <= 1e-6 * bound


@SETTINGS
@given(problems(min_n=1), st.integers(0, 2 ** 32 - 1))
def test_factor_adjoint_is_the_linear_map(p, seed):
    """L(f) = Re sum_k conj(G_k) A_k(f) is linear in f, so L(df) = Re sum_j conj(gf_j) df_j
    for the factor adjoint gf (torch's convention dL/dRe f + i dL/dIm f)."""
    xyz, _, S = p
    rng = np.random.default_rng(seed)
    G = rng.normal(size=len(S)) + 1j * rng.normal(size=len(S))
    df = rng.normal(size=len(xyz)) + 1j * rng.normal(size=len(xyz))
    gf = oracle.adjoint_f(xyz, S, G)
    lhs = float(np.real(np.sum(np.conj(G) * oracle.forward(xyz, df, S))))
    rhs = float(np.real(np.sum(np.conj(gf) * df)))
    assert abs(lhs - rhs) <= 1e-12 * (float(np.sum(np.abs(G))) + 1) * (float(np.sum(np.abs(df))) + 1)
