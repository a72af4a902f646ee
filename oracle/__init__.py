"""FP64 CPU oracle for the direct scattering sum -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The GPU library never imports, links or calls it, and this
package imports nothing from the GPU library: the two share no code.

What it computes (Favre-Nicolin et al., 2010):

* ``forward``  -- Section 2.1, Eq. 2, A(S_k) = sum_j f_j exp(2 i pi S_k . r_j),
  written out as a plain double loop in FP64.
* ``loss``     -- L = sum_k (|A_k|^2 - I_k)^2 with seed G_k = 4 (|A_k|^2 - I_k) A_k,
  the intensity misfit used to fit displacement fields (motivated in Section 6;
  the paper prints no loss).
* ``adjoint``  -- the chain rule through Eq. 2,
  dL/dr_j = Re sum_k conj(G_k) f_j (2 i pi S_k) exp(2 i pi S_k . r_j).
* ``adjoint_f`` -- the same for the factors, dL/df_j = conj(sum_k conj(G_k) exp(2 i pi S_k . r_j)).
* ``forward_species`` / ``adjoint_species`` -- the species-factorised sum of Section 4.2,
  A_k = sum_s fs[s][k] sum_{j in s} exp(2 i pi S_k . r_j), composed from the functions
  above (per-species unit-factor sums; the seed of species s is G conj(fs[s])).

Inputs are the caller's arrays widened exactly to float64 (FP32 inputs become the
same numbers in FP64), so the oracle evaluates exactly the problem the GPU sees.
The C source is ``nx_oracle.c``; ``build()`` compiles it with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nx_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_DP = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
             "-shared", "-o", tmp, _SRC, "-lm"],
            check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _bind(path):
    lib = ctypes.CDLL(path)
    lib.nxo_forward.argtypes = [_I64, _DP, _DP, _I64, _DP, _DP]
    lib.nxo_forward.restype = None
    lib.nxo_loss.argtypes = [_I64, _DP, _DP, _DP]
    lib.nxo_loss.restype = ctypes.c_double
    lib.nxo_adjoint.argtypes = [_I64, _DP, _DP, _I64, _DP, _DP, _DP]
    lib.nxo_adjoint.restype = None
    lib.nxo_adjoint_f.argtypes = [_I64, _DP, _I64, _DP, _DP, _DP]
    lib.nxo_adjoint_f.restype = None
    lib.nxo_threads.argtypes = []
    lib.nxo_threads.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _bind(_LIB)
    return _lib


def _f64(a, cols=None):
    a = np.ascontiguousarray(np.asarray(a), dtype=np.float64)
    if cols is not None:
        a = a.reshape(-1, cols)
    return a


def _ptr(a):
    return a.ctypes.data_as(_DP) if a is not None else None


def _f_pairs(f, n):
    """Complex per-atom factors as an (n, 2) float64 array, or None for f_j = 1."""
    if f is None:
        return None
    f = np.asarray(f)
    if f.ndim == 2 and not np.iscomplexobj(f):
        return _f64(f, 2)                         # already (re, im) pairs
    f = f.reshape(-1)
    out = np.zeros((n, 2), dtype=np.float64)
    out[:, 0] = f.real
    if np.iscomplexobj(f):
        out[:, 1] = f.imag
    return out


def forward(xyz, f, S, lib=None) -> np.ndarray:
    """Eq. 2 at every row of S.  xyz (N,3), f (N,) complex / (N,2) pairs / None, S (K,3).

    Returns complex128 (K,)."""
    lib = lib or _load()
    xyz = _f64(xyz, 3)
    S = _f64(S, 3)
    n, k = xyz.shape[0], S.shape[0]
    fp = _f_pairs(f, n)
    A = np.zeros((k, 2), dtype=np.float64)
    lib.nxo_forward(n, _ptr(xyz), _ptr(fp), k, _ptr(S), _ptr(A))
    return A[:, 0] + 1j * A[:, 1]


def loss(A, I, lib=None):
    """Misfit L = sum (|A|^2 - I)^2 and seed G = 4 (|A|^2 - I) A (complex128)."""
    lib = lib or _load()
    A = np.asarray(A)
    Ap = np.empty((A.size, 2), dtype=np.float64)
    Ap[:, 0] = A.real.reshape(-1)
    Ap[:, 1] = A.imag.reshape(-1)
    I = _f64(I).reshape(-1)
    G = np.empty_like(Ap)
    L = lib.nxo_loss(A.size, _ptr(Ap), _ptr(I), _ptr(G))
    return float(L), G[:, 0] + 1j * G[:, 1]


def adjoint(xyz, f, S, G, lib=None) -> np.ndarray:
    """dL/dr_j = Re sum_k conj(G_k) f_j (2 i pi S_k) exp(2 i pi S_k . r_j).  Returns (N,3)."""
    lib = lib or _load()
    xyz = _f64(xyz, 3)
    S = _f64(S, 3)
    n, k = xyz.shape[0], S.shape[0]
    fp = _f_pairs(f, n)
    G = np.asarray(G)
    Gp = np.empty((k, 2), dtype=np.float64)
    Gp[:, 0] = G.real.reshape(-1)
    Gp[:, 1] = G.imag.reshape(-1)
    grad = np.zeros((n, 3), dtype=np.float64)
    lib.nxo_adjoint(n, _ptr(xyz), _ptr(fp), k, _ptr(S), _ptr(Gp), _ptr(grad))
    return grad


def adjoint_f(xyz, S, G, lib=None) -> np.ndarray:
    """dL/dRe f_j + i dL/dIm f_j = conj(sum_k conj(G_k) exp(2 i pi S_k . r_j)).  Complex (N,)."""
    lib = lib or _load()
    xyz = _f64(xyz, 3)
    S = _f64(S, 3)
    n, k = xyz.shape[0], S.shape[0]
    G = np.asarray(G)
    Gp = np.empty((k, 2), dtype=np.float64)
    Gp[:, 0] = G.real.reshape(-1)
    Gp[:, 1] = G.imag.reshape(-1)
    out = np.zeros((n, 2), dtype=np.float64)
    lib.nxo_adjoint_f(n, _ptr(xyz), k, _ptr(S), _ptr(Gp), _ptr(out))
    return out[:, 0] + 1j * out[:, 1]


def forward_species(xyz, species_start, fs, S, lib=None):
    """A_k = sum_s fs[s][k] sum_{j in s} exp(2 i pi S_k . r_j); returns (A, A_species)."""
    xyz = _f64(xyz, 3)
    k = np.asarray(S).reshape(-1, 3).shape[0]
    start = [int(v) for v in species_start]
    As = np.stack([forward(xyz[start[s]:start[s + 1]], None, S, lib=lib)
                   for s in range(len(start) - 1)]) if len(start) > 1 else np.zeros((0, k))
    f = np.ones_like(As) if fs is None else np.asarray(fs, dtype=np.complex128).reshape(As.shape)
    return (f * As).sum(axis=0), As


def adjoint_species(xyz, species_start, fs, S, G, A_species=None, lib=None):
    """dL/dr for every atom (species s driven by the seed G conj(fs[s])) and, when the
    per-species sums are given, dL/dfs = G conj(A_species)."""
    xyz = _f64(xyz, 3)
    start = [int(v) for v in species_start]
    G = np.asarray(G, dtype=np.complex128).reshape(-1)
    grads = []
    for s in range(len(start) - 1):
        seed = G if fs is None else G * np.conj(np.asarray(fs, dtype=np.complex128)[s])
        grads.append(adjoint(xyz[start[s]:start[s + 1]], None, S, seed, lib=lib))
    grad = np.concatenate(grads) if grads else np.zeros((0, 3))
    gfs = None if A_species is None else G[None, :] * np.conj(np.asarray(A_species))
    return grad, gfs


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().nxo_threads())


class Variant:
    """The same three functions bound to another build of the oracle source (used by
    the mutation test, which compiles deliberately broken copies of the source and
    checks that the pins reject every one of them)."""

    def __init__(self, path):
        self.lib = _bind(path)

    def forward(self, xyz, f, S):
        return forward(xyz, f, S, lib=self.lib)

    def loss(self, A, I):
        return loss(A, I, lib=self.lib)

    def adjoint(self, xyz, f, S, G):
        return adjoint(xyz, f, S, G, lib=self.lib)

    def adjoint_f(self, xyz, S, G):
        return adjoint_f(xyz, S, G, lib=self.lib)


def compile_variant(source_text: str, out_path: str) -> "Variant":
    """Compile C source text with the oracle's flags into out_path and bind it."""
    src = out_path + ".c"
    with open(src, "w") as fh:
        fh.write(source_text)
    subprocess.run(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
                    "-shared", "-o", out_path, src, "-lm"], check=True)
    return Variant(out_path)


def source() -> str:
    with open(_SRC) as fh:
        return fh.read()
