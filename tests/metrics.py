"""Error measures used by the GPU parity tests (definitions, not arithmetic of the
method).  All inputs are numpy arrays; references come from the FP64 oracle.

* ``t1``  pointwise intensity error: max |(|A|^2 - |A_ref|^2)| / |A_ref|^2 over the
          points with |A_ref|^2 >= floor * max |A_ref|^2 (max over evaluated points);
* ``t2``  normwise amplitude error ||A - A_ref|| / ||A_ref|| (complex, so it sees phase);
* ``t3``  adjoint errors: (||g - g_ref|| / ||g_ref||, max|g - g_ref| / max|g_ref|);
* ``incoherent``  max_k |A_k - A_ref,k| / sqrt(sum_j |f_j|^2): for atoms at random
          positions the sum is a random walk, |A| ~ sqrt(sum |f|^2) and no point is
          far above that scale, so per-term rounding is judged against it (T1's
          1e-6 floor is meant for crystals, whose peaks reach N |f|);
* ``dynamic_range``  the paper's reliability measure (Section 2.3): max I_ref divided
          by the largest I_ref at which the relative intensity error first exceeds
          `rel` when the points are visited from the strongest down.
"""
import numpy as np

# tolerances of the FP64-phase FP32 mode (and of the all-FP64 path, much tighter)
T1_TOL, T2_TOL = 1e-5, 1e-6
T3_NORM_TOL, T3_MAX_TOL = 1e-5, 1e-4
F64_T1_TOL, F64_T2_TOL = 1e-9, 1e-12
F64_T3_TOL = 1e-11
# random-position problems: pointwise error against the random-walk scale
INC_TOL, F64_INC_TOL = 2e-6, 1e-12


def incoherent(A, A_ref, f, n):
    A = np.asarray(A, dtype=np.complex128)
    A_ref = np.asarray(A_ref, dtype=np.complex128)
    scale = np.sqrt(n) if f is None else np.sqrt(np.sum(np.abs(np.asarray(f, np.complex128)) ** 2))
    return float(np.max(np.abs(A - A_ref)) / scale) if A.size else 0.0


def t1(A, A_ref, floor=1e-6):
    I = np.abs(np.asarray(A, dtype=np.complex128)) ** 2
    Ir = np.abs(np.asarray(A_ref, dtype=np.complex128)) ** 2
    if Ir.size == 0 or Ir.max() == 0:
        return 0.0
    m = Ir >= floor * Ir.max()
    return float(np.max(np.abs(I[m] - Ir[m]) / Ir[m]))


def t2(A, A_ref):
    A = np.asarray(A, dtype=np.complex128)
    A_ref = np.asarray(A_ref, dtype=np.complex128)
    den = np.linalg.norm(A_ref)
    return float(np.linalg.norm(A - A_ref) / den) if den > 0 else float(np.linalg.norm(A))


def t3(g, g_ref):
    g = np.asarray(g, dtype=np.float64)
    g_ref = np.asarray(g_ref, dtype=np.float64)
    return (float(np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)),
            float(np.max(np.abs(g - g_ref)) / np.max(np.abs(g_ref))))


def dynamic_range(A, A_ref, rel=1e-2):
    I = np.abs(np.asarray(A, dtype=np.complex128)) ** 2
    Ir = np.abs(np.asarray(A_ref, dtype=np.complex128)) ** 2
    order = np.argsort(-Ir)
    e = np.abs(I[order] - Ir[order]) / np.maximum(Ir[order], 1e-300)
    bad = np.nonzero(e > rel)[0]
    if bad.size == 0:
        return np.inf
    return float(Ir[order[0]] / max(Ir[order[bad[0]]], 1e-300))
