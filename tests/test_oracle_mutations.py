"""The oracle's pins must reject plausible mistakes.  Each case below plants one
mistake in a copy of the oracle's C source (a flipped sign, a dropped term, a
transposed index, a missing conjugate or factor), compiles it on the CPU and runs
every pin against it: at least one pin has to fail.  The real oracle is never
modified."""
import os

import pytest

import oracle
from tests import test_oracle_pins as pins

MUTATIONS = {
    "sin_sign": ("*s = sin(a);", "*s = -sin(a);"),
    "missing_2pi": ("double a = 2.0 * M_PI * t;", "double a = M_PI * t;"),
    "dropped_z_term": ("sx * xyz[3 * j] + sy * xyz[3 * j + 1] + sz * xyz[3 * j + 2];",
                       "sx * xyz[3 * j] + sy * xyz[3 * j + 1];"),
    "transposed_yz": ("sx * xyz[3 * j] + sy * xyz[3 * j + 1] + sz * xyz[3 * j + 2];",
                      "sx * xyz[3 * j] + sy * xyz[3 * j + 2] + sz * xyz[3 * j + 1];"),
    "conj_f_re": ("re += fr * c - fi * s;", "re += fr * c + fi * s;"),
    "conj_f_im": ("im += fr * s + fi * c;", "im += fr * s - fi * c;"),
    "last_atom_dropped": ("for (int64_t j = 0; j < n_atoms; ++j) {\n            double phase",
                          "for (int64_t j = 0; j + 1 < n_atoms; ++j) {\n            double phase"),
    "loss_factor": ("G[2 * k] = 4.0 * e * re;", "G[2 * k] = 2.0 * e * re;"),
    "loss_not_squared": ("L += e * e;", "L += e;"),
    "loss_sign_I": ("double e = re * re + im * im - I[k];", "double e = re * re + im * im + I[k];"),
    "adjoint_no_conj_G": ("double gr = G[2 * k], gi = -G[2 * k + 1];", "double gr = G[2 * k], gi = G[2 * k + 1];"),
    "adjoint_sign_2pi": ("double qr = -2.0 * M_PI * pi_;", "double qr = 2.0 * M_PI * pi_;"),
    "adjoint_wrong_index": ("gy += zr * sy;", "gy += zr * sx;"),
    "adjoint_phase_sign": ("double zr = qr * c - qi * s;", "double zr = qr * c + qi * s;"),
    "adjoint_f_no_conj_G": ("double gr = G[2 * k], gi = -G[2 * k + 1];      /* conj(G_k) */",
                            "double gr = G[2 * k], gi = G[2 * k + 1];      /* conj(G_k) */"),
    "adjoint_f_sign": ("gradf[2 * j + 1] = -wi;", "gradf[2 * j + 1] = wi;"),
    "adjoint_ignores_f": ("double pr = gr * fr - gi * fi;\n            double pi_ = gr * fi + gi * fr;",
                          "double pr = gr;\n            double pi_ = gi;"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_mutation(name, tmp_path):
    old, new = MUTATIONS[name]
    src = oracle.source()
    assert src.count(old) >= 1, "mutation target not found in the oracle source"
    mutant = oracle.compile_variant(src.replace(old, new, 1), os.path.join(tmp_path, f"mut_{name}.so"))
    failed = []
    for pin in pins.PINS:
        try:
            pin(mutant)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"no pin rejects the planted mistake '{name}'"


# ----------------------------------------------------------------------------- Python compositions

PY_MUTATIONS = {
    "species_seed_no_conj": ("adjoint_species",
                             "seed = G if fs is None else G * np.conj(np.asarray(fs, dtype=np.complex128)[s])",
                             "seed = G if fs is None else G * np.asarray(fs, dtype=np.complex128)[s]"),
    "species_gradf_no_conj": ("adjoint_species",
                              "gfs = None if A_species is None else G[None, :] * np.conj(np.asarray(A_species))",
                              "gfs = None if A_species is None else G[None, :] * np.asarray(A_species)"),
    "species_factor_conj": ("forward_species", "return (f * As).sum(axis=0), As",
                            "return (np.conj(f) * As).sum(axis=0), As"),
    "species_boundary_off_by_one": ("forward_species", "forward(xyz[start[s]:start[s + 1]], None, S, lib=lib)",
                                    "forward(xyz[start[s]:max(start[s], start[s + 1] - 1)], None, S, lib=lib)"),
}


@pytest.mark.parametrize("name", sorted(PY_MUTATIONS))
def test_species_pins_reject_mutation(name):
    """The same check for the species compositions, which are Python: a mutated copy of
    the function is compiled from its source and handed to the species pins."""
    import inspect
    import types

    fn_name, old, new = PY_MUTATIONS[name]
    src = inspect.getsource(getattr(oracle, fn_name))
    assert src.count(old) == 1, "mutation target not found in the oracle source"
    namespace = dict(vars(oracle))
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), namespace)
    mutant = types.SimpleNamespace(forward=oracle.forward, loss=oracle.loss,
                                   forward_species=oracle.forward_species,
                                   adjoint_species=oracle.adjoint_species)
    setattr(mutant, fn_name, namespace[fn_name])
    failed = []
    for pin in pins.SPECIES_PINS:
        try:
            pin(mutant)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"no pin rejects the planted mistake '{name}'"
