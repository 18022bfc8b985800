"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU,
in a temporary directory), rebuilds it, and checks that at least one pin
fails for the mutant.  The real oracle is untouched.
"""
import os

import pytest

import oracle
from tests import pins

MUTANTS = {
    # dH_ba read as dH_ab instead of its transpose
    "no_transpose": ("Aj[n * No + l]", "Aj[l * No + n]"),
    # kz + qz instead of kz - qz
    "kz_sign": ("((k - q) % d->Nkz + d->Nkz) % d->Nkz", "((k + q) % d->Nkz + d->Nkz) % d->Nkz"),
    # E + omega instead of E - omega
    "energy_sign": ("const int ee = e - shift[w];", "const int ee = e + shift[w];"),
    # D~ indexed (j, i)
    "d_transposed": ("* N3 + i) * N3 + j;", "* N3 + j) * N3 + i;"),
    # last frequency dropped
    "dropped_w": ("for (int w = 0; w < d->Nw; ++w)", "for (int w = 0; w < d->Nw - 1; ++w)"),
    # sign error in the complex product
    "complex_sign": ("acc[2 * x + 1] += dr * ti + dim * tr;", "acc[2 * x + 1] += dr * ti - dim * tr;"),
    # G of atom a instead of its neighbour f(a, b)
    "g_of_a": ("* d->NA + f;", "* d->NA + a;"),
    # conjugated prefactor
    "alpha_conj": ("out[2 * x] = alpha_re * r - alpha_im * im;",
                   "out[2 * x] = alpha_re * r + alpha_im * im;"),
    # dH of the neighbour atom instead of the bond (a, b)
    "dh_of_f": ("const double *Ai = dH + (((size_t)a * d->NB + b) * N3 + i) * nn;",
                "const double *Ai = dH + (((size_t)(f % d->NA) * d->NB + b) * N3 + i) * nn;"),
    # sampled evaluation: (k, e) of a listed block swapped
    "blk_k_e_swapped": ("k = blk[3 * t];\n            e = blk[3 * t + 1];",
                        "k = blk[3 * t + 1];\n            e = blk[3 * t];"),
    # sampled evaluation: G block looked up with energy and momentum exchanged
    "gslot_index": ("const int64_t s = gslot[bidx];",
                    "const int64_t s = gslot[((int64_t)ee * d->Nkz + kk) * d->NA + f];"),
    # sampled evaluation: output slot of a listed block off by one
    "blk_out_slot": ("out + (size_t)t * nn2);", "out + (size_t)((t + 1) % nblk) * nn2);"),
    # out-of-range energies wrapped instead of zero-padded
    "energy_wrap": ("if (ee < 0 || ee >= d->NE)\n                    continue;",
                    "if (ee < 0 || ee >= d->NE)\n                    ee_wrap_marker;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) >= 1, f"pattern for {name} not found"
    if name == "energy_wrap":
        new = new.replace("ee_wrap_marker;", "{ const int eee = ((ee % d->NE) + d->NE) % d->NE;"
                          " (void)eee; }")
        mutated = src.replace(old, new).replace(
            "const int64_t bidx = ((int64_t)kk * d->NE + ee) * d->NA + f;",
            "const int64_t bidx = ((int64_t)kk * d->NE + ((ee % d->NE) + d->NE) % d->NE)"
            " * d->NA + f;")
    else:
        mutated = src.replace(old, new)
    path = os.path.join(tmp_path, f"m_{name}.c")
    with open(path, "w") as fh:
        fh.write(mutated)
    lib = oracle.build(src=path, out=os.path.join(tmp_path, f"libm_{name}.so"))
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(lib=lib)
        except (AssertionError, ValueError):
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every pin"


# Mistakes in the bookkeeping of the sampled evaluation (oracle/__init__.py).
PY_MUTANTS = {
    "needed_kz_sign": ("kk = (k - q) % Nkz", "kk = (k + q) % Nkz"),
    "needed_energy_sign": ("ee = e - s", "ee = e + s"),
    "needed_atom_a": ("* NA + int(f))", "* NA + int(a))"),
    "needed_drops_top_edge": ("0 <= ee < NE", "0 <= ee < NE - 1"),
    # the atom's own G blocks listed as well as its neighbours'
    "needed_extra_self": ("need.add((kk * NE + ee) * NA + int(f))",
                          "need.add((kk * NE + ee) * NA + int(f)); "
                          "need.add((kk * NE + ee) * NA + int(a))"),
}


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_needed_blocks_mutant_is_caught(name, monkeypatch):
    import inspect
    import textwrap
    import numpy as np
    old, new = PY_MUTANTS[name]
    src = textwrap.dedent(inspect.getsource(oracle.needed_g_blocks))
    assert src.count(old) == 1, f"pattern for {name} not found"
    ns = {"np": np}
    exec(src.replace(old, new), ns)
    monkeypatch.setattr(oracle, "needed_g_blocks", ns["needed_g_blocks"])
    caught = []
    for pin in (pins.pin_sampled_blocks, pins.pin_needed_blocks_exact):
        try:
            pin()
        except (AssertionError, ValueError):
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every pin"


# Plausible mistakes in the phonon self-energy oracle (oracle/pi_oracle.c).
PI_MUTANTS = {
    # dH_ba read as dH_ab instead of its transpose
    "pi_no_transpose": ("sr += Ai[l * No + m] * x[2 * (l * No + n)];\n"
                        "                                si += Ai[l * No + m] * x[2 * (l * No + n) + 1];",
                        "sr += Ai[m * No + l] * x[2 * (l * No + n)];\n"
                        "                                si += Ai[m * No + l] * x[2 * (l * No + n) + 1];"),
    # kz - qz instead of kz + qz
    "pi_kz_sign": ("const int kk = (k + q) % d->Nkz;", "const int kk = (k - q + d->Nkz) % d->Nkz;"),
    # E - omega instead of E + omega
    "pi_energy_sign": ("const int ee = e + shift[w];", "const int ee = e - shift[w];"),
    # Y transposed inside the trace
    "pi_y_transposed": ("const double br = y[2 * (l * No + m)], bi = y[2 * (l * No + m) + 1];",
                        "const double br = y[2 * (m * No + l)], bi = y[2 * (m * No + l) + 1];"),
    # the shifted Green's function taken from the neighbour, the other from the atom
    "pi_roles_swapped": ("kk, ee, a, &missing);", "kk, ee, f, &missing);"),
    # diagonal block with the sign of the neighbour blocks
    "pi_diag_sign": ("out[2 * ((size_t)NB * N3 * N3 + x)] = -(beta_re * r - beta_im * im);",
                     "out[2 * ((size_t)NB * N3 * N3 + x)] = (beta_re * r - beta_im * im);"),
    # last neighbour left out of the diagonal
    "pi_diag_drops_b": ("for (int b = 0; b < NB; ++b) {\n            r += ",
                        "for (int b = 0; b < NB - 1; ++b) {\n            r += "),
    # last kz point dropped
    "pi_dropped_k": ("for (int k = 0; k < d->Nkz; ++k) {", "for (int k = 0; k < d->Nkz - 1; ++k) {"),
    # conjugated prefactor
    "pi_beta_conj": ("out[2 * ((size_t)b * N3 * N3 + x) + 1] = beta_re * im + beta_im * r;",
                     "out[2 * ((size_t)b * N3 * N3 + x) + 1] = beta_re * im - beta_im * r;"),
    # (i, j) of the output exchanged
    "pi_ij_swapped": ("Pb[2 * (i * N3 + j)] += tr;\n                        Pb[2 * (i * N3 + j) + 1] += ti;",
                      "Pb[2 * (j * N3 + i)] += tr;\n                        Pb[2 * (j * N3 + i) + 1] += ti;"),
    # sign error in the complex trace
    "pi_complex_sign": ("ti += ar * bi + ai * br;", "ti += ar * bi - ai * br;"),
    # sampled evaluation: (q, w) of a listed block swapped
    "pi_blk_q_w_swapped": ("q = blk[3 * t];\n            w = blk[3 * t + 1];",
                           "q = blk[3 * t + 1] % Nqz;\n            w = blk[3 * t] % Nw;"),
    # sampled evaluation: slot looked up with energy and momentum exchanged
    "pi_gslot_index": ("if (gslot[flat] < 0) {", "if (gslot[flat] < 0 || (flat = ((int64_t)e * d->Nkz + k) * d->NA + atom, 0)) {"),
}


@pytest.mark.parametrize("name", sorted(PI_MUTANTS))
def test_pi_mutant_is_caught(name, tmp_path):
    from tests import pins_pi
    old, new = PI_MUTANTS[name]
    src = open(oracle.PI_SRC).read()
    assert src.count(old) >= 1, f"pattern for {name} not found"
    mutated = src.replace(old, new)
    if name == "pi_gslot_index":
        mutated = mutated.replace("const int64_t flat = ((int64_t)k * d->NE + e) * d->NA + atom;",
                                  "int64_t flat = ((int64_t)k * d->NE + e) * d->NA + atom;")
    path = os.path.join(tmp_path, f"m_{name}.c")
    with open(path, "w") as fh:
        fh.write(mutated)
    lib = oracle.build(src=path, out=os.path.join(tmp_path, f"libm_{name}.so"))
    caught = []
    for pin in pins_pi.PI_PINS:
        try:
            pin(lib=lib)
        except (AssertionError, ValueError):
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every pin"


# Mistakes in the D~ combination and the retarded relation (oracle/__init__.py).
DT_MUTANTS = {
    "dt_no_reverse_map": ("D[:, :, f, r] - D[:, :, f, NB]", "D[:, :, a, b] - D[:, :, f, NB]"),
    "dt_diag_of_a_for_b": ("- D[:, :, f, NB] - D[:, :, a, NB]", "- D[:, :, a, NB] - D[:, :, a, NB]"),
    "dt_sign": ("- D[:, :, a, NB] + D[:, :, a, b]", "+ D[:, :, a, NB] + D[:, :, a, b]"),
    "dt_reverse_slot": ("r = slots[0]", "r = (slots[0] + 1) % NB"),
}


@pytest.mark.parametrize("name", sorted(DT_MUTANTS))
def test_dtilde_mutant_is_caught(name, monkeypatch):
    import inspect
    import textwrap
    import numpy as np
    from tests import pins_pi
    old, new = DT_MUTANTS[name]
    src = textwrap.dedent(inspect.getsource(oracle.dtilde))
    assert src.count(old) == 1, f"pattern for {name} not found"
    ns = {"np": np}
    exec(src.replace(old, new), ns)
    monkeypatch.setattr(oracle, "dtilde", ns["dtilde"])
    caught = []
    for pin in (pins_pi.pin_dtilde_structure, pins_pi.pin_dtilde_sigma_antihermitian):
        try:
            pin()
        except (AssertionError, ValueError):
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every pin"
