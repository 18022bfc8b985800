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
