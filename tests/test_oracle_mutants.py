"""Mutation check of the oracle's pins (CPU only).

Each mutant is a copy of ``oracle/dct_oracle.c`` (or of a normalisation step)
with one plausible mistake planted: a dropped term, a wrong index, a wrong sign,
a transposed operand, a wrong argument reduction.  The mutant is compiled in a
temporary directory and the pins of ``test_oracle_pins`` are run against it;
at least one pin must fail for every mutant.  The committed oracle is never
modified.
"""
import os
import subprocess

import numpy as np
import pytest

import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "dct_oracle.c")

C_MUTANTS = {
    "index_without_half": ("(2 * (int64_t)n + 1)", "(2 * (int64_t)n)"),
    "dropped_half_on_first_term": ("if (kind == 3 && m == 0) c *= 0.5;", ""),
    "transposed_coefficients": (
        "(kind == 2) ? C[(size_t)q * N + m] : C[(size_t)m * N + q]",
        "(kind == 2) ? C[(size_t)m * N + q] : C[(size_t)q * N + m]"),
    "reduction_mod_2N": ("% fourN", "% (2 * (int64_t)N)"),
    "sign_on_last_axis": ("dst[0] = s;", "dst[0] = -s;"),
    "dropped_first_term_last_axis": ("for (int m = 0; m < N; ++m) s += krow[m] * src[m];",
                                     "for (int m = 1; m < N; ++m) s += krow[m] * src[m];"),
    "dropped_last_term_inner_axes": ("for (int m = 0; m < N; ++m) {\n                    const double c",
                                     "for (int m = 0; m < N - 1; ++m) {\n                    const double c"),
}


def _run_pins(orc):
    """Return the names of the pins that fail."""
    failed = []
    checks = {
        "constant": lambda: pins.test_constant_maps_to_dc(orc, (6, 8)),
        "basis": lambda: pins.test_basis_maps_to_delta(orc, (5, 7)),
        "ramp": lambda: pins.test_ramp_closed_form(orc, (6, 9)),
        "brute": lambda: pins.test_brute_force_nonseparable(orc, (4, 6, 8)),
        "scaled_identity": lambda: pins.test_dct3_after_dct2_is_scaled_identity(orc, (5, 7)),
        "roundtrip_b": lambda: pins.test_roundtrip(orc, "backward", (6, 8)),
        "roundtrip_o": lambda: pins.test_roundtrip(orc, "ortho", (5, 7)),
        "parseval": lambda: pins.test_parseval_ortho(orc, (6, 8)),
        "poisson": lambda: pins.test_poisson_residual(orc, (12, 20)),
    }
    for name, fn in checks.items():
        try:
            fn()
        except (AssertionError, ValueError):
            failed.append(name)
    return failed


def test_pins_pass_on_committed_oracle(orc):
    assert _run_pins(orc) == []


@pytest.mark.parametrize("name", sorted(C_MUTANTS))
def test_c_mutant_is_caught(orc, tmp_path, name):
    old, new = C_MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new, 1))
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-o", str(so), str(mut), "-lm"],
                   check=True)
    prev = orc._swap_library(str(so))
    try:
        failed = _run_pins(orc)
    finally:
        orc._restore_library(prev)
    assert failed, f"no pin caught mutant {name}"


def test_norm_mutant_is_caught(orc, monkeypatch):
    """Orthonormal weight of the first index taken as sqrt(2/N) instead of sqrt(1/N)."""
    def bad(n):
        return np.full(n, np.sqrt(2.0 / n))
    monkeypatch.setattr(orc, "_ortho_scale", bad)
    assert _run_pins(orc)
