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
        "(kind == 2) ? cos_coef(q, m, N) : cos_coef(m, q, N)",
        "(kind == 2) ? cos_coef(m, q, N) : cos_coef(q, m, N)"),
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


# ------------------------------------------------------------- IDXST mutants
import test_oracle_idxst as idxst_pins


def _idxst_variant(orc, reverse="shifted", zero_first=True, sign=1):
    """A copy of the oracle's idxst_axis with one step changed."""
    def fn(x, axis, norm="backward", sel=None):
        x = np.asarray(x, dtype=np.float64)
        axis = axis % x.ndim
        n = x.shape[axis]
        if reverse == "shifted":
            src = [0] + list(range(n - 1, 0, -1))
        elif reverse == "plain":
            src = list(range(n - 1, -1, -1))
        else:
            src = list(range(n))
        y = np.take(x, np.array(src, dtype=np.int64), axis=axis)
        if zero_first:
            first = [slice(None)] * x.ndim
            first[axis] = 0
            y[tuple(first)] = 0.0
        keep = None if sel is None else list(sel)
        z = orc.idctn(y, norm, axes=[axis], sel=None if keep is None else {axis: keep})
        k = np.arange(n) if keep is None else np.asarray(keep)
        s = np.ones(k.size) if sign == 0 else np.where((k + (sign < 0)) % 2 == 0, 1.0, -1.0)
        return z * orc._bcast(s, z.ndim, axis)
    return fn


IDXST_MUTANTS = {
    "reversal_without_shift": dict(reverse="plain", zero_first=False),
    "first_element_not_zeroed": dict(zero_first=False, reverse="plain_shifted"),
    "no_reversal": dict(reverse="none", zero_first=False),
    "no_sign": dict(sign=0),
    "sign_shifted": dict(sign=-1),
}


def _run_idxst_pins(orc):
    failed = []
    checks = {
        "sine_b": lambda: idxst_pins.test_idxst_is_a_sine_sum(orc, "backward", 8),
        "sine_o": lambda: idxst_pins.test_idxst_is_a_sine_sum(orc, "ortho", 9),
        "first": lambda: idxst_pins.test_idxst_ignores_first_element(orc),
        "brute": lambda: idxst_pins.test_mixed_2d_brute_force(orc, "backward", (4, 6)),
    }
    for name, fn in checks.items():
        try:
            fn()
        except (AssertionError, ValueError):
            failed.append(name)
    return failed


def test_idxst_pins_pass_on_committed_oracle(orc):
    assert _run_idxst_pins(orc) == []


@pytest.mark.parametrize("name", sorted(IDXST_MUTANTS))
def test_idxst_mutant_is_caught(orc, monkeypatch, name):
    kw = dict(IDXST_MUTANTS[name])
    if kw.get("reverse") == "plain_shifted":
        kw["reverse"] = "shifted"
    monkeypatch.setattr(orc, "idxst_axis", _idxst_variant(orc, **kw))
    assert _run_idxst_pins(orc), f"no pin caught mutant {name}"


def test_mixed_axes_swapped_is_caught(orc, monkeypatch):
    """IDCT_IDXST with the two axes exchanged (IDXST along axis 1)."""
    def swapped(x, norm="backward", sel=None):
        return orc.idctn(orc.idxst_axis(x, 1, norm), norm, axes=[0])
    monkeypatch.setattr(orc, "idct_idxst2", swapped)
    assert _run_idxst_pins(orc)
