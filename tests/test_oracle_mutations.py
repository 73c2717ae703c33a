"""Plausible mistakes planted in copies of the oracle are caught by the pins.

Each mutant is a textual edit of oracle/oracle_dft.c compiled on the CPU into
a temporary directory; the real oracle is never modified.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle_pins as P

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "oracle_dft.c")

MUTANTS = {
    "twiddle_sign": ("wi[m] = (double)sign * s;", "wi[m] = -(double)sign * s;"),
    "dropped_first_term": ("for (int64_t j = 0; j < n; ++j)", "for (int64_t j = 1; j < n; ++j)"),
    "exponent_index": ("idx += k;", "idx += k + 1;"),
    "imag_product_sign": ("a * d + bb * c", "a * d - bb * c"),
    "real_product_sign": ("a * c - bb * d", "a * c + bb * d"),
    "octant3_swapped": ("case 3: *c = -cp; *s = sp;", "case 3: *c = -sp; *s = cp;"),
    "exact_value_table": ("0.0, -0.70710678118654752440, -1.0,", "0.0, -0.70710678118654752440, 1.0,"),
    "octant_angle_scale": ("/ (4.0 * (double)n)", "/ (2.0 * (double)n)"),
    "imag_output_comp": ("out[2 * bk + 1] = si + ci;", "out[2 * bk + 1] = si - 8 * ci + 1e-14;"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                    "-ffp-contract=off", "-o", str(lib), str(path), "-lm"], check=True)
    so = ctypes.CDLL(str(lib))
    so.oracle_dft.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                              ctypes.c_int64, ctypes.c_int, ctypes.c_int]

    def dft(x, sign=-1):
        x = np.asarray(x)
        x2 = np.ascontiguousarray(np.atleast_2d(x), dtype=np.complex128)
        out = np.empty_like(x2)
        rc = so.oracle_dft(x2.ctypes.data, out.ctypes.data, x2.shape[1], x2.shape[0], sign, 0)
        assert rc == 0
        return out[0] if x.ndim == 1 else out
    return dft


def test_unmutated_copy_passes(tmp_path):
    dft = _build(tmp_path, "identity", "idx += k;", "idx += k;")
    for pin in P.ALL_PINS:
        pin(dft)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    dft = _build(tmp_path, name, *MUTANTS[name])
    failed = []
    for pin in P.ALL_PINS:
        try:
            pin(dft)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"mutant {name} passed every pin"
