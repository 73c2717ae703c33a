"""Plausible mistakes planted in copies of the formula oracle are caught by
the formula pins.  Each mutant is a textual edit of oracle/formula.py loaded
as a separate module; the real oracle is never modified."""
import importlib.util
import os
import sys

import pytest

from formula_pins import ALL_PINS

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "formula.py")

MUTANTS = {
    "permute_reading": ("return j * K + i", "return i * M + j"),
    "twiddle_other_subscript": ("i, j = t // M, t % M", "i, j = t // (N // M), t % (N // M)"),
    "twiddle_modulus": ("return _powers(N)[(i * j) % N]", "return _powers(N)[(i * j) % (2 * N)] ** 2"),
    "kron_operand_order": ('return np.kron(A, B) if op == "kron" else A @ B',
                           'return np.kron(B, A) if op == "kron" else A @ B'),
    "product_order": ('return np.kron(A, B) if op == "kron" else A @ B',
                      'return np.kron(A, B) if op == "kron" else B @ A'),
    "apply_product_order": ("return _apply(tree[1], _apply(tree[2], X))",
                            "return _apply(tree[2], _apply(tree[1], X))"),
    "apply_kron_axes": ("Z = X.reshape(rows, a, b)",
                        "Z = np.ascontiguousarray(X.reshape(rows, b, a).transpose(0, 2, 1))"),
    "dft_exponent": ("return _powers(n)[np.outer(j, j) % n]", "return _powers(n)[np.outer(j, j + 1) % n]"),
    "inverse_drops_conj": ("    if sign == INVERSE:\n        Y = np.conj(Y)", "    if False:\n        Y = np.conj(Y)"),
    "left_grouping": ('return ("kron", left, self.expr())', 'return ("kron", left, self.primary())'),
}


def _load(tmp_path, name, old, new):
    src = open(SRC, encoding="utf-8").read()
    assert src.count(old) >= 1, name
    pkg = tmp_path / f"oracle_{name}"
    pkg.mkdir()
    # the copy imports the real C-oracle helpers through the package `oracle`
    (pkg / "__init__.py").write_text("from oracle import dft, twiddles\n")
    (pkg / "formula.py").write_text(src.replace(old, new), encoding="utf-8")
    sys.path.insert(0, str(tmp_path))
    try:
        spec = importlib.util.spec_from_file_location(f"oracle_{name}.formula", pkg / "formula.py",
                                                      submodule_search_locations=None)
        mod = importlib.util.module_from_spec(spec)
        mod.__package__ = f"oracle_{name}"
        spec.loader.exec_module(mod)
    finally:
        sys.path.remove(str(tmp_path))
    return mod


def test_unmutated_copy_passes(tmp_path):
    mod = _load(tmp_path, "identity", "return j * K + i", "return j * K + i")
    for pin in ALL_PINS:
        pin(mod)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    mod = _load(tmp_path, name, *MUTANTS[name])
    failed = []
    for pin in ALL_PINS:
        try:
            pin(mod)
        except (AssertionError, ValueError, IndexError):
            failed.append(pin.__name__)
    assert failed, f"mutant {name} passed every pin"
