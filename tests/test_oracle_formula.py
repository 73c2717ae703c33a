"""Pins of the formula oracle (oracle/formula.py) against what the paper and
the mathematics fix: the printed factors of Eq. 1, the DFT_4 closed form,
NumPy's FFT and 2-D FFT (library special cases), the reshape-transpose form
of the stride permutation, and the grammar's right grouping."""
import numpy as np
import pytest

from oracle import formula as of
from golden_io import eq1_factors, listing1_input
from formula_pins import ALL_PINS

from paper_2207_06803_amd import formulas


@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(of)


def test_syntax_errors():
    for bad in ["DFT(3", "DFT 3", "twiddle(4)", "foo(2)", "DFT(2) ⊗", "(DFT(2)", "DFT(2) DFT(2)",
                "DFT(-2)", "I(2) $ I(2)"]:
        with pytest.raises(ValueError):
            of.size(of.parse(bad))


def test_shape_errors():
    for bad in ["DFT(4) · DFT(2)", "twiddle(4, 3)", "Permute(6, 4)", "DFT(0)",
                "DFT(4096) ⊗ DFT(8192)"]:
        with pytest.raises(ValueError):
            of.size(of.parse(bad))


def test_right_grouping_without_parentheses():
    # DFT(2) ⊗ I(2) · twiddle(4,2) groups as DFT(2) ⊗ (I(2) · twiddle(4,2)):
    # a product of sizes 2 and 4, rejected by the shape rule
    with pytest.raises(ValueError):
        of.size(of.parse("DFT(2) ⊗ I(2) · twiddle(4,2)"))
    assert of.size(of.parse("(DFT(2) ⊗ I(2)) · twiddle(4,2)")) == 4
    # I(2) ⊗ DFT(2) · DFT(2) is I(2) ⊗ (DFT(2) · DFT(2)) = I(2) ⊗ 2 I(2)
    F = of.dense("I(2) ⊗ DFT(2) · DFT(2)")
    assert np.array_equal(F, np.kron(np.eye(2), 2 * np.eye(2)))


def test_trailing_operand_and_spellings():
    ref = of.dense("(DFT(2) ⊗ I(2)) · twiddle(4,2) · (I(2) ⊗ DFT(2)) · Permute(4,2)")
    for text in ["(DFT(2) ⊗ I(2)) · twiddle(4,2) · (I(2) ⊗ DFT(2)) · Permute(4,2) · InputComplex",
                 "(dft(2) (x) i(2)) . TWIDDLE(4, 2) . (identity(2) kron DFT(2)) * permute(4,2)",
                 "(DFT(2) (x) I(2)) @ twiddle(4,2) @ (I(2) (x) DFT(2)) @ Permute(4,2)"]:
        assert np.array_equal(of.dense(text), ref)


def test_apply_matches_dense():
    rng = np.random.default_rng(3)
    texts = [formulas.recursive_ct(16, (4,)), formulas.recursive_dif(12, (3, 2)), formulas.dft2d(3, 5),
             "Permute(12, 3) · (I(3) ⊗ twiddle(4, 2)) · (DFT(3) ⊗ I(4))",
             "(DFT(2) ⊗ Permute(6, 2)) · (twiddle(6, 3) ⊗ I(2)) · (I(3) ⊗ DFT(4))",
             "DFT(7) ⊗ (DFT(2) · twiddle(2, 1)) ⊗ I(3)"]
    for t in texts:
        n = of.size(of.parse(t))
        x = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
        for sign in (of.FORWARD, of.INVERSE):
            F = of.dense(t, sign)
            np.testing.assert_allclose(of.apply(t, x, sign), x @ F.T, rtol=0, atol=1e-12 * n)


def test_listing1_program_output():
    # Listing 1: the factorised DFT_4 applied to createComplex([1,2,3,4], [1,2,3,4]);
    # by the definition y = (1 + i) DFT_4 [1,2,3,4] = (1 + i) [10, -2+2i, -2, -2-2i]
    x = listing1_input()
    y = of.apply(formulas.recursive_ct(4), x)
    assert np.array_equal(y, np.array([10 + 10j, -4 + 0j, -2 - 2j, 0 - 4j]))


def test_eq1_factors_match_print():
    names = ["(DFT(2) ⊗ I(2))", "twiddle(4, 2)", "(I(2) ⊗ DFT(2))", "Permute(4, 2)"]
    for text, (_, printed) in zip(names, eq1_factors()):
        assert np.array_equal(of.dense(text), printed), text
