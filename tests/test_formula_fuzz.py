"""Differential fuzzing of the formula front end (host only): the library's
parser (csrc/formula.cpp) and the oracle's independent parser
(oracle/formula.py) must agree on what is accepted and on its size; random
well-formed formulas must lower to pass lists that replay to the oracle."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle.formula as of
from paper_2207_06803_amd import fftc

from test_formula_host import replay

TOKENS = ["DFT(2)", "DFT(3)", "DFT(4)", "DFT(8)", "DFT(12)", "DFT(11)", "I(1)", "I(2)", "I(4)", "I(6)",
          "twiddle(4,2)", "twiddle(8, 4)", "twiddle(6,3)", "twiddle(4,3)", "Permute(4,2)", "Permute(8,2)",
          "Permute(6,2)", "Permute(6,4)", "identity(2)", "dft(2)", "(", ")", "⊗", "·", "(x)", "*", "@", ".",
          " kron ", "Input", "foo(2)", "DFT(", ",", "2", " ", "DFT 2", "I(0)", "DFT(99999999999999)"]


def lib_result(text):
    try:
        return True, fftc.formula_lower(text)[0]
    except fftc.FFTCError as e:
        assert e.status in (1, 2), e
        return False, e.status


def oracle_result(text):
    try:
        return True, of.size(of.parse(text))
    except ValueError:
        return False, None


@settings(max_examples=600, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.lists(st.sampled_from(TOKENS), min_size=1, max_size=9))
def test_parsers_agree_on_token_soup(parts):
    text = "".join(parts)
    ok_lib, v_lib = lib_result(text)
    ok_or, v_or = oracle_result(text)
    if ok_lib and ok_or:
        assert v_lib == v_or, text
    elif ok_or and not ok_lib:
        # accepted by the oracle, refused by the library: only for a size the
        # library cannot lower (status 2), never a syntax or shape disagreement
        assert v_lib == 2, (text, v_lib)
    else:
        assert not ok_lib and not ok_or, (text, ok_lib, ok_or)


# well-formed formulas from the grammar: (size, text)
@st.composite
def formula(draw, depth=0):
    kind = draw(st.sampled_from(["dft", "id", "tw", "perm", "kron", "mul"] if depth < 3 else ["dft", "id", "tw", "perm"]))
    if kind == "dft":
        n = draw(st.sampled_from([1, 2, 3, 4, 5, 6, 8, 11, 12, 16]))
        return n, f"DFT({n})"
    if kind == "id":
        n = draw(st.sampled_from([1, 2, 3, 4]))
        return n, f"I({n})"
    if kind in ("tw", "perm"):
        n = draw(st.sampled_from([4, 6, 8, 12]))
        m = draw(st.sampled_from([d for d in range(1, n + 1) if n % d == 0]))
        return n, f"{'twiddle' if kind == 'tw' else 'Permute'}({n}, {m})"
    a, ta = draw(formula(depth + 1))
    if kind == "kron":
        b, tb = draw(formula(depth + 1))
        if a * b > 256:
            return a, ta
        return a * b, f"({ta}) ⊗ ({tb})"
    # a product needs equal sizes: pad the right operand with an identity
    b, tb = draw(formula(depth + 1))
    if b != a:
        if a % b == 0:
            tb, b = f"I({a // b}) ⊗ ({tb})", a
        else:
            return a, ta
    return a, f"({ta}) · ({tb})"


@settings(max_examples=200, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(formula(), st.sampled_from([0, fftc.FORMULA_NO_FOLD, fftc.FORMULA_NO_FOLD | fftc.FORMULA_EQ2]))
def test_random_formulas_lower_to_the_oracle(f, flags):
    n, text = f
    dim, desc = fftc.formula_lower(text, flags)
    assert dim == n == of.size(of.parse(text))
    rng = np.random.default_rng(n)
    x = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    want = of.apply(text, x)
    if "plan I(" in desc:
        p, m = [int(t.split(")")[0]) for t in desc.split("plan I(")[1].split("DFT(")]
        got = np.fft.fft(x.reshape(2, p, m), axis=2).reshape(2, n)
    else:
        got = replay(desc, x)
    assert np.abs(got - want).max() < 1e-10 * max(1, n), (text, desc)


# texts the token soup has drawn where the two parsers once disagreed; each
# must be judged the same way by both, every run
@pytest.mark.parametrize("text", [
    "DFT(2)· kron ",            # the word form of the Kronecker product is no vector name
    "DFT(2) . KRON",
    "DFT(2) · kron_x",          # an identifier that only starts with the keyword is a vector
    "DFT(4) · Input",
])
def test_parsers_agree_on_recorded_cases(text):
    ok_lib, v_lib = lib_result(text)
    ok_or, v_or = oracle_result(text)
    assert ok_lib == ok_or, (text, ok_lib, ok_or)
    if ok_lib:
        assert v_lib == v_or, text
