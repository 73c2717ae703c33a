"""Pins for the formula oracle (oracle/formula.py), written against facts
fixed outside it.  Each check takes the oracle module (or a mutated copy,
see test_oracle_formula_mutations.py) and raises AssertionError on failure.

Sources of truth (none of them is the formula oracle's own code):
  * the four factor matrices printed in Eq. 1 and the DFT_4 they multiply to
  * the Listing 1 program's output, derived by hand from the definition
  * numpy.fft.fft / ifft / fft2 (pocketfft): Eq. 2 written out recursively
    is DFT_N, and DFT_a (x) DFT_b is the 2-D DFT of the row-major a x b array
  * numpy's reshape / transpose for the stride permutation Pi^N_K
  * closed-form twiddle entries (surds) for D^8_4 and D^9_3
  * the Kronecker product's index rule on explicit small cases
"""
import math

import numpy as np

from golden_io import eq1_factors, listing1_input

from paper_2207_06803_amd import formulas


def _rng(seed):
    return np.random.default_rng(seed)


def _cvec(rng, *shape):
    return rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape)


def pin_eq1_factors(of):
    texts = ["(DFT(2) ⊗ I(2))", "twiddle(4, 2)", "(I(2) ⊗ DFT(2))", "Permute(4, 2)"]
    prod = np.eye(4, dtype=np.complex128)
    for text, (_, printed) in zip(texts, eq1_factors()):
        assert np.array_equal(of.dense(text), printed), text
        prod = prod @ printed
    assert np.array_equal(of.dense(formulas.recursive_ct(4)), prod)


def pin_dft4_closed_form(of):
    i = 1j
    want = np.array([[1, 1, 1, 1], [1, -i, -1, i], [1, -1, 1, -1], [1, i, -1, -i]])
    assert np.array_equal(of.dense("DFT(4)"), want)
    assert np.array_equal(of.dense(formulas.recursive_ct(4)), want)
    assert np.array_equal(of.dense(formulas.recursive_dif(4)), want)


def pin_listing1_output(of):
    y = of.apply(formulas.recursive_ct(4) + " · InputComplex", listing1_input())
    assert np.array_equal(y, np.array([10 + 10j, -4 + 0j, -2 - 2j, -4j])), y


def pin_recursive_ct_is_fft(of):
    for n, rs in [(2, (2,)), (6, (2, 3)), (8, (2,)), (12, (3, 2)), (16, (4,)), (16, (2,)),
                  (27, (3,)), (30, (5, 3, 2)), (32, (2,)), (64, (4, 2)), (64, (8,))]:
        want = np.fft.fft(np.eye(n), axis=0)
        for text in (formulas.recursive_ct(n, rs), formulas.recursive_dif(n, rs)):
            got = of.dense(text)
            assert np.abs(got - want).max() < 1e-14 * n, (n, rs, text)


def pin_inverse_is_conjugate(of):
    rng = _rng(5)
    for n in (5, 8, 12):
        x = _cvec(rng, 2, n)
        got = of.apply(formulas.recursive_ct(n, (2, 3, 5)), x, of.INVERSE)
        assert np.abs(got - n * np.fft.ifft(x, axis=1)).max() < 1e-13 * n


def pin_dft2d_is_fft2(of):
    rng = _rng(7)
    for a, b in [(2, 3), (4, 4), (3, 8), (8, 5)]:
        x = _cvec(rng, 2, a * b)
        want = np.fft.fft2(x.reshape(2, a, b)).reshape(2, a * b)
        assert np.abs(of.apply(formulas.dft2d(a, b), x) - want).max() < 1e-13 * a * b
        assert np.abs(x @ of.dense(formulas.dft2d(a, b)).T - want).max() < 1e-13 * a * b


def pin_permute_is_reshape_transpose(of):
    # (Pi^N_K x)[i M + j] = x[j K + i]: x viewed as an M x K row-major array, transposed
    rng = _rng(9)
    for N, K in [(4, 2), (6, 2), (6, 3), (12, 4), (30, 5), (64, 8)]:
        M = N // K
        x = _cvec(rng, N)
        want = x.reshape(M, K).T.reshape(-1)
        assert np.array_equal(of.apply(f"Permute({N}, {K})", x), want), (N, K)
        assert np.array_equal(of.dense(f"Permute({N}, {K})") @ x, want), (N, K)


def pin_twiddle_closed_forms(of):
    h = math.sqrt(0.5)
    w8 = complex(h, -h)
    # D^8_4: positions i 4 + j, i < 2, j < 4 hold w_8^{i j}
    want8 = [1, 1, 1, 1, 1, w8, -1j, complex(-h, -h)]
    got8 = np.diag(of.dense("twiddle(8, 4)"))
    assert np.abs(got8 - np.array(want8)).max() < 2e-16
    # D^9_3: positions i 3 + j hold w_9^{i j}; w_9^4 = cos(8 pi/9) - i sin(8 pi/9)
    got9 = np.diag(of.dense("twiddle(9, 3)"))
    ang = [0, 0, 0, 0, 1, 2, 0, 2, 4]
    want9 = np.array([complex(math.cos(2 * math.pi * a / 9), -math.sin(2 * math.pi * a / 9)) for a in ang])
    assert np.abs(got9 - want9).max() < 4e-16
    # D^N_M is the identity when M = 1 or M = N
    assert np.array_equal(of.dense("twiddle(6, 1)"), np.eye(6))
    assert np.array_equal(of.dense("twiddle(6, 6)"), np.eye(6))


def pin_kron_index_rule(of):
    x = np.arange(6) + 1j * np.arange(6, 12)
    y = of.apply("DFT(2) ⊗ I(3)", x)          # y[a 3 + c] = x[c] + (-1)^a x[3 + c]
    assert np.array_equal(y, np.concatenate([x[:3] + x[3:], x[:3] - x[3:]]))
    y = of.apply("I(3) ⊗ DFT(2)", x)          # y[2 c + a] = x[2 c] + (-1)^a x[2 c + 1]
    want = np.empty(6, complex)
    want[0::2] = x[0::2] + x[1::2]
    want[1::2] = x[0::2] - x[1::2]
    assert np.array_equal(y, want)
    assert np.array_equal(of.dense("DFT(2) ⊗ I(3)") @ x, np.concatenate([x[:3] + x[3:], x[:3] - x[3:]]))


def pin_products_apply_right_to_left(of):
    # Permute(6, 2) · DFT(6) reorders the transform's outputs; DFT(6) · Permute(6, 2) its inputs
    rng = _rng(13)
    x = _cvec(rng, 6)
    f = np.fft.fft(x)
    src = np.arange(6).reshape(3, 2).T.reshape(-1)
    assert np.abs(of.apply("Permute(6, 2) · DFT(6)", x) - f[src]).max() < 1e-14
    assert np.abs(of.apply("DFT(6) · Permute(6, 2)", x) - np.fft.fft(x[src])).max() < 1e-14


def pin_right_grouping(of):
    # One precedence level, grouping to the right (the grammar of Listing 2):
    # DFT(2) ⊗ I(2) · twiddle(4, 2) is DFT(2) ⊗ (I(2) · twiddle(4, 2)), sizes 2 and 4
    try:
        of.size(of.parse("DFT(2) ⊗ I(2) · twiddle(4, 2)"))
    except ValueError:
        pass
    else:
        raise AssertionError("DFT(2) ⊗ I(2) · twiddle(4, 2) accepted")
    # I(2) ⊗ DFT(2) · DFT(2) = I(2) ⊗ (DFT_2 DFT_2) = 2 I_4
    assert np.array_equal(of.dense("I(2) ⊗ DFT(2) · DFT(2)"), 2 * np.eye(4))
    # DFT(2) · DFT(2) ⊗ I(1) = DFT_2 (DFT_2 (x) I_1) = 2 I_2
    assert np.array_equal(of.dense("DFT(2) · DFT(2) ⊗ I(1)"), 2 * np.eye(2))


ALL_PINS = [pin_right_grouping, pin_eq1_factors, pin_dft4_closed_form, pin_listing1_output, pin_recursive_ct_is_fft,
            pin_inverse_is_conjugate, pin_dft2d_is_fft2, pin_permute_is_reshape_transpose,
            pin_twiddle_closed_forms, pin_kron_index_rule, pin_products_apply_right_to_left]
