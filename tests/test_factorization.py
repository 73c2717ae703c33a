"""Eq. 1, Eq. 2 and the Stockham stage, checked as dense matrices on the CPU.

These pin the readings of the stride permutation Pi^N_K and the twiddle
diagonal D^N_M (Section II names them without defining their index maps) and
the index formulas of the Stockham stages that the GPU kernels implement.
"""
import itertools

import numpy as np
import pytest

import factor_algebra as F
from golden_io import eq1_factors


def _divisor_pairs(n):
    return [(k, n // k) for k in range(1, n + 1) if n % k == 0]


def test_eq1_factors_are_eq2_at_n4():
    # Eq. 1 is Eq. 2 with N = 4, K = M = 2: compare factor by factor.
    names = dict(eq1_factors())
    assert np.allclose(names["DFT2_kron_I2"], np.kron(F.dft_matrix(2), np.eye(2)))
    assert np.allclose(names["twiddle_diag"], F.twiddle_diag(4, 2), atol=1e-15)
    assert np.allclose(names["I2_kron_DFT2"], np.kron(np.eye(2), F.dft_matrix(2)))
    assert np.array_equal(names["permute"], F.stride_perm(4, 2))


@pytest.mark.parametrize("n", range(1, 65))
def test_eq2_identity_all_splits(n):
    want = F.dft_matrix(n)
    for k, _ in _divisor_pairs(n):
        for sign in (-1, 1):
            got = F.eq2(n, k, sign)
            assert np.abs(got - F.dft_matrix(n, sign)).max() < 1e-13, (n, k, sign)
    assert want.shape == (n, n)


def test_stride_reading_of_pi_is_forced():
    # The other stride reading (gather at stride M) breaks Eq. 2 whenever K != M.
    for n in (6, 8, 12, 18, 24, 32):
        for k, m in _divisor_pairs(n):
            if k == m or k == 1 or m == 1:
                continue
            alt = (np.kron(F.dft_matrix(k), np.eye(m)) @ F.twiddle_diag(n, m)
                   @ np.kron(np.eye(k), F.dft_matrix(m)) @ F.stride_perm(n, m))
            assert np.abs(alt - F.dft_matrix(n)).max() > 1e-3, (n, k)


SEQUENCES = [[2], [4], [8], [16], [3], [5], [7], [2, 2, 2], [4, 4], [8, 8], [4, 16], [16, 4],
             [16, 16], [2, 8, 4], [3, 16], [16, 3], [4, 3], [3, 4, 5], [7, 8], [8, 7],
             [5, 2], [7, 2, 4], [3, 3], [5, 5], [7, 7], [2, 16, 2]]


@pytest.mark.parametrize("radices", SEQUENCES, ids=lambda r: "x".join(map(str, r)))
def test_stockham_stages_multiply_to_dft(radices):
    n = int(np.prod(radices))
    for sign in (-1, 1):
        got = F.stockham_product(n, radices, sign)
        assert np.abs(got - F.dft_matrix(n, sign)).max() < 1e-12, (radices, sign)


@pytest.mark.parametrize("radices", [[4, 16], [3, 4, 5], [7, 8], [2, 2, 2], [16, 3]],
                         ids=lambda r: "x".join(map(str, r)))
def test_stage_index_form_equals_kronecker_form(radices):
    n = int(np.prod(radices))
    ns = 1
    for r in radices:
        a = F.stockham_stage_matrix(n, r, ns)
        b = F.stockham_stage_kron(n, r, ns)
        assert np.abs(a - b).max() < 1e-13, (radices, r, ns)
        ns *= r


def test_stage_is_sparse():
    # Each stage has exactly R nonzeros per row: O(N R) work, not O(N^2).
    for radices in ([4, 16], [8, 8], [3, 4, 5]):
        n = int(np.prod(radices))
        ns = 1
        for r in radices:
            s = F.stockham_stage_matrix(n, r, ns)
            assert all(np.count_nonzero(np.abs(row) > 1e-14) == r for row in s)
            ns *= r


def test_kronecker_as_matrix_product():
    # (A (x) I_n) vec_row(X) = vec_row(A X): the form a DFT_16 stage takes as
    # a dense 16 x 16 matrix times a 16 x n matrix.
    g = np.random.default_rng(0)
    a = g.standard_normal((16, 16)) + 1j * g.standard_normal((16, 16))
    x = g.standard_normal((16, 12)) + 1j * g.standard_normal((16, 12))
    assert np.allclose(np.kron(a, np.eye(12)) @ x.reshape(-1), (a @ x).reshape(-1))


def test_all_orders_of_a_factorisation_work():
    for perm in set(itertools.permutations([2, 3, 4])):
        got = F.stockham_product(24, list(perm))
        assert np.abs(got - F.dft_matrix(24)).max() < 1e-12, perm
