"""The FP64 oracle against facts fixed by the paper and by mathematics."""
import mpmath
import numpy as np
import pytest

import oracle
import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(oracle.dft)


def test_eq1_factors_multiply_to_dft4_definition():
    # The printed factors of Eq. 1 against the Section II definition written
    # out for N = 4 (w_4 = -i).
    w4 = np.array([[1, 1, 1, 1], [1, -1j, -1, 1j], [1, -1, 1, -1], [1, 1j, -1, -1j]])
    assert np.array_equal(P.eq1_product(), w4)


def test_paper_correctness_protocol():
    # Section VI: random complex double inputs, N = 32 .. 1024 powers of two,
    # compared with NumPy's FFT; the paper's error |delta| / N stays < 1e-7.
    g = np.random.default_rng(2207)
    for k in range(5, 11):
        n = 1 << k
        x = g.uniform(-1, 1, n) + 1j * g.uniform(-1, 1, n)
        err = np.linalg.norm(oracle.dft(x) - np.fft.fft(x)) / n
        assert err < 1e-7 and err < 1e-15, (n, err)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 8, 12, 56, 97, 1000, 4096])
def test_twiddle_table(n):
    w = oracle.twiddles(n, -1)
    m = np.arange(n)
    # against 40-digit values from mpmath (independent arbitrary precision)
    mpmath.mp.dps = 40
    exact = np.array([complex(mpmath.cos(2 * mpmath.pi * j / n), -mpmath.sin(2 * mpmath.pi * j / n))
                      for j in range(n)])
    # within one unit in the last place of each component
    assert np.abs(w.real - exact.real).max() <= 1.2e-16
    assert np.abs(w.imag - exact.imag).max() <= 1.2e-16
    # exact symmetries: w[N-m] = conj(w[m]); w[m + N/2] = -w[m]
    assert np.array_equal(w[(-m) % n], w.conj())
    if n % 2 == 0:
        assert np.array_equal(w[(m + n // 2) % n], -w)
    assert np.array_equal(oracle.twiddles(n, +1), w.conj())
    assert w[0] == 1


def test_large_n_against_numpy():
    g = np.random.default_rng(5)
    for n in (8192, 16384):
        x = g.uniform(-1, 1, n) + 1j * g.uniform(-1, 1, n)
        ref = np.fft.fft(x)
        err = np.linalg.norm(oracle.dft(x) - ref) / np.linalg.norm(ref)
        assert err < 5e-15, (n, err)


def test_complex64_inputs_promoted_exactly():
    g = np.random.default_rng(3)
    x = (g.uniform(-1, 1, 64) + 1j * g.uniform(-1, 1, 64)).astype(np.complex64)
    assert np.array_equal(oracle.dft(x), oracle.dft(x.astype(np.complex128)))


def test_batch_rows_independent():
    g = np.random.default_rng(4)
    x = g.standard_normal((5, 48)) + 1j * g.standard_normal((5, 48))
    y = oracle.dft(x)
    for b in range(5):
        assert np.array_equal(y[b], oracle.dft(x[b]))


def test_threads_do_not_change_result():
    g = np.random.default_rng(6)
    x = g.standard_normal((7, 300)) + 1j * g.standard_normal((7, 300))
    assert np.array_equal(oracle.dft(x, threads=1), oracle.dft(x, threads=4))


def test_bad_arguments():
    with pytest.raises(ValueError):
        oracle.dft(np.zeros((2, 0), np.complex128))
    with pytest.raises(RuntimeError):
        oracle.dft(np.zeros(4, np.complex128), sign=0)


def test_points_match_full_transform():
    # the sampled-output entry point against the full transform, bit for bit
    g = np.random.default_rng(8)
    for n in (1, 7, 96, 1000):
        x = g.uniform(-1, 1, n) + 1j * g.uniform(-1, 1, n)
        ks = np.unique(np.r_[0, n - 1, g.integers(0, n, 10)])
        for sign in (-1, 1):
            assert np.array_equal(oracle.dft_points(x, ks, sign), oracle.dft(x, sign)[ks])
    with pytest.raises(RuntimeError):
        oracle.dft_points(np.zeros(4), [4])


def test_points_large_n_against_numpy():
    g = np.random.default_rng(9)
    n = 1 << 16
    x = g.uniform(-1, 1, n) + 1j * g.uniform(-1, 1, n)
    ks = np.array([0, 1, 12345, n - 1])
    ref = np.fft.fft(x)[ks]
    assert np.abs(oracle.dft_points(x, ks) - ref).max() / np.abs(ref).max() < 1e-13
