"""Pins for the FP64 DFT oracle, written against facts fixed outside it.

Each check takes a `dft(x, sign)` callable so the same checks can be run on
deliberately broken copies of the oracle (see test_oracle_mutations.py).  A
check returns None on success and raises AssertionError otherwise.

Sources of truth used here (none of them is the oracle's own code):
  * the four factor matrices printed in Eq. 1, whose product is DFT_4
  * the DFT_N definition, Section II: entry (m, n) is w_N^{mn},
    w_N = exp(-2 pi i / N) -- written out as explicit closed-form entries
    for N = 2, 3, 4, 5, 8 (surds, no trigonometric calls)
  * the Listing 1 input vector, through the Eq. 1 product
  * textbook identities of the DFT: delta -> ones, tone -> N delta,
    Parseval, linearity, Hermitian symmetry, shift, inverse round trip
  * numpy.fft (pocketfft), an independent third-party implementation, as
    the paper itself compared against NumPy's FFT (Section VI)
"""
import math

import numpy as np

from golden_io import eq1_factors, listing1_input

FWD, INV = -1, +1


def _mat(dft, n, sign=FWD):
    """Dense matrix of the transform: column j is the image of e_j."""
    return dft(np.eye(n, dtype=np.complex128), sign).T


def eq1_product():
    p = np.eye(4, dtype=np.complex128)
    for _, m in eq1_factors():
        p = p @ m
    return p


def pin_dft4_equals_eq1(dft):
    # The product of the printed factors has entries in {1, -1, i, -i}:
    # every product step is exact in floating point, so equality is exact.
    want = eq1_product()
    got = _mat(dft, 4)
    assert np.array_equal(got, want), (got, want)


def pin_listing1(dft):
    x = listing1_input()
    want = eq1_product() @ x   # small integers: exact
    got = dft(x, FWD)
    assert np.array_equal(got, want), (got, want)
    # the same numbers written out: [10+10i, -4, -2-2i, -4i]
    assert np.array_equal(got, np.array([10 + 10j, -4 + 0j, -2 - 2j, -4j]))


def pin_small_closed_forms(dft):
    h = math.sqrt(0.5)
    r3 = math.sqrt(3.0) / 2.0
    c5a = (math.sqrt(5.0) - 1.0) / 4.0        # cos(2 pi/5)
    c5b = -(math.sqrt(5.0) + 1.0) / 4.0       # cos(4 pi/5)
    s5a = math.sqrt((5.0 + math.sqrt(5.0)) / 8.0)  # sin(2 pi/5)
    s5b = math.sqrt((5.0 - math.sqrt(5.0)) / 8.0)  # sin(4 pi/5)
    w = {
        1: [[1]],
        2: [[1, 1], [1, -1]],
        3: [[1, 1, 1],
            [1, -0.5 - 1j * r3, -0.5 + 1j * r3],
            [1, -0.5 + 1j * r3, -0.5 - 1j * r3]],
    }
    # w_5^m = cos(2 pi m/5) - i sin(2 pi m/5)
    p5 = [1, c5a - 1j * s5a, c5b - 1j * s5b, c5b + 1j * s5b, c5a + 1j * s5a]
    w[5] = [[p5[(m * n) % 5] for n in range(5)] for m in range(5)]
    # w_8^m
    p8 = [1, h - 1j * h, -1j, -h - 1j * h, -1, -h + 1j * h, 1j, h + 1j * h]
    w[8] = [[p8[(m * n) % 8] for n in range(8)] for m in range(8)]
    for n, rows in w.items():
        want = np.array(rows, dtype=np.complex128)
        got = _mat(dft, n)
        assert np.allclose(got, want, rtol=0, atol=4e-16), (n, np.abs(got - want).max())
        # inverse is the conjugate matrix (unnormalised)
        goti = _mat(dft, n, INV)
        assert np.allclose(goti, want.conj(), rtol=0, atol=4e-16), n


def pin_delta_and_constant(dft):
    for n in (1, 2, 3, 7, 16, 60, 97, 256):
        d = np.zeros(n, np.complex128)
        d[0] = 1
        assert np.array_equal(dft(d, FWD), np.ones(n)), n
        c = np.ones(n, np.complex128)
        y = dft(c, FWD)
        want = np.zeros(n, np.complex128)
        want[0] = n
        assert np.allclose(y, want, rtol=0, atol=1e-13 * n), (n, np.abs(y - want).max())


def pin_shifted_delta_and_tone(dft):
    for n in (5, 12, 64, 100, 243):
        k = np.arange(n)
        for j in (1, n // 3, n - 1):
            d = np.zeros(n, np.complex128)
            d[j] = 1
            want = np.exp(-2j * np.pi * ((j * k) % n) / n)
            assert np.allclose(dft(d, FWD), want, rtol=0, atol=2e-15), (n, j)
        for f in (1, n // 2, n - 2):
            tone = np.exp(2j * np.pi * ((f * k) % n) / n)
            want = np.zeros(n, np.complex128)
            want[f] = n
            assert np.allclose(dft(tone, FWD), want, rtol=0, atol=1e-13 * n), (n, f)


def pin_invariants(dft, seed=7):
    g = np.random.default_rng(seed)
    for n in (8, 30, 128, 210, 1024):
        x = g.uniform(-1, 1, (3, n)) + 1j * g.uniform(-1, 1, (3, n))
        z = g.uniform(-1, 1, (3, n)) + 1j * g.uniform(-1, 1, (3, n))
        y = dft(x, FWD)
        # Parseval: sum |y|^2 = N sum |x|^2
        lhs = (np.abs(y) ** 2).sum(axis=1)
        rhs = n * (np.abs(x) ** 2).sum(axis=1)
        assert np.allclose(lhs, rhs, rtol=1e-13, atol=0), n
        # linearity
        a, b = 0.75 - 0.5j, -1.25 + 2j
        assert np.allclose(dft(a * x + b * z, FWD), a * y + b * dft(z, FWD),
                           rtol=0, atol=1e-12 * n), n
        # round trip: inverse(forward(x)) = N x
        assert np.allclose(dft(y, INV), n * x, rtol=0, atol=1e-12 * n), n
        # Hermitian symmetry for real input: y[N-k] = conj(y[k])
        yr = dft(x.real.astype(np.complex128), FWD)
        assert np.allclose(yr[:, (-np.arange(n)) % n], yr.conj(), rtol=0, atol=1e-12 * n), n
        # shift: x[j - s] -> w^{s k} y[k]
        s = 3
        k = np.arange(n)
        ys = dft(np.roll(x, s, axis=1), FWD)
        assert np.allclose(ys, y * np.exp(-2j * np.pi * ((s * k) % n) / n),
                           rtol=0, atol=1e-12 * n), n


def pin_numpy(dft, seed=11):
    g = np.random.default_rng(seed)
    for n in (2, 3, 5, 6, 7, 10, 12, 14, 17, 31, 64, 96, 160, 224, 509, 1000, 3584, 4096):
        x = g.uniform(-1, 1, (2, n)) + 1j * g.uniform(-1, 1, (2, n))
        for sign, ref in ((FWD, np.fft.fft(x, axis=1)), (INV, n * np.fft.ifft(x, axis=1))):
            y = dft(x, sign)
            err = np.linalg.norm(y - ref, axis=1) / np.linalg.norm(ref, axis=1)
            assert err.max() < 5e-15, (n, sign, err.max())


ALL_PINS = [pin_dft4_equals_eq1, pin_listing1, pin_small_closed_forms,
            pin_delta_and_constant, pin_shifted_delta_and_tone, pin_invariants,
            pin_numpy]
