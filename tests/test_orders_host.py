"""Alternative factorisation orders on the host: the compiled set, argument
checks, and order-tagged lines of the tuning database."""
import ctypes
import os

import pytest

from paper_2207_06803_amd import fftc


def test_compiled_orders():
    for dt in ("c64", "c128"):
        got = fftc.compiled_orders(dt)
        want = {(n, o, r) for n, r in [(64, 2), (64, 4), (64, 8), (256, 2), (256, 4), (256, 16), (1024, 2),
                                        (1024, 4), (4096, 2), (4096, 4), (4096, 8), (4096, 16)]
                for o in (fftc.ORDER_CT, fftc.ORDER_PEASE, fftc.ORDER_FOURSTEP)}
        want.add((256, fftc.ORDER_WAVE, 16))       # the in-wave exchange: N = 256 only
        assert set(got) == want
        for n, _, r in got:
            m = n
            while m % r == 0:
                m //= r
            assert m == 1, (n, r)


def _plan_status(n, order, radix, dtype="c64", batch=1, direction=fftc.FORWARD):
    h = ctypes.c_void_p()
    st = fftc.lib.fftc_plan_order(n, batch, direction, fftc.dtype_code(dtype), order, radix, ctypes.byref(h))
    assert not h.value
    return st


def test_plan_order_errors():
    assert _plan_status(1024, 0, 2) == 1          # Stockham goes through fftc_plan
    assert _plan_status(1024, 7, 2) == 1          # no such order
    assert _plan_status(1024, fftc.ORDER_WAVE, 16) == 2  # the in-wave exchange is compiled for N = 256 only
    assert _plan_status(1024, fftc.ORDER_CT, 16) == 2   # 1024 is not a power of 16
    assert _plan_status(2048, fftc.ORDER_PEASE, 2) == 2  # not compiled
    assert _plan_status(1024, fftc.ORDER_CT, 2, dtype="split_f16") == 1
    assert _plan_status(1024, fftc.ORDER_CT, 2, batch=0) == 1
    assert _plan_status(1024, fftc.ORDER_CT, 2, direction=0) == 1


def test_tuning_db_order_lines(tmp_path):
    fftc.tune_clear()
    src = tmp_path / "in.txt"
    key = fftc.tune_key()
    src.write_text(f"{key} c64 1024 pease:4,4,4,4,4 0.05\n"
                   f"{key} c64 256 foo:2,2,2,2,2,2,2,2 0.1\n"      # unknown order
                   f"{key} c64 4096 ct:4,4 0.1\n"                  # does not multiply to n
                   f"{key} c64 512 ct:2,2,2,2,2,2,2,2,2 0.1\n"     # not compiled
                   f"{key} c128 64 ct:8,8 0.01\n"
                   f"{key} c128 4096 fourstep:16,16,16 0.03\n"
                   f"{key} c64 256 16,16 0.02\n")
    try:
        assert fftc.tune_load(str(src)) == 4
        out = tmp_path / "out.txt"
        assert fftc.tune_save(str(out)) == 4
        text = out.read_text()
        assert "c64 1024 pease:4,4,4,4,4" in text and "c128 64 ct:8,8" in text and "c64 256 16,16" in text
        assert "c128 4096 fourstep:16,16,16" in text
        # an order entry is not a Stockham list: the planner's own choice stays
        assert fftc.factorize(1024)[0] == fftc.candidates(1024)[0]
        assert fftc.factorize(256)[0] == [16, 16]
    finally:
        fftc.tune_clear()


def _fourstep_replay(x, n, r):
    """The four-step order's steps in NumPy (Eq. 2 once, N = K M with
    M = R^ceil(t/2), K = R^floor(t/2)): Pi^N_K as the load address, radix-R
    Stockham stages on the K rows, D^N_M with the first column stage, radix-R
    Stockham stages on the M stride-M columns."""
    import numpy as np
    t = round(np.log(n) / np.log(r))
    tk = t // 2
    tm = t - tk
    m, k = r ** tm, r ** tk
    w = np.exp(-2j * np.pi * np.arange(n) / n)
    dft_r = np.exp(-2j * np.pi * np.outer(np.arange(r), np.arange(r)) / r)
    a = np.empty(n, complex)
    e = np.arange(n)
    a[(e % k) * m + e // k] = x
    for s in range(t):
        b = np.empty(n, complex)
        if s < tm:  # rows: stage s of DFT_M, ns = R^s
            ns, mr = r ** s, m // r
            bf = np.arange(n // r)
            row, j = bf // mr, bf % mr
            kk = j % ns
            v = np.stack([a[row * m + j + q * mr] for q in range(r)])
            if s:
                v = v * np.stack([w[q * kk * (n // (ns * r))] for q in range(r)])
            v = dft_r @ v
            for q in range(r):
                b[row * m + (j // ns) * ns * r + q * ns + kk] = v[q]
        else:  # columns: stage s - tm of DFT_K; the first applies D^N_M
            ns, kr = r ** (s - tm), k // r
            bf = np.arange(n // r)
            j, p = bf // m, bf % m
            kk = j % ns
            v = np.stack([a[(j + q * kr) * m + p] for q in range(r)])
            if s == tm:
                v = v * np.stack([w[(j + q * kr) * p] for q in range(r)])
            else:
                v = v * np.stack([w[q * kk * (n // (ns * r))] for q in range(r)])
            v = dft_r @ v
            for q in range(r):
                b[((j // ns) * ns * r + q * ns + kk) * m + p] = v[q]
        a = b
    return a


@pytest.mark.parametrize("n,r", [(64, 2), (64, 4), (64, 8), (256, 2), (256, 4), (256, 16), (1024, 2), (1024, 4),
                                 (4096, 8), (4096, 16)])
def test_fourstep_order_steps_are_a_dft(n, r):
    import numpy as np
    g = np.random.default_rng(n + r)
    x = g.standard_normal(n) + 1j * g.standard_normal(n)
    want = np.fft.fft(x)
    assert np.abs(_fourstep_replay(x, n, r) - want).max() <= 1e-12 * np.abs(want).max()
