"""Layout plans: argument checks on the host (no device call is made before
they pass)."""
import ctypes

import pytest

from paper_2207_06803_amd import fftc

FWD = fftc.FORWARD


def status(n, b, dtype, lin, lout):
    h = ctypes.c_void_p()
    mk = lambda l: None if l is None else ctypes.byref(fftc.Layout(*l))  # noqa: E731
    st = fftc.lib.fftc_plan_layout(n, b, FWD, fftc.dtype_code(dtype), mk(lin), mk(lout), ctypes.byref(h))
    assert not h.value
    return st


@pytest.mark.parametrize("lin", [(0, 64, 0), (1, 0, 0), (1, 64, 2), (1, 63, 0), (2, 100, 1), (3, 1, 0),
                                 (1, 1 << 41, 0)])
def test_bad_layouts(lin):
    assert status(64, 4, "c64", lin, None) == 1
    assert status(64, 4, "c64", None, lin) == 1
    assert "layout" in fftc.last_error()


def test_overlap_rule_edges():
    # one block per transform needs dist >= (n - 1) stride + 1; interleaved needs stride >= batch dist
    assert status(64, 4, "c64", (2, 126, 0), (2, 127, 0)) == 1   # in overlaps
    assert status(64, 4, "c64", (4, 1, 0), (2, 126, 0)) == 1     # out overlaps
    assert status(64, 5, "c64", (4, 1, 0), None) == 1            # 5 columns in a row of 4


def test_unsupported():
    assert status(1, 1, "c64", None, None) == 2
    assert status(11, 1, "c64", None, None) == 2
    assert status(1 << 15, 1, "c64", None, None) == 2   # beyond one kernel: column-like layouts only
    assert status(16384, 1, "c128", None, None) == 2
    assert status(1 << 21, 1, "c64", (1, 1 << 21, 0), (1, 1, 0)) == 2
    assert status(11 * 1024, 4, "c64", (4, 1, 0), None) == 2  # a factor with a prime above 7


def test_bad_dtype_and_execute():
    assert status(64, 1, "split_f16", None, None) == 1
    assert fftc.lib.fftc_execute_layout(None, None, None, None, None, None) == 1
