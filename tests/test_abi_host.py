"""The C-ABI library on the CPU: it loads, exports every declared symbol, and
its host-only planner emits factorisations that multiply to DFT_N."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import factor_algebra as F
from paper_2207_06803_amd import fftc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(fftc_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("fftc_plan", "fftc_execute", "fftc_destroy_plan", "fftc_status_string",
                 "fftc_last_error", "fftc_factorize"):
        assert must in names


@pytest.mark.parametrize("name", declared_functions())
def test_library_exports_symbol(name):
    lib = ctypes.CDLL(fftc.LIB_PATH)
    assert hasattr(lib, name), name


def test_status_strings():
    for code, text in fftc.STATUS.items():
        assert fftc.status_string(code) == text


SIZES = sorted({1 << k for k in range(1, 15)} | {3 << k for k in range(0, 10)} |
               {5 << k for k in range(0, 10)} | {7 << k for k in range(0, 10)} | {9, 15, 21, 35, 105, 225})


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_factorize_products(dtype):
    for n in SIZES:
        if n > fftc.max_single_n(dtype):
            continue
        rs, m = fftc.factorize(n, dtype)
        assert m == 0
        assert int(np.prod(rs)) == n, (n, rs)
        assert all(r in (2, 3, 4, 5, 7, 8, 16) for r in rs)


@pytest.mark.parametrize("n", [n for n in SIZES if 1 < n <= 256])
def test_planner_lists_multiply_to_dft(n):
    rs, _ = fftc.factorize(n, "c64")
    got = F.stockham_product(n, rs)
    assert np.abs(got - F.dft_matrix(n)).max() < 1e-11, (n, rs)


def test_two_pass_split():
    # lengths past the single-kernel limit without a compiled wide list,
    # including 7-smooth lengths below the complex64 wide length
    for n in (3 * 8192, 5 * 4096, 7 * 4096, 65536, 1 << 18, 1 << 20, 3 * 16384, 7 * 4096 * 2):
        rs, m = fftc.factorize(n, "c64")
        assert m > 0 and n % m == 0 and m <= 1024 and n // m <= 1024, (n, m)
        assert int(np.prod(rs)) == n
    for n in (3 * 4096, 32768):
        rs, m = fftc.factorize(n, "c128")
        assert m > 0


WIDE = {"c64": 32768, "c128": 16384}


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_wide_length_is_one_kernel(dtype):
    """complex64 32768 and complex128 16384 (past fftc_max_single_n) run as
    one kernel with their first compiled wide list; a list that is not
    compiled for them is refused on the host."""
    n = WIDE[dtype]
    assert n > fftc.max_single_n(dtype)
    wide = [tuple(rs) for m, rs in fftc.compiled_lists(dtype) if m == n]
    assert len(wide) == 3 and all(int(np.prod(rs)) == n and len(rs) == 4 for rs in wide)
    # the wide entries come last in the compiled list
    assert [m for m, _ in fftc.compiled_lists(dtype)][-3:] == [n] * 3
    rs, m = fftc.factorize(n, dtype)
    assert m == 0 and tuple(rs) == wide[0]
    bads = ([8, 8, 8, 8, 8], [2, 16, 16, 16, 4]) if dtype == "c64" else ([4, 4, 4, 16, 16], [2, 8, 16, 16, 4])
    for bad in bads:
        assert int(np.prod(bad)) == n
        with pytest.raises(fftc.FFTCError) as e:
            fftc.Plan(n, 2, radices=bad, dtype=dtype)
        assert e.value.status == 2 and "compiled radix lists" in str(e.value)


@pytest.mark.parametrize("n", [0, -4, 11, 13 * 4, (1 << 20) * 2, 3 ** 13])
def test_unsupported_sizes_rejected_on_host(n):
    with pytest.raises(fftc.FFTCError) as e:
        fftc.Plan(n, 4)
    assert e.value.status == 2
    with pytest.raises(fftc.FFTCError):
        fftc.factorize(n)


def test_bad_arguments_rejected_on_host():
    with pytest.raises(fftc.FFTCError) as e:
        fftc.Plan(64, 0)
    assert e.value.status == 1 and "batch" in fftc.last_error()
    with pytest.raises(fftc.FFTCError) as e:
        fftc.Plan(64, 1, direction=0)
    assert e.value.status == 1
    h = ctypes.c_void_p()
    assert fftc.lib.fftc_plan(64, 1, -1, 7, ctypes.byref(h)) == 1 and not h.value
    assert fftc.lib.fftc_plan(64, 1, -1, 0, None) == 1
    with pytest.raises(fftc.FFTCError) as e:
        fftc.Plan(64, 1, radices=[4, 4, 2])
    assert e.value.status == 1
    with pytest.raises(fftc.FFTCError) as e:
        fftc.Plan(64, 1, radices=[64])
    assert e.value.status == 1
    # the copy reference checks its arguments before any launch
    assert fftc.lib.fftc_copy(None, None, 0, None) == 0
    assert fftc.lib.fftc_copy(1 << 20, (1 << 20) + 8, 16, None) == 1   # 8-byte aligned out
    assert fftc.lib.fftc_copy(1 << 20, 2 << 20, 24, None) == 1          # not a multiple of 16
    assert fftc.lib.fftc_copy(1 << 20, (1 << 20) + 16, 64, None) == 1   # overlapping ranges
    assert fftc.lib.fftc_copy(None, 1 << 20, 16, None) == 1
    # NULL plan
    assert fftc.lib.fftc_execute(None, None, None, None) == 1
    assert fftc.lib.fftc_destroy_plan(None) == 0


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_compiled_lists_are_valid_factorisations(dtype):
    lists = fftc.compiled_lists(dtype)
    assert len(lists) > 100
    seen = set()
    for n, rs in lists:
        assert int(np.prod(rs)) == n and all(r in (2, 3, 4, 5, 7, 8, 16) for r in rs)
        assert (n, tuple(rs)) not in seen
        seen.add((n, tuple(rs)))
    # every length of the mixed-size workload has its preferred list compiled
    from paper_2207_06803_amd import synth
    for n in synth.mixed_size_set():
        assert (n, tuple(fftc.candidates(n)[0])) in seen, n


def test_compiled_lists_multiply_to_dft_small():
    for n, rs in fftc.compiled_lists("c64"):
        if n <= 128:
            assert np.abs(F.stockham_product(n, rs) - F.dft_matrix(n)).max() < 1e-11, (n, rs)


def test_binding_refuses_host_and_strided_tensors():
    """The binding's buffer checks run before any library call: a host tensor
    and a non-contiguous device view are refused (the kernels would take a host
    address, or ignore the view's strides)."""
    import torch

    class FakeDeviceTensor:  # a device view as far as the checks can see
        def __init__(self, contiguous, nbytes, index=0):
            self.device = torch.device("cuda", index)
            self._c, self.nbytes = contiguous, nbytes

        def is_contiguous(self):
            return self._c

    with pytest.raises(fftc.FFTCError) as e:
        fftc.check_extent(torch.zeros(16, dtype=torch.complex64), 128, "input")
    assert e.value.status == 1 and "not on a GPU" in str(e.value)
    with pytest.raises(fftc.FFTCError):
        fftc.check_extent(FakeDeviceTensor(False, 1 << 20), 128, "input")
    with pytest.raises(fftc.FFTCError):
        fftc.check_extent(FakeDeviceTensor(True, 120), 128, "input")
    with pytest.raises(fftc.FFTCError):
        fftc.check_extent(FakeDeviceTensor(True, 128, index=1), 128, "input", device=0)
    fftc.check_extent(FakeDeviceTensor(True, 128), 128, "input", device=0)
    with pytest.raises(fftc.FFTCError):
        fftc.copy(torch.zeros(4, dtype=torch.complex64), torch.zeros(4, dtype=torch.complex64), 32)
