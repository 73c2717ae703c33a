"""FP64 O(N^2) DFT oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The GPU library and its Python binding
never import it, and the two share no code.

`dft` is the paper's definition of the transform (Section II, DFT_N[m,n] =
w_N^{mn}, w_N = exp(-2 pi i/N)) evaluated as a dense matrix-vector product,
one transform per row, by the C library built from `oracle_dft.c`.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        lib.oracle_dft.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                   ctypes.c_int64, ctypes.c_int, ctypes.c_int]
        lib.oracle_dft.restype = ctypes.c_int
        lib.oracle_twiddles.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_void_p]
        lib.oracle_twiddles.restype = ctypes.c_int
        lib.oracle_dft_points.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_int]
        lib.oracle_dft_points.restype = ctypes.c_int
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


FORWARD = -1
INVERSE = +1


def dft(x, sign: int = FORWARD, threads: int = 0) -> np.ndarray:
    """DFT of each row of `x` (shape (n,) or (batch, n)), complex128 out.

    `x` is promoted exactly to complex128 (complex64 inputs keep their fp32
    values).  sign=-1: forward, w_N = exp(-2 pi i/N); sign=+1: inverse with
    w_N^{-1}.  Neither direction is scaled.
    """
    x = np.asarray(x)
    squeeze = x.ndim == 1
    x2 = np.ascontiguousarray(np.atleast_2d(x), dtype=np.complex128)
    if x2.ndim != 2:
        raise ValueError("x must be 1-D or 2-D")
    batch, n = x2.shape
    if n < 1:
        raise ValueError("transform length must be >= 1")
    out = np.empty_like(x2)
    rc = _load().oracle_dft(x2.ctypes.data, out.ctypes.data, n, batch, int(sign), int(threads))
    if rc != 0:
        raise RuntimeError(f"oracle_dft failed with code {rc}")
    return out[0] if squeeze else out


def dft_points(x, ks, sign: int = FORWARD, threads: int = 0) -> np.ndarray:
    """Outputs y[k] for k in `ks` of the DFT of the 1-D vector `x` (complex128)."""
    x = np.ascontiguousarray(np.asarray(x).reshape(-1), dtype=np.complex128)
    ks = np.ascontiguousarray(np.asarray(ks, dtype=np.int64).reshape(-1))
    out = np.empty(len(ks), np.complex128)
    rc = _load().oracle_dft_points(x.ctypes.data, len(x), int(sign), ks.ctypes.data, len(ks),
                                   out.ctypes.data, int(threads))
    if rc != 0:
        raise RuntimeError(f"oracle_dft_points failed with code {rc}")
    return out


def twiddles(n: int, sign: int = FORWARD) -> np.ndarray:
    """The oracle's table exp(sign 2 pi i m / n), m in [0, n)."""
    wr = np.empty(n)
    wi = np.empty(n)
    rc = _load().oracle_twiddles(int(n), int(sign), wr.ctypes.data, wi.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_twiddles failed with code {rc}")
    return wr + 1j * wi


def max_threads() -> int:
    """Threads an oracle call uses by default (OpenMP max threads)."""
    return int(_load().oracle_max_threads())
