"""Seeded synthetic inputs for the batched-FFT workloads.

This module only draws numbers: it holds none of the transform's arithmetic,
and it is the one piece of code that both the GPU path's tests/benchmarks and
the CPU oracle's callers share.  Values are drawn in float64 and rounded to the
run's precision, so the oracle can be handed exactly the values the GPU sees.

Workload recipes (the paper only says "random input vectors", Section VI):
  * plain batched transforms: re and im i.i.d. uniform[-1, 1)
  * precision study: re and im i.i.d. standard Gaussian
  * mixed sizes: 37 lengths (powers of two 8..4096 and 3*2^k, 5*2^k, 7*2^k up
    to 3584), each transform's length drawn uniformly over the 37
  * serving: Poisson arrivals, batch uniform in [1, 256], length uniform over
    the 11 powers of two 2^6..2^16, direction forward/inverse with p = 1/2
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 220706803

FORWARD = -1
INVERSE = +1


def rng(config_index: int, *spawn_path: int) -> np.random.Generator:
    """PCG64 generator for a workload, optionally for a spawned sub-case."""
    ss = np.random.SeedSequence(BASE_SEED + int(config_index))
    for idx in spawn_path:
        ss = ss.spawn(int(idx) + 1)[int(idx)]
    return np.random.Generator(np.random.PCG64(ss))


def _as_complex(re: np.ndarray, im: np.ndarray, dtype) -> np.ndarray:
    dtype = np.dtype(dtype)
    if dtype == np.complex64:
        out = np.empty(re.shape, np.complex64)
        out.real = re.astype(np.float32)
        out.imag = im.astype(np.float32)
        return out
    if dtype == np.complex128:
        return re + 1j * im
    raise ValueError(f"unsupported dtype {dtype}")


def uniform_complex(g: np.random.Generator, shape, dtype=np.complex64) -> np.ndarray:
    """re and im i.i.d. uniform[-1, 1), drawn in float64, rounded to dtype."""
    re = g.uniform(-1.0, 1.0, size=shape)
    im = g.uniform(-1.0, 1.0, size=shape)
    return _as_complex(re, im, dtype)


def gaussian_complex(g: np.random.Generator, shape, dtype=np.complex64) -> np.ndarray:
    """re and im i.i.d. N(0, 1), drawn in float64, rounded to dtype."""
    re = g.standard_normal(size=shape)
    im = g.standard_normal(size=shape)
    return _as_complex(re, im, dtype)


def mixed_size_set() -> list[int]:
    """The 37 lengths of the mixed-size workload, ascending."""
    s = {1 << k for k in range(3, 13)}                 # 8 .. 4096
    s |= {3 << k for k in range(2, 11)}                # 12 .. 3072
    s |= {5 << k for k in range(1, 10)}                # 10 .. 2560
    s |= {7 << k for k in range(1, 10)}                # 14 .. 3584
    return sorted(s)


def draw_mixed_sizes(g: np.random.Generator, count: int) -> np.ndarray:
    """Lengths drawn uniformly over the 37-member set (int64)."""
    sizes = np.asarray(mixed_size_set(), dtype=np.int64)
    return sizes[g.integers(0, len(sizes), size=count)]


def serving_requests(g: np.random.Generator, count: int, rate_per_s: float,
                     min_log2: int = 6, max_log2: int = 16, max_batch: int = 256):
    """Open-loop request stream.

    Returns a dict of arrays: arrival_s (cumulative exponential gaps at
    `rate_per_s`), n, batch, direction (-1 forward / +1 inverse).
    """
    gaps = g.exponential(1.0 / rate_per_s, size=count)
    arrival = np.cumsum(gaps) - gaps[0]
    n = np.left_shift(1, g.integers(min_log2, max_log2 + 1, size=count)).astype(np.int64)
    batch = g.integers(1, max_batch + 1, size=count).astype(np.int64)
    direction = np.where(g.random(count) < 0.5, FORWARD, INVERSE).astype(np.int32)
    return {"arrival_s": arrival, "n": n, "batch": batch, "direction": direction}
