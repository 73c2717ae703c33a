"""Formula texts for fftc_plan_formula (the DSL of the paper's Section IV-A).

Generators of the Cooley-Tukey programs the paper runs (Section V: recursive
Cooley-Tukey formulas produced by a script, Listing 1 being the 4-point
case) and of a few other Kronecker-product formulas.  Pure text: nothing
here computes a transform.
"""
from __future__ import annotations

KRON = " ⊗ "
MUL = " · "


def _split(n: int, radices) -> int:
    for r in radices:
        if n % r == 0 and r < n:
            return r
    raise ValueError(f"no radix of {list(radices)} splits {n}")


def recursive_ct(n: int, radices=(2,)) -> str:
    """DFT(n) written out by Eq. 2 recursively, down to DFT(r) factors:
        (DFT(K) ⊗ I(M)) · twiddle(n, M) · (I(K) ⊗ <DFT(M)>) · Permute(n, K),
    K = the first radix in `radices` that divides n (and is < n), M = n / K.
    recursive_ct(4) is the formula of Listing 1."""
    if n in radices or n == 1:
        return f"DFT({n})"
    k = _split(n, radices)
    m = n // k
    inner = recursive_ct(m, radices)
    inner = inner if inner.startswith("DFT") else f"({inner})"
    return (f"(DFT({k}){KRON}I({m})){MUL}twiddle({n}, {m}){MUL}(I({k}){KRON}{inner})"
            f"{MUL}Permute({n}, {k})")


def recursive_dif(n: int, radices=(2,)) -> str:
    """The transposed (decimation-in-frequency) form of Eq. 2, recursively:
        Permute(n, M) · (I(K) ⊗ <DFT(M)>) · twiddle(n, M) · (DFT(K) ⊗ I(M))."""
    if n in radices or n == 1:
        return f"DFT({n})"
    k = _split(n, radices)
    m = n // k
    inner = recursive_dif(m, radices)
    inner = inner if inner.startswith("DFT") else f"({inner})"
    return (f"Permute({n}, {m}){MUL}(I({k}){KRON}{inner}){MUL}twiddle({n}, {m})"
            f"{MUL}(DFT({k}){KRON}I({m}))")


def dft2d(rows: int, cols: int) -> str:
    """Two-dimensional DFT of a row-major rows x cols array."""
    return f"DFT({rows}){KRON}DFT({cols})"


def four_step_no_transpose(k: int, m: int) -> str:
    """Eq. 2 for N = k m without the input permutation: DFT_N applied to the
    stride-k reordering of its input (a transform whose input is already
    in the Pi^N_k order)."""
    n = k * m
    return f"(DFT({k}){KRON}I({m})){MUL}twiddle({n}, {m}){MUL}(I({k}){KRON}DFT({m}))"
