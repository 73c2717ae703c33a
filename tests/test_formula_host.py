"""Formula front end on the host (no GPU): parsing, the shape rule, Eq. 2
folding and the lowering to passes.

The lowering is checked by replaying the pass list that
fftc_formula_lower prints with a small NumPy interpreter of the pass
semantics (written here from the pass definitions, not from the kernels) and
comparing with the formula oracle.
"""
import numpy as np
import pytest

import oracle.formula as of
from paper_2207_06803_amd import fftc, formulas

NO_FOLD, EQ2, HBM = fftc.FORMULA_NO_FOLD, fftc.FORMULA_EQ2, fftc.FORMULA_HBM_PASSES


def lower(text, flags=0, dtype="c64"):
    return fftc.formula_lower(text, flags, dtype)


def _fields(line):
    kind, *kv = line.split()
    return kind, {k: int(v) for k, v in (t.split("=") for t in kv)}


def replay(desc, x):
    """Apply the printed pass list to the rows of x."""
    lines = desc.strip().splitlines()
    assert lines[0].startswith("dim ") and lines[1].startswith("formula ")
    y = np.array(x, dtype=np.complex128)
    rows, dim = y.shape
    for line in lines[2:]:
        kind, f = _fields(line)
        if kind == "copy":
            continue
        n, p, q = f["n"], f["p"], f["q"]
        assert p * n * q == dim, line
        v = y.reshape(rows, p, n, q)
        t = np.arange(n)
        if kind in ("dft", "direct"):
            v = np.fft.fft(v, axis=2)
        elif kind == "diag":
            M = f["M"]
            v = v * np.exp(-2j * np.pi * ((t // M) * (t % M) % n) / n)[None, None, :, None]
        elif kind == "perm":
            K = f["K"]
            M = n // K
            v = v[:, :, (t % M) * K + t // M, :]
        elif kind == "stage":
            r, ns = f["r"], f["ns"]
            nr = n // r
            out = np.empty_like(v)
            j = np.arange(nr)
            k = j % ns
            vals = [v[:, :, j + s * nr, :] * np.exp(-2j * np.pi * s * k / (ns * r))[None, None, :, None]
                    for s in range(r)]
            for m in range(r):  # DFT_r over s
                acc = sum(vals[s] * np.exp(-2j * np.pi * s * m / r) for s in range(r))
                out[:, :, (j // ns) * ns * r + m * ns + k, :] = acc
            v = out
        else:
            raise AssertionError(line)
        y = np.ascontiguousarray(v).reshape(rows, dim)
    return y


FORMULAS = [
    formulas.recursive_ct(4),
    formulas.recursive_ct(64, (2,)),
    formulas.recursive_ct(48, (4, 3)),
    formulas.recursive_dif(40, (5, 2)),
    formulas.dft2d(8, 12),
    formulas.four_step_no_transpose(8, 16),
    "DFT(22)", "DFT(13) ⊗ I(3)", "I(2) ⊗ DFT(26) ⊗ I(2)", "DFT(1024)", "DFT(96)", "DFT(11) ⊗ DFT(7)",
    "Permute(24, 4) · (I(4) ⊗ twiddle(6, 2)) · (DFT(4) ⊗ I(6))",
    "(DFT(2) ⊗ Permute(6, 2)) · (twiddle(6, 3) ⊗ I(2)) · (I(3) ⊗ DFT(4))",
    "I(5)", "twiddle(36, 6) · Permute(36, 6)",
]


@pytest.mark.parametrize("flags", [0, NO_FOLD, NO_FOLD | EQ2])
@pytest.mark.parametrize("text", FORMULAS)
def test_lowering_replays_to_oracle(text, flags):
    dim, desc = lower(text, flags)
    assert dim == of.size(of.parse(text))
    rng = np.random.default_rng(dim)
    x = rng.standard_normal((2, dim)) + 1j * rng.standard_normal((2, dim))
    want = of.apply(text, x)
    if "plan I(" in desc:  # folded: the ordinary plan computes I(p) (x) DFT(n)
        p, n = [int(t.split(")")[0]) for t in desc.split("plan I(")[1].split("DFT(")]
        got = np.fft.fft(x.reshape(2, p, n), axis=2).reshape(2, dim)
    else:
        got = replay(desc, x)
    assert np.abs(got - want).max() < 1e-11 * dim, desc


@pytest.mark.parametrize("n,rs", [(4, (2,)), (8, (2,)), (64, (2,)), (1024, (2,)), (1024, (4,)),
                                  (4096, (16,)), (12, (3, 2)), (3 * 5 * 7 * 8, (8, 7, 5, 3)),
                                  (65536, (16,)), (1 << 20, (2,))])
def test_eq2_programs_fold(n, rs):
    for text in (formulas.recursive_ct(n, rs), formulas.recursive_dif(n, rs)):
        dim, desc = lower(text)
        assert dim == n
        assert f"plan I(1) (x) DFT({n})" in desc, desc
        dim, desc = lower(f"I(3) ⊗ ({text})")
        assert f"plan I(3) (x) DFT({n})" in desc, desc


def test_no_fold_keeps_the_factors():
    _, desc = lower(formulas.recursive_ct(4), NO_FOLD)
    kinds = [ln.split()[0] for ln in desc.strip().splitlines()[2:]]
    assert kinds == ["perm", "dft", "diag", "dft"]
    _, desc = lower("DFT(1024)", NO_FOLD)
    assert [ln.split()[0] for ln in desc.strip().splitlines()[2:]] == ["stage"] * 3
    _, desc = lower("DFT(1024)", NO_FOLD | EQ2)
    kinds = [ln.split()[0] for ln in desc.strip().splitlines()[2:]]
    assert "perm" in kinds and "diag" in kinds and "stage" not in kinds


def test_partial_folds():
    # inner Eq. 2 windows fold even when the whole formula is not a DFT
    text = f"Permute(64, 8) · (I(8) ⊗ ({formulas.recursive_ct(8)}))"
    _, desc = lower(text)
    assert "formula Permute(64, 8) . (I(8) (x) DFT(8))" in desc, desc
    # a window with mismatched sizes does not fold
    _, desc = lower("(DFT(2) ⊗ I(4)) · twiddle(8, 2) · (I(2) ⊗ DFT(4)) · Permute(8, 2)")
    assert "plan" not in desc


@pytest.mark.parametrize("bad", ["DFT(3", "DFT 3", "twiddle(4)", "foo(2)", "DFT(2) ⊗", "(DFT(2)",
                                 "DFT(2) DFT(2)", "I(2) $ I(2)", ""])
def test_syntax_errors(bad):
    with pytest.raises(fftc.FFTCError) as e:
        lower(bad)
    assert e.value.status == 1


@pytest.mark.parametrize("bad", ["DFT(4) · DFT(2)", "twiddle(4, 3)", "Permute(6, 4)", "DFT(0)",
                                 "DFT(4096) ⊗ DFT(8192)", "DFT(2) ⊗ I(2) · twiddle(4,2)"])
def test_shape_errors(bad):
    with pytest.raises(fftc.FFTCError) as e:
        lower(bad)
    assert e.value.status == 1
    assert "formula" in fftc.last_error()


def test_unsupported_direct_size():
    p = 16411  # prime above the direct-sum limit of 16384
    assert all(p % d for d in range(2, 129))
    with pytest.raises(fftc.FFTCError) as e:
        lower(f"DFT({p})")
    assert e.value.status == 2


def test_bad_flags_and_dtype():
    with pytest.raises(fftc.FFTCError):
        fftc.formula_lower("DFT(4)", 64)
    with pytest.raises(fftc.FFTCError):
        fftc.formula_lower("DFT(4)", 0, "split_f16")


def test_lds_limits():
    assert fftc.formula_max_lds_dim("c64") == 9638  # two buffers of L + L / 16 complex64 in 160 KiB
    assert fftc.formula_max_lds_dim("c128") == 4819


def test_generators_text():
    assert formulas.recursive_ct(4) == "(DFT(2) ⊗ I(2)) · twiddle(4, 2) · (I(2) ⊗ DFT(2)) · Permute(4, 2)"
    assert formulas.dft2d(3, 5) == "DFT(3) ⊗ DFT(5)"
