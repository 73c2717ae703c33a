"""Formula plans on the GPU against the formula oracle (oracle/formula.py)
and the FP64 DFT oracle: every pass kind, both execution paths (one
LDS-resident kernel, one HBM kernel per pass), both directions, ragged
batches, in place, and folded formulas."""

import numpy as np
import pytest

import oracle
import oracle.formula as of
from gpu_util import np_dtype, rel_l2, say, tol_for
from paper_2207_06803_amd import formulas, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2207_06803_amd import fftc  # noqa: E402

FWD, INV = fftc.FORWARD, fftc.INVERSE
NO_FOLD, EQ2, HBM = fftc.FORMULA_NO_FOLD, fftc.FORMULA_EQ2, fftc.FORMULA_HBM_PASSES


def run(plan, x, inplace=False):
    xd = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    yd = xd if inplace else torch.empty_like(xd)
    plan.execute(xd, yd)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


def tol(text, dim, dtype):
    # the stated bounds, also for sizes with a prime factor above 7 that are
    # summed directly (an fp32 sum of s terms errs by about sqrt(s) eps, so
    # DFT(127) sits near 1e-6, inside its 7e-6 bound)
    return tol_for(dim, dtype)


FORMULAS = [
    formulas.recursive_ct(4),
    formulas.recursive_ct(64, (2,)),
    formulas.recursive_ct(48, (4, 3)),
    formulas.recursive_dif(40, (5, 2)),
    formulas.recursive_ct(1024, (4,)),
    formulas.dft2d(8, 12),
    formulas.dft2d(64, 64),
    formulas.four_step_no_transpose(8, 16),
    "DFT(22)", "DFT(13) ⊗ I(3)", "I(2) ⊗ DFT(26) ⊗ I(2)", "DFT(96)", "DFT(11) ⊗ DFT(7)",
    "DFT(16) ⊗ DFT(3) ⊗ DFT(5) ⊗ DFT(7)",
    "Permute(24, 4) · (I(4) ⊗ twiddle(6, 2)) · (DFT(4) ⊗ I(6))",
    "(DFT(2) ⊗ Permute(6, 2)) · (twiddle(6, 3) ⊗ I(2)) · (I(3) ⊗ DFT(4))",
    "I(5)", "twiddle(36, 6) · Permute(36, 6)", "DFT(127)",
]


@pytest.mark.parametrize("flags", [NO_FOLD, NO_FOLD | EQ2, NO_FOLD | HBM, NO_FOLD | EQ2 | HBM])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("text", FORMULAS)
def test_formula_vs_oracle(text, dtype, flags):
    dim = of.size(of.parse(text))
    b = 5 if dim <= 4096 else 2
    x = synth.uniform_complex(synth.rng(120, dim % 1009, flags), (b, dim), np_dtype(dtype))
    for d in (FWD, INV):
        say(f"formula {text[:60]!r} dim={dim} {dtype} flags={flags} dir={d}")
        with fftc.plan_formula(text, b, d, dtype, flags) as p:
            desc = p.describe()
            assert desc["variant"] == "formula" and desc["n"] == dim
            assert desc["formula_lds"] == (not (flags & HBM) and dim <= fftc.formula_max_lds_dim(dtype))
            if flags & HBM:
                assert desc["formula_kernels"] == desc["formula_passes"], desc
            y = run(p, x)
            y_in = run(p, x, inplace=True)
        want = of.apply(text, x, d)
        err = rel_l2(y, want)
        say(f"  max rel L2 {err.max():.3e} (bound {tol(text, dim, dtype):.1e})")
        assert err.max() <= tol(text, dim, dtype), (err.max(), desc)
        assert np.array_equal(y, y_in)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_listing1_program(dtype):
    # createComplex([1,2,3,4], [1,2,3,4]) through the Listing 1 formula: small
    # integers, every operation exact in either precision
    text = formulas.recursive_ct(4) + " · InputComplex"
    x = np.array([[1 + 1j, 2 + 2j, 3 + 3j, 4 + 4j]], dtype=np_dtype(dtype))
    for flags in (0, NO_FOLD, NO_FOLD | HBM):
        with fftc.plan_formula(text, 1, FWD, dtype, flags) as p:
            assert p.describe()["formula_folded"] == (flags == 0)
            y = run(p, x)
        assert np.array_equal(y[0], np.array([10 + 10j, -4, -2 - 2j, -4j])), (flags, y)


@pytest.mark.parametrize("n,rs,dtype", [(1024, (2,), "c64"), (4096, (4,), "c64"), (256, (2,), "c128"),
                                        (3 * 5 * 7 * 8, (8, 7, 5, 3), "c64"), (32768, (8,), "c64")])
def test_folded_recursive_ct_runs_the_plan(n, rs, dtype):
    b = 3
    x = synth.uniform_complex(synth.rng(121, n % 997), (b, n), np_dtype(dtype))
    for text in (formulas.recursive_ct(n, rs), formulas.recursive_dif(n, rs)):
        for d in (FWD, INV):
            with fftc.plan_formula(text, b, d, dtype) as p:
                desc = p.describe()
                assert desc["formula_folded"] and desc["formula_fold_n"] == n and desc["formula_fold_p"] == 1
                y = run(p, x)
            with fftc.Plan(n, b, d, dtype) as q:
                y_plan = run(q, x)
            assert np.array_equal(y, y_plan)
            assert rel_l2(y, oracle.dft(x, d)).max() <= tol_for(n, dtype)


def test_folded_batched_identity_kron():
    n, p_, b = 512, 6, 4
    text = f"I({p_}) ⊗ ({formulas.recursive_ct(n, (8,))})"
    x = synth.uniform_complex(synth.rng(122), (b, p_ * n), np.complex64)
    with fftc.plan_formula(text, b, FWD, "c64") as p:
        desc = p.describe()
        assert desc["formula_folded"] and desc["formula_fold_p"] == p_
        y = run(p, x)
    want = oracle.dft(x.reshape(b * p_, n)).reshape(b, p_ * n)
    assert rel_l2(y, want).max() <= tol_for(n, "c64")


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_hbm_path_beyond_lds(dtype):
    # 128 x 128 2-D DFT (16384 > the LDS limit) and a 2^16 Eq. 2 program without folding
    for text in (formulas.dft2d(128, 128), formulas.recursive_ct(1 << 16, (16,))):
        dim = of.size(of.parse(text))
        x = synth.uniform_complex(synth.rng(123, dim % 1013), (2, dim), np_dtype(dtype))
        for flags in (NO_FOLD, NO_FOLD | EQ2):
            with fftc.plan_formula(text, 2, FWD, dtype, flags) as p:
                desc = p.describe()
                assert not desc["formula_lds"] and desc["scratch_bytes"] == 2 * dim * x.itemsize
                if text.startswith("DFT(128)"):
                    # rows then columns: two LDS runs of 128-element sub-vectors
                    assert desc["formula_kernels"] == 2, desc
                assert desc["formula_kernels"] < desc["formula_passes"], desc
                y = run(p, x)
                y_in = run(p, x, inplace=True)
            if text.startswith("DFT(128)"):
                want = of.apply(text, x)
            else:
                want = oracle.dft(x)
            assert rel_l2(y, want).max() <= tol_for(dim, dtype), (text[:40], flags)
            assert np.array_equal(y, y_in)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_runs_of_strided_subvectors(dtype):
    # vectors beyond the LDS limit whose passes group into runs with inner
    # strides Q0 that are not multiples of 16 (tile columns Cc < 16)
    cap = fftc.formula_max_lds_dim(dtype)
    for text in ("DFT(2048) ⊗ DFT(12)", "DFT(24) ⊗ DFT(1536)", "(DFT(9) ⊗ I(3000)) · (I(9) ⊗ DFT(3000))",
                 "DFT(5) ⊗ I(7) ⊗ DFT(600)"):
        dim = of.size(of.parse(text))
        assert dim > cap
        b = 3
        x = synth.uniform_complex(synth.rng(126, dim % 1019), (b, dim), np_dtype(dtype))
        for d in (FWD, INV):
            say(f"runs {text} {dtype} dir={d}")
            with fftc.plan_formula(text, b, d, dtype, NO_FOLD) as p:
                desc = p.describe()
                assert 1 < desc["formula_kernels"] < desc["formula_passes"], desc
                y = run(p, x)
                y_in = run(p, x, inplace=True)
                xd = torch.from_numpy(x).cuda()
                yd = torch.zeros_like(xd)
                p.execute_batch(xd, yd, 1)
                torch.cuda.synchronize()
                y1 = yd.cpu().numpy()
            want = of.apply(text, x, d)
            assert rel_l2(y, want).max() <= tol(text, dim, dtype), text
            assert np.array_equal(y, y_in)
            assert np.array_equal(y1[0], y[0]) and not y1[1:].any()


def test_partial_batches_and_ragged_tiles():
    # dim 12: 341 vectors per LDS tile; batches that end mid-tile
    text = "Permute(12, 3) · (I(3) ⊗ DFT(4)) · twiddle(12, 4) · (DFT(3) ⊗ I(4))"
    b = 1000
    x = synth.uniform_complex(synth.rng(124), (b, 12), np.complex64)
    want = of.apply(text, x)
    with fftc.plan_formula(text, b, FWD, "c64", NO_FOLD) as p:
        for nb in (1, 340, 341, 342, 999, 1000):
            xd = torch.from_numpy(x[:nb].copy()).cuda()
            yd = torch.full_like(xd, complex(7, 7))
            p.execute_batch(xd, yd, nb)
            torch.cuda.synchronize()
            y = yd.cpu().numpy()
            assert rel_l2(y, want[:nb]).max() <= tol_for(12, "c64"), nb


def test_determinism():
    text = formulas.dft2d(64, 64)
    x = synth.uniform_complex(synth.rng(125), (8, 4096), np.complex64)
    with fftc.plan_formula(text, 8, FWD, "c64", NO_FOLD) as p:
        y0 = run(p, x)
        y1 = run(p, x)
    with fftc.plan_formula(text, 3, FWD, "c64", NO_FOLD) as p:
        y2 = run(p, x[:3])
    assert np.array_equal(y0, y1) and np.array_equal(y0[:3], y2)


def test_plan_errors():
    with pytest.raises(fftc.FFTCError):
        fftc.plan_formula("DFT(4) · DFT(2)", 1)
    with pytest.raises(fftc.FFTCError):
        fftc.plan_formula("DFT(4)", 0)
    with pytest.raises(fftc.FFTCError):
        fftc.plan_formula("DFT(1048576) ⊗ I(2)", 1 << 11)  # batch * dim >= 2^31


@pytest.mark.parametrize("text,flags", [
    (formulas.recursive_ct(1024, (2,)), NO_FOLD),
    (formulas.recursive_ct(1024, (16, 4)), NO_FOLD),
    ("DFT(1024)", NO_FOLD | EQ2),
    (formulas.dft2d(64, 64), 0),
    (formulas.dft2d(128, 128), 0),
    (formulas.dft2d(1024, 1024), 0),
], ids=["rct1024_r2_as_written", "rct1024_r16_as_written", "dft1024_eq2", "dft2d_64", "dft2d_128", "dft2d_1024"])
def test_full_size_sampled(text, flags):
    # the launch the benchmark times (2^24 complex64 elements); sampled vectors
    # (first, middle, last) against the formula oracle
    dim = of.size(of.parse(text))
    b = (1 << 24) // dim
    g = synth.rng(127, dim % 1021, flags)
    x = synth.uniform_complex(g, (b, dim), np.complex64)
    say(f"full size {text[:50]!r} dim={dim} batch={b}")
    with fftc.plan_formula(text, b, FWD, "c64", flags) as p:
        y = run(p, x)
    rows = sorted({0, b // 2, b - 1})
    want = of.apply(text, x[rows])
    err = rel_l2(y[rows], want)
    assert err.max() <= tol(text, dim, "c64"), err
