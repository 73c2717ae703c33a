"""Split-precision MFMA plans (DFT_16 stages on the matrix cores) against the
FP64 oracle.  Their error is reported rather than gated by the complex64
tolerance; the bounds here are loose enough for each mode's arithmetic and
tight enough that any operand-layout or indexing mistake (an O(1) error)
fails."""
import numpy as np
import pytest

import oracle
from gpu_util import rel_l2, run_plan, say
from paper_2207_06803_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2207_06803_amd import fftc  # noqa: E402

# mode -> bound on the max per-transform relative L2 error (Gaussian inputs)
BOUNDS = {"split_f16": 1e-6, "split_bf16": 4e-5, "split3_bf16": 1e-6, "f16": 4e-3}
SIZES = [256, 512, 1024, 2048, 4096, 8192, 16384]


@pytest.mark.parametrize("mode", sorted(BOUNDS))
def test_split_modes_against_oracle(mode):
    rows = []
    for n in SIZES:
        b = 5 if n <= 4096 else 3
        x = synth.gaussian_complex(synth.rng(4, n, len(mode)), (b, n), np.complex64)
        for d in (fftc.FORWARD, fftc.INVERSE):
            with fftc.Plan(n, b, d, mode) as p:
                desc = p.describe()
                assert desc["variant"] == "split_mfma"
                y = run_plan(p, x)
            err = rel_l2(y, oracle.dft(x, d))
            rows.append((n, d, err.max()))
            say(f"{mode} n={n} dir={d} max rel L2 {err.max():.3e} radices {desc['radices']}")
            assert err.max() <= BOUNDS[mode], (mode, n, d, err.max())


def test_split_more_accurate_than_plain_f16_and_close_to_c64():
    n, b = 4096, 6
    x = synth.gaussian_complex(synth.rng(4, 1), (b, n), np.complex64)
    ref = oracle.dft(x)
    errs = {}
    for mode in ("c64", "split_f16", "split_bf16", "split3_bf16", "f16"):
        with fftc.Plan(n, b, fftc.FORWARD, mode) as p:
            errs[mode] = rel_l2(run_plan(p, x), ref).max()
    say("errors at n=4096:", errs)
    assert errs["split_f16"] < errs["f16"] / 50
    assert errs["split3_bf16"] < errs["split_bf16"]
    assert errs["split_f16"] < 20 * errs["c64"]


def test_split_ragged_batch_and_inplace():
    n, b = 1024, 37
    x = synth.gaussian_complex(synth.rng(4, 2), (b, n), np.complex64)
    with fftc.Plan(n, b, fftc.FORWARD, "split_f16") as p:
        y1 = run_plan(p, x)
        y2 = run_plan(p, x, inplace=True)
    assert np.array_equal(y1, y2)
    assert rel_l2(y1, oracle.dft(x)).max() <= BOUNDS["split_f16"]


def test_split_unsupported_lengths():
    for n in (64, 3072, 32768):
        with pytest.raises(fftc.FFTCError) as e:
            fftc.Plan(n, 1, fftc.FORWARD, "split_f16")
        assert e.value.status == 2


@pytest.mark.parametrize("n", [1024, 4096, 16384])
def test_split_modes_at_benchmark_batch(n):
    """Batch 8192, the precision study's launch: the study's Gaussian input,
    every mode, checked on sampled transforms (always the first and the last)
    against the FP64 oracle."""
    b = 8192
    x = synth.gaussian_complex(synth.rng(4, n), (b * n,), np.complex64)
    g = synth.rng(4, n, 98)
    rows = np.unique(np.concatenate([[0, 1, b // 2, b - 1], g.choice(b, 4, replace=False)]))
    ref = oracle.dft(x.reshape(b, n)[rows])
    xd = torch.from_numpy(x).to("cuda")
    del x
    yd = torch.empty_like(xd)
    rows_d = torch.from_numpy(rows).to("cuda")
    for mode in sorted(BOUNDS):
        say(f"{mode} n={n} batch={b}")
        with fftc.Plan(n, b, fftc.FORWARD, mode) as p:
            p.execute(xd, yd)
            torch.cuda.synchronize()
        got = yd.view(b, n).index_select(0, rows_d).cpu().numpy()
        err = rel_l2(got, ref)
        say(f"  sampled rows {rows.tolist()}: max rel L2 {err.max():.3e} mean {err.mean():.3e}")
        assert err.max() <= BOUNDS[mode], (mode, n, err.max())
    del xd, yd
    torch.cuda.empty_cache()
