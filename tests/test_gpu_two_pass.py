"""Two-pass (Eq. 2 four-step) plans against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import np_dtype, rel_l2, run_plan, say, tol_for
from paper_2207_06803_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2207_06803_amd import fftc  # noqa: E402

FWD, INV = fftc.FORWARD, fftc.INVERSE


@pytest.mark.parametrize("n,dtype", [(3 * 8192, "c64"), (65536, "c64"), (3 * 16384, "c64"),
                                     (7 * 8192, "c64"), (32768, "c128"), (65536, "c128")])
def test_two_pass_full_oracle(n, dtype):
    b = 3
    x = synth.uniform_complex(synth.rng(93, n % 997), (b, n), np_dtype(dtype))
    for d in (FWD, INV):
        say(f"two-pass n={n} {dtype} dir={d}")
        with fftc.Plan(n, b, d, dtype) as p:
            desc = p.describe()
            assert desc["variant"] == "two_pass" and desc["split_m"] * desc["split_k"] == n, desc
            y = run_plan(p, x)
            y_in = run_plan(p, x, inplace=True)
        err = rel_l2(y, oracle.dft(x, d))
        assert err.max() <= tol_for(n, dtype), (err.max(), desc)
        assert np.array_equal(y, y_in)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_two_pass_2pow20_sampled(dtype):
    n, b = 1 << 20, 2
    g = synth.rng(94, 1 if dtype == "c128" else 0)
    x = synth.uniform_complex(g, (b, n), np_dtype(dtype))
    ks = np.unique(np.r_[0, 1, n // 2, n - 1, g.integers(0, n, 28)])
    for d in (FWD, INV):
        say(f"two-pass n=2^20 {dtype} dir={d}")
        with fftc.Plan(n, b, d, dtype) as p:
            y = run_plan(p, x)
        for row in range(b):
            ref = oracle.dft_points(x[row], ks, d)
            # sampled outputs: error relative to the transform's RMS output size
            scale = np.sqrt(n * (np.abs(x[row].astype(np.complex128)) ** 2).sum())
            err = np.linalg.norm(y[row, ks] - ref) / (scale * np.sqrt(len(ks) / n))
            assert err <= tol_for(n, dtype), err
        ex = (np.abs(x.astype(np.complex128)) ** 2).sum(axis=1) * n
        ey = (np.abs(y.astype(np.complex128)) ** 2).sum(axis=1)
        assert (np.abs(ey - ex) / ex).max() <= 2 * tol_for(n, dtype)


def test_two_pass_batch_and_roundtrip():
    n, b = 65536, 17
    x = synth.uniform_complex(synth.rng(95), (b, n), np.complex64)
    with fftc.Plan(n, b, FWD) as pf, fftc.Plan(n, b, INV) as pi:
        y = run_plan(pf, x)
        z = run_plan(pi, y)
    assert rel_l2(z / n, x).max() <= 2 * tol_for(n, "c64")
    rows = [0, 8, 16]
    assert rel_l2(y[rows], oracle.dft(x[rows])).max() <= tol_for(n, "c64")
