"""Alternative factorisation orders (recursive Cooley-Tukey with explicit
digit reversal, Pease constant geometry) against the FP64 oracle, and the
order autotuner with the planner honouring a recorded order."""
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


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_every_compiled_order(dtype):
    for n, order, radix in fftc.compiled_orders(dtype):
        b = 37 if n <= 256 else 5  # ragged last workgroup
        x = synth.uniform_complex(synth.rng(140, n, order, radix), (b, n), np_dtype(dtype))
        for d in (FWD, INV):
            say(f"order n={n} {fftc.ORDER_NAMES[order]} r={radix} {dtype} dir={d}")
            with fftc.plan_order(n, b, d, dtype, order, radix) as p:
                desc = p.describe()
                assert desc["variant"] == "order" and desc["order_radix"] == radix
                y = run_plan(p, x)
                y_in = run_plan(p, x, inplace=True)
            err = rel_l2(y, oracle.dft(x, d))
            assert err.max() <= tol_for(n, dtype), (n, order, radix, err.max())
            assert np.array_equal(y, y_in)


def test_autotune_orders_and_recorded_order(tmp_path):
    fftc.tune_clear()
    try:
        res, best = fftc.autotune_orders(1024, 2048, "c64", reps=5)
        names = [(o, r) for o, r, _ in res]
        assert names[0] == ("stockham", 0) and ("ct", 2) in names and ("pease", 4) in names
        assert all(us > 0 for _, _, us in res)
        say("orders at 1024:", res, "best", best)
        # a recorded order is what fftc_plan runs
        db = tmp_path / "db.txt"
        db.write_text(f"{fftc.tune_key()} c64 256 pease:16,16 0.01\n")
        assert fftc.tune_load(str(db)) == 1
        x = synth.uniform_complex(synth.rng(141), (9, 256), np.complex64)
        with fftc.Plan(256, 9, FWD, "c64") as p:
            desc = p.describe()
            assert desc["variant"] == "order" and desc["order"] == "pease" and desc["order_radix"] == 16
            y = run_plan(p, x)
        assert rel_l2(y, oracle.dft(x)).max() <= tol_for(256, "c64")
    finally:
        fftc.tune_clear()


@pytest.mark.parametrize("n", [256, 1024, 4096])
def test_full_size_sampled(n):
    # the benchmark's launches: 2^24 complex64 elements, every compiled order
    b = (1 << 24) // n
    x = synth.uniform_complex(synth.rng(142, n), (b, n), np.complex64)
    picks = sorted({0, 1, b // 2, b - 1})
    want = oracle.dft(x[picks])
    for nn, order, radix in fftc.compiled_orders("c64"):
        if nn != n:
            continue
        say(f"full-size order n={n} {fftc.ORDER_NAMES[order]} r={radix}")
        with fftc.plan_order(n, b, FWD, "c64", order, radix) as p:
            y = run_plan(p, x)
        assert rel_l2(y[picks], want).max() <= tol_for(n, "c64"), (order, radix)
