"""fftc_execute_static, the entry point that allocates no device memory,
against fftc_plan + fftc_execute on the same inputs: bit-identical outputs
(same kernels, same tables), two calls in a row on one stream with the
second smaller, single-kernel and two-pass lengths, out of place and in
place (the in-place two-pass intermediate runs through the static array a
chunk of transforms at a time), plus the FP64 oracle on sampled rows."""
import os
import tempfile

import numpy as np
import pytest

import oracle
from gpu_util import np_dtype, rel_l2, say, tol_for
from paper_2207_06803_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2207_06803_amd import fftc  # noqa: E402


@pytest.fixture(autouse=True)
def default_planner():
    """Both paths plan from the built-in heuristic: a tuning database left by
    earlier tests (which may name an alternative order that fftc_plan would
    take) is set aside and restored afterwards."""
    fd, path = tempfile.mkstemp(suffix=".tune")
    os.close(fd)
    try:
        fftc.tune_save(path)
        fftc.tune_clear()
        yield
        fftc.tune_clear()
        fftc.tune_load(path)
    finally:
        os.unlink(path)


def planned(n, b, direction, dtype, x, inplace):
    y = x.clone()
    out = y if inplace else torch.empty_like(x)
    with fftc.Plan(n, b, direction, dtype) as p:
        p.execute(y, out)
        torch.cuda.synchronize()
    return out.cpu().numpy()


# (n, batch, dtype, in place) of the first and the (smaller) second call
PAIRS = [
    ((4096, 64, "c64", False), (1024, 3, "c64", False)),
    ((1024, 32, "c128", False), (256, 5, "c128", True)),
    ((16384, 12, "c64", True), (12, 7, "c64", False)),
    ((65536, 8, "c64", False), (32768, 3, "c64", False)),
    ((1 << 20, 9, "c64", True), (32768, 5, "c64", True)),     # 9 x 8 MiB: two chunks of the intermediate
    ((32768, 6, "c128", True), (16384, 2, "c128", False)),
]


@pytest.mark.parametrize("pair", PAIRS, ids=lambda p: "-".join(f"{n}x{b}{d}{'ip' if ip else ''}" for n, b, d, ip in p))
@pytest.mark.parametrize("direction", [fftc.FORWARD, fftc.INVERSE])
def test_static_matches_plan(pair, direction):
    assert fftc.static_scratch_bytes() == 64 << 20
    xs, bufs = [], []
    for i, (n, b, dtype, inplace) in enumerate(pair):
        x = synth.uniform_complex(synth.rng(140, n, i), (b, n), np_dtype(dtype))
        xd = torch.from_numpy(x).to("cuda")
        yd = xd.clone() if inplace else torch.full_like(xd, complex(7, 7))
        xs.append(x)
        bufs.append((xd, yd))
    say(f"static pair {pair} direction {direction}")
    s = torch.cuda.current_stream()
    # two calls in a row on one stream, no synchronisation between them
    for (n, b, dtype, inplace), (xd, yd) in zip(pair, bufs):
        fftc.execute_static(n, b, yd if inplace else xd, yd, direction, dtype, s)
    torch.cuda.synchronize()
    for (n, b, dtype, inplace), x, (xd, yd) in zip(pair, xs, bufs):
        got = yd.cpu().numpy()
        want = planned(n, b, direction, dtype, xd, inplace)
        assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), (n, b, dtype, inplace)
        if n <= 65536:
            rows = sorted({0, b - 1})
            err = rel_l2(got[rows], oracle.dft(x[rows], direction)).max()
            say(f"  n={n} b={b} {dtype}: bit-identical to the plan; oracle rows {rows} max rel L2 {err:.2e}")
            assert err <= tol_for(n, dtype)


def test_static_errors():
    x = torch.zeros(64, dtype=torch.complex64, device="cuda")
    for args, code in (((64, 1, 0, fftc.C64), 1),           # bad direction
                       ((64, 1, fftc.FORWARD, fftc.C64_SPLIT_F16), 1),
                       ((11, 1, fftc.FORWARD, fftc.C64), 2),
                       ((64, 0, fftc.FORWARD, fftc.C64), 1)):
        st = fftc.lib.fftc_execute_static(*args, x.data_ptr(), x.data_ptr(), None)
        assert st == code, (args, st, fftc.last_error())
    st = fftc.lib.fftc_execute_static(64, 1, fftc.FORWARD, fftc.C64, x.data_ptr() + 4, x.data_ptr(), None)
    assert st == 1
    with pytest.raises(fftc.FFTCError):
        fftc.execute_static(64, 2, x, x)          # buffer holds one transform
