"""Planar and strided layouts (fftc_plan_layout) against the FP64 oracle:
every compiled layout length, both dtypes and directions; planar, strided,
column (interleaved transforms) and mixed layouts; in place; elements outside
the layout untouched; agreement with the interleaved plan and run-to-run
determinism.  (The layout kernels are separate compilations of the same
stages: the compiler may contract a different set of products into FMAs, so
agreement with the interleaved plan is to rounding, not to the bit.)"""
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

FWD, INV = fftc.FORWARD, fftc.INVERSE
SENTINEL = 12345.0


def real_dtype(dtype):
    return np.float32 if dtype == "c64" else np.float64


def extent(batch, n, stride, dist):
    return (batch - 1) * dist + (n - 1) * stride + 1


def index(batch, n, stride, dist):
    return np.arange(batch)[:, None] * dist + np.arange(n)[None, :] * stride


def to_device(x, layout, dtype, pad=7):
    """Scatter logical x (batch, n) into device buffer(s) of the layout;
    every other element holds SENTINEL."""
    stride, dist, planar = layout
    b, n = x.shape
    size = extent(b, n, stride, dist) + pad
    idx = index(b, n, stride, dist)
    if planar:
        re = np.full(size, SENTINEL, real_dtype(dtype))
        im = np.full(size, SENTINEL, real_dtype(dtype))
        re[idx], im[idx] = x.real, x.imag
        return torch.from_numpy(re).cuda(), torch.from_numpy(im).cuda()
    buf = np.full(size, SENTINEL + 1j * SENTINEL, np_dtype(dtype))
    buf[idx] = x
    return torch.from_numpy(buf).cuda(), None


def from_device(bufs, layout, b, n):
    stride, dist, planar = layout
    idx = index(b, n, stride, dist)
    if planar:
        re, im = bufs[0].cpu().numpy(), bufs[1].cpu().numpy()
        mask = np.ones(re.shape, bool)
        mask[idx] = False
        return re[idx] + 1j * im[idx], (re[mask] == SENTINEL).all() and (im[mask] == SENTINEL).all()
    a = bufs[0].cpu().numpy()
    mask = np.ones(a.shape, bool)
    mask[idx] = False
    return a[idx], (a[mask] == SENTINEL + 1j * SENTINEL).all()


def run_layout(plan, x, lin, lout, dtype, inplace=False):
    b, n = x.shape
    xin = to_device(x, lin, dtype)
    xout = xin if inplace else to_device(np.zeros_like(x), lout, dtype)
    if not inplace:  # fresh output: sentinel everywhere
        for t in xout:
            if t is not None:
                t.fill_(SENTINEL) if t.dtype in (torch.float32, torch.float64) else t.fill_(complex(SENTINEL, SENTINEL))
    fftc.execute_layout(plan, xin[0], xin[1], xout[0], xout[1])
    torch.cuda.synchronize()
    return from_device(xout, lout, b, n)


def layout_lengths(dtype):
    # the lengths compiled with the layout accessors (the wide lengths past
    # fftc_max_single_n have plain kernels only)
    return sorted({n for n, _ in fftc.compiled_lists(dtype) if n <= fftc.max_single_n(dtype)})


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_planar_every_length(dtype):
    for n in layout_lengths(dtype):
        b = 3
        say(f"planar n={n} {dtype}")
        x = synth.uniform_complex(synth.rng(130, n), (b, n), np_dtype(dtype))
        lay = (1, n, 1)
        for d in (FWD, INV):
            with fftc.plan_layout(n, b, d, dtype, lay, lay) as p:
                y, clean = run_layout(p, x, lay, lay, dtype)
            err = rel_l2(y, oracle.dft(x, d))
            assert err.max() <= tol_for(n, dtype), (n, d, err.max())
            assert clean


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n", [2, 8, 12, 64, 256, 1024, 4096, 7 * 512, 16384])
def test_layout_kinds(n, dtype):
    if n > fftc.max_single_n(dtype):
        pytest.skip("beyond the single-kernel lengths of this dtype")
    b = 5 if n <= 4096 else 3
    x = synth.uniform_complex(synth.rng(131, n), (b, n), np_dtype(dtype))
    cases = [
        ((1, n, 1), (1, n, 0)),                    # planar in, interleaved out (createComplex)
        ((1, n, 0), (1, n, 1)),                    # interleaved in, planar out
        ((2, 2 * n + 3, 0), (3, 3 * n + 1, 1)),    # strided with gaps
        ((b, 1, 0), (b + 2, 1, 0)),                # columns of a row-major array
        ((b, 1, 1), (1, n + 5, 1)),                # planar columns in, padded planar rows out
        ((1, n, 0), (b + 1, 1, 1)),                # rows in, planar columns out
        ((2 * b, 2, 0), (2 * b + 1, 2, 0)),        # every other column
    ]
    for lin, lout in cases:
        for d in (FWD, INV):
            say(f"layout n={n} {dtype} in={lin} out={lout} dir={d}")
            with fftc.plan_layout(n, b, d, dtype, lin, lout) as p:
                desc = p.describe()
                assert desc["has_layout"] and desc["layout_in"] == lin and desc["layout_out"] == lout
                y, clean = run_layout(p, x, lin, lout, dtype)
            err = rel_l2(y, oracle.dft(x, d))
            assert err.max() <= tol_for(n, dtype), (lin, lout, err.max())
            assert clean, (lin, lout)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_agrees_with_interleaved_plan_and_is_deterministic(dtype):
    for n in (16, 256, 1024, 4096):
        b = 6
        x = synth.uniform_complex(synth.rng(132, n), (b, n), np_dtype(dtype))
        with fftc.Plan(n, b, FWD, dtype) as q:
            xd = torch.from_numpy(x.copy()).cuda()
            yd = torch.empty_like(xd)
            q.execute(xd, yd)
            torch.cuda.synchronize()
            want = yd.cpu().numpy()
        with fftc.plan_layout(n, b, FWD, dtype, (1, n, 1), (1, n, 1)) as p:
            y, _ = run_layout(p, x, (1, n, 1), (1, n, 1), dtype)
            y2, _ = run_layout(p, x, (1, n, 1), (1, n, 1), dtype)
        assert np.array_equal(y, y2), n
        assert rel_l2(y, want).max() <= tol_for(n, dtype) / 4, n


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_two_pass_columns(dtype):
    # column-like sides beyond the tile kernel: two passes through scratch
    for n in (4096, 8192, 3 * 2048, 32768, 1 << 20) + ((16384,) if dtype == "c64" else ()):
        b = 21 if n <= 32768 else 3
        x = synth.uniform_complex(synth.rng(137, n), (b, n), np_dtype(dtype))
        for lin, lout in [((b, 1, 0), (b, 1, 0)), ((b + 2, 1, 1), (1, n, 0)), ((1, n + 3, 1), (b, 1, 1))]:
            for d in (FWD, INV):
                say(f"two-pass columns n={n} {dtype} {lin}->{lout} dir={d}")
                with fftc.plan_layout(n, b, d, dtype, lin, lout) as p:
                    assert p.describe()["scratch_bytes"] == b * n * np.dtype(np_dtype(dtype)).itemsize
                    y, clean = run_layout(p, x, lin, lout, dtype)
                    if lin == lout:
                        y_in, clean_in = run_layout(p, x, lin, lout, dtype, inplace=True)
                        assert np.array_equal(y, y_in) and clean_in
                if n <= 8192:
                    assert rel_l2(y, oracle.dft(x, d)).max() <= tol_for(n, dtype), (n, lin, lout)
                else:  # sampled outputs of sampled transforms (the O(n^2) oracle one output at a time)
                    g = synth.rng(138, n)
                    ks = np.unique(np.r_[0, 1, n // 3, n - 1, g.integers(0, n, 12)])
                    for row in sorted({0, b // 2, b - 1}):
                        ref = oracle.dft_points(x[row], ks, d)
                        scale = np.sqrt(n * (np.abs(x[row].astype(np.complex128)) ** 2).sum())
                        err = np.linalg.norm(y[row][ks] - ref) / (scale * np.sqrt(len(ks) / n))
                        assert err <= tol_for(n, dtype), (n, row, err)
                assert clean


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_columns_every_length(dtype):
    # the tile kernel of every compiled length, with a ragged last tile
    for n in layout_lengths(dtype):
        b = 37
        x = synth.uniform_complex(synth.rng(135, n), (b, n), np_dtype(dtype))
        lay = (b + 3, 1, 0)
        say(f"columns n={n} {dtype}")
        with fftc.plan_layout(n, b, INV, dtype, lay, lay) as p:
            y, clean = run_layout(p, x, lay, lay, dtype)
        assert rel_l2(y, oracle.dft(x, INV)).max() <= tol_for(n, dtype), n
        assert clean


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_in_place(dtype):
    for n, lay in [(1024, (1, 1024, 1)), (64, (7, 1, 0)), (4096, (2, 8200, 1))]:
        b = 7 if lay[1] == 1 else 3
        if lay[1] == 1:
            lay = (b, 1, lay[2])
        x = synth.uniform_complex(synth.rng(133, n), (b, n), np_dtype(dtype))
        with fftc.plan_layout(n, b, FWD, dtype, lay, lay) as p:
            y, clean = run_layout(p, x, lay, lay, dtype, inplace=True)
        assert rel_l2(y, oracle.dft(x)).max() <= tol_for(n, dtype)
        assert clean


def test_listing1_create_complex():
    # Listing 1's createComplex(InputReal, InputImg): planar [1,2,3,4] + i [1,2,3,4]
    re = torch.tensor([1.0, 2.0, 3.0, 4.0], dtype=torch.float32).cuda()
    im = re.clone()
    out = torch.empty(4, dtype=torch.complex64).cuda()
    with fftc.plan_layout(4, 1, FWD, "c64", (1, 4, 1), None) as p:
        fftc.execute_layout(p, re, im, out, None)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), np.array([10 + 10j, -4, -2 - 2j, -4j], np.complex64))


def test_interleaved_layout_through_execute():
    n, b = 256, 4
    x = synth.uniform_complex(synth.rng(134), (b, n), np.complex64)
    lay = (1, n + 16, 0)
    with fftc.plan_layout(n, b, FWD, "c64", lay, lay) as p:
        xin = to_device(x, lay, "c64")[0]
        yout = torch.full_like(xin, complex(SENTINEL, SENTINEL))
        p.execute(xin, yout)
        torch.cuda.synchronize()
        y, clean = from_device((yout, None), lay, b, n)
    assert rel_l2(y, oracle.dft(x)).max() <= tol_for(n, "c64") and clean


def test_execute_errors():
    with fftc.plan_layout(64, 2, FWD, "c64", (1, 64, 1), (1, 64, 1)) as p:
        a = torch.zeros(128, dtype=torch.float32).cuda()
        c = torch.zeros(128, dtype=torch.float32).cuda()
        with pytest.raises(fftc.FFTCError):
            fftc.execute_layout(p, a, None, c, c)       # planar input without im
        with pytest.raises(fftc.FFTCError):
            fftc.execute_layout(p, a, c, a, a)          # partial overlap
        with pytest.raises(fftc.FFTCError):
            p.execute(a, c)                             # planar plans need execute_layout


@pytest.mark.parametrize("n", [256, 1024, 4096])
def test_full_size_sampled(n):
    # the benchmark's launches (2^24 complex64 elements): planar rows and
    # columns of the n x (2^24 / n) row-major array; sampled transforms
    E = 1 << 24
    b = E // n
    g = synth.rng(136, n)
    host = synth.uniform_complex(g, (E,), np.complex64)
    picks = sorted({0, 1, b // 2, b - 1})
    # planar rows: transform q is host[q n : (q + 1) n]
    re = torch.from_numpy(np.ascontiguousarray(host.real)).cuda()
    im = torch.from_numpy(np.ascontiguousarray(host.imag)).cuda()
    ore, oim = torch.empty_like(re), torch.empty_like(im)
    say(f"full-size planar n={n}")
    with fftc.plan_layout(n, b, FWD, "c64", (1, n, 1), (1, n, 1)) as p:
        fftc.execute_layout(p, re, im, ore, oim)
    torch.cuda.synchronize()
    y = (ore.cpu().numpy() + 1j * oim.cpu().numpy()).reshape(b, n)
    x = host.reshape(b, n)
    assert rel_l2(y[picks], oracle.dft(x[picks])).max() <= tol_for(n, "c64")
    del re, im, ore, oim
    # columns: transform q is host[q + j b]
    xd = torch.from_numpy(host).cuda()
    yd = torch.empty_like(xd)
    say(f"full-size columns n={n}")
    with fftc.plan_layout(n, b, FWD, "c64", (b, 1, 0), (b, 1, 0)) as p:
        fftc.execute_layout(p, xd, None, yd, None)
    torch.cuda.synchronize()
    yc = yd.cpu().numpy().reshape(n, b)
    xc = host.reshape(n, b)
    assert rel_l2(yc[:, picks].T, oracle.dft(np.ascontiguousarray(xc[:, picks].T))).max() <= tol_for(n, "c64")
