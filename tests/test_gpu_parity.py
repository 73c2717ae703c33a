"""GPU path against the FP64 oracle through the C ABI (single-kernel plans)."""
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


def check(n, batch, direction, dtype, radices=None, seed=0, inplace=False, x=None):
    say(f"case n={n} batch={batch} dir={direction} dtype={dtype} radices={radices} inplace={inplace}")
    if x is None:
        x = synth.uniform_complex(synth.rng(90, seed, n % 1000), (batch, n), np_dtype(dtype))
    with fftc.Plan(n, batch, direction, dtype, radices=radices) as p:
        y = run_plan(p, x, inplace=inplace)
        desc = p.describe()
    ref = oracle.dft(x, direction)
    err = rel_l2(y, ref)
    assert err.max() <= tol_for(n, dtype), (n, dtype, direction, radices, err.max(), desc)
    return err, desc


def test_config1_n64_batch1024_full():
    # forward complex64, N = 64, 1024 transforms, uniform[-1,1): every output
    x = synth.uniform_complex(synth.rng(0), (1024, 64), np.complex64)
    err, desc = check(64, 1024, FWD, "c64", x=x)
    assert err.max() <= 6e-6
    say("config1 max rel L2", err.max(), desc["variant"], desc["radices"])


def _ragged_batch(n):
    # several workgroups and a partial last one
    per = max(1, 256 // max(1, n // 16))
    b = 3 * per + 1
    while b * n > (1 << 18) and b > 3:
        b = b // 2 + 1
    return b


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_every_compiled_list(dtype):
    # every specialised kernel, both directions, several groups + ragged tail
    lists = fftc.compiled_lists(dtype)
    assert len(lists) > 100
    for n, rs in lists:
        for d in (FWD, INV):
            _, desc = check(n, _ragged_batch(n), d, dtype, radices=rs)
            assert desc["variant"] == "single_specialised", desc


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_default_plans_are_compiled(dtype):
    for n in [1 << k for k in range(3, 14)] + synth.mixed_size_set():
        with fftc.Plan(n, 4, FWD, dtype) as p:
            assert p.describe()["variant"] == "single_specialised", (n, p.describe())


GENERIC_C64 = [(12, [4, 3]), (12, [3, 4]), (3072, [3, 4, 16, 16]), (3584, [7, 8, 8, 8]),
               (2560, [5, 8, 4, 16]), (64, [2, 2, 2, 2, 2, 2]), (4096, [4, 4, 4, 4, 4, 4]),
               (1024, [2, 8, 4, 16]), (16384, [2, 8, 16, 4, 16]), (105, [3, 5, 7]),
               (225, [3, 3, 5, 5]), (343, [7, 7, 7]), (10, [2, 5]), (14, [7, 2])]


@pytest.mark.parametrize("n,rs", GENERIC_C64, ids=lambda v: str(v))
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_generic_explicit_lists(n, rs, dtype):
    if n > fftc.max_single_n(dtype):
        pytest.skip("two-pass length for this dtype")
    for d in (FWD, INV):
        _, desc = check(n, _ragged_batch(n), d, dtype, radices=rs)
        assert desc["radices"] == rs


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_mixed_size_set_default_plans(dtype):
    for n in synth.mixed_size_set() + [1, 2, 3, 4, 5, 6, 7, 9, 15, 21, 35, 49, 125, 6561 // 27 * 3]:
        for d in (FWD, INV):
            check(n, _ragged_batch(n), d, dtype)


@pytest.mark.parametrize("n", [256, 1024, 4096])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_config2_sizes_full_oracle(n, dtype):
    # batch scaled down so the O(N^2) oracle finishes in seconds
    batch = (1 << 17) // n + 3
    for d in (FWD, INV):
        err, desc = check(n, batch, d, dtype, seed=2)
        say(f"config2 n={n} {dtype} dir={d} max rel L2 {err.max():.3e} {desc['variant']} {desc['radices']}")


@pytest.mark.parametrize("n", [256, 1024, 4096])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_config2_full_size_sampled(n, dtype):
    # the benchmarked shape: 2^24 elements per run; sampled transforms against
    # the oracle, Parseval on every transform
    batch = (1 << 24) // n
    g = synth.rng(1, n, 0 if dtype == "c64" else 1)
    x = synth.uniform_complex(g, (batch, n), np_dtype(dtype))
    rows = np.unique(np.r_[0, batch - 1, g.integers(0, batch, 6)])
    for d in (FWD, INV):
        say(f"config2 full n={n} batch={batch} {dtype} dir={d}")
        with fftc.Plan(n, batch, d, dtype) as p:
            y = run_plan(p, x)
        err = rel_l2(y[rows], oracle.dft(x[rows], d))
        assert err.max() <= tol_for(n, dtype), err.max()
        ex = (np.abs(x.astype(np.complex128)) ** 2).sum(axis=1) * n
        ey = (np.abs(y.astype(np.complex128)) ** 2).sum(axis=1)
        rel = np.abs(ey - ex) / ex
        assert rel.max() <= 2 * tol_for(n, dtype), rel.max()


@pytest.mark.parametrize("n,dtype", [(8192, "c64"), (16384, "c64"), (32768, "c64"), (4096, "c128"), (8192, "c128"),
                                     (16384, "c128")])
def test_half_exchange_full_size_sampled(n, dtype):
    # the lengths whose kernels exchange real and imaginary parts through LDS
    # separately, at the benchmarked launch size (2^24 elements, several
    # workgroups per CU): sampled transforms against the oracle, Parseval on
    # every transform, both directions
    batch = (1 << 24) // n
    g = synth.rng(1, n, 2 if dtype == "c64" else 3)
    x = synth.uniform_complex(g, (batch, n), np_dtype(dtype))
    rows = np.unique(np.r_[0, batch - 1, g.integers(0, batch, 2)])
    for d in (FWD, INV):
        say(f"half-exchange full n={n} batch={batch} {dtype} dir={d}")
        with fftc.Plan(n, batch, d, dtype) as p:
            y = run_plan(p, x)
        err = rel_l2(y[rows], oracle.dft(x[rows], d))
        say(f"  sampled rows {rows.tolist()}: max rel L2 {err.max():.3e}")
        assert err.max() <= tol_for(n, dtype), err.max()
        ex = (np.abs(x.astype(np.complex128)) ** 2).sum(axis=1) * n
        ey = (np.abs(y.astype(np.complex128)) ** 2).sum(axis=1)
        assert (np.abs(ey - ex) / ex).max() <= 2 * tol_for(n, dtype)


@pytest.mark.parametrize("n,dtype", [(32768, "c64"), (16384, "c128")])
def test_wide_length_default_plan(n, dtype):
    # past fftc_max_single_n: one kernel with the first compiled wide list,
    # in place bit-identical to out of place, against the oracle
    wide = [list(rs) for m, rs in fftc.compiled_lists(dtype) if m == n]
    for d in (FWD, INV):
        err, desc = check(n, 3, d, dtype, seed=4)
        assert desc["variant"] == "single_specialised" and desc["radices"] == wide[0], desc
        assert desc["split_m"] == 0 and desc["scratch_bytes"] == 0, desc
        x = synth.uniform_complex(synth.rng(92, n), (3, n), np_dtype(dtype))
        with fftc.Plan(n, 3, d, dtype) as p:
            assert np.array_equal(run_plan(p, x), run_plan(p, x, inplace=True))


def test_inplace_single_kernel():
    for n, dtype in ((1024, "c64"), (3584, "c64"), (4096, "c128"), (64, "c64")):
        check(n, 37, FWD, dtype, inplace=True)
        check(n, 37, INV, dtype, inplace=True)


def test_round_trip_and_delta():
    n, b = 4096, 8
    g = synth.rng(91)
    x = synth.uniform_complex(g, (b, n), np.complex64)
    with fftc.Plan(n, b, FWD) as pf, fftc.Plan(n, b, INV) as pi:
        y = run_plan(pf, x)
        z = run_plan(pi, y)
        assert rel_l2(z / n, x).max() <= 2 * tol_for(n, "c64")
        d = np.zeros((b, n), np.complex64)
        d[:, 0] = 1
        yd = run_plan(pf, d)
        assert np.abs(yd - 1).max() <= 1e-5


def test_bitwise_deterministic():
    n, b = 1024, 333
    x = synth.uniform_complex(synth.rng(92), (b, n), np.complex64)
    with fftc.Plan(n, b, FWD) as p:
        y1 = run_plan(p, x)
        y2 = run_plan(p, x)
    assert np.array_equal(y1.view(np.uint32), y2.view(np.uint32))


def test_misaligned_pointer_rejected():
    x = torch.zeros(65, dtype=torch.complex64, device="cuda")
    with fftc.Plan(64, 1, FWD, "c64") as p:
        with pytest.raises(fftc.FFTCError) as e:
            p.execute(x.data_ptr() + 4, x.data_ptr() + 8 * 0)
        assert e.value.status == 1
    xd = torch.zeros(65, dtype=torch.complex128, device="cuda")
    with fftc.Plan(64, 1, FWD, "c128") as p:
        with pytest.raises(fftc.FFTCError):
            p.execute(xd.data_ptr() + 8, xd.data_ptr())


@pytest.mark.parametrize("n", [4, 16, 64, 256, 1024, 4096, 12, 3584, 32768])
def test_eight_byte_offsets(n):
    """complex64 buffers that are 8- but not 16-byte aligned (input at element
    1, output at element 3 of their allocations): the kernels that move two
    elements per 16-byte access take their 8-byte path, and nothing outside
    the output range is written."""
    b = 5 if n <= 4096 else 2
    say(f"case n={n} batch={b} offsets 8 / 24 bytes")
    x = synth.uniform_complex(synth.rng(96, n), (b, n), np.complex64)
    xt = torch.zeros(b * n + 4, dtype=torch.complex64, device="cuda")
    yt = torch.zeros(b * n + 4, dtype=torch.complex64, device="cuda")
    xt[1:1 + b * n] = torch.from_numpy(x.reshape(-1)).to("cuda")
    with fftc.Plan(n, b, FWD, "c64") as p:
        p.execute(xt.data_ptr() + 8, yt.data_ptr() + 24)
    torch.cuda.synchronize()
    yall = yt.cpu().numpy()
    assert not yall[:3].any() and not yall[3 + b * n:].any()
    y = yall[3:3 + b * n].reshape(b, n)
    if n <= 4096:
        assert rel_l2(y, oracle.dft(x)).max() <= tol_for(n, "c64")
    else:
        ks = np.array([0, 1, 7, n // 2, n - 1])
        for row in range(b):
            ref = oracle.dft_points(x[row], ks)
            scale = np.sqrt(n * (np.abs(x[row].astype(np.complex128)) ** 2).sum())
            err = np.linalg.norm(y[row, ks] - ref) / (scale * np.sqrt(len(ks) / n))
            assert err <= tol_for(n, "c64"), err


def test_copy_reference():
    """fftc_copy (the benchmark's bandwidth reference) copies bytes exactly."""
    n = (1 << 20) + 3
    x = torch.from_numpy(synth.uniform_complex(synth.rng(97), (n,), np.complex64)).to("cuda")
    y = torch.zeros(n + 1, dtype=torch.complex64, device="cuda")
    fftc.copy(x, y, 8 * (n - 1))  # 16-byte multiple: n - 1 elements
    torch.cuda.synchronize()
    assert torch.equal(y[:n - 1], x[:n - 1]) and not y[n - 1:].any()


def test_undersized_tensors_refused_before_launch():
    """The binding compares tensor extents with what a plan touches and
    raises before anything is launched (the kernels cannot see sizes)."""
    n, b = 1024, 4
    x = torch.zeros(n * b - 1, dtype=torch.complex64, device="cuda")
    y = torch.zeros(n * b, dtype=torch.complex64, device="cuda")
    with fftc.Plan(n, b, FWD, "c64") as p:
        assert p.bytes_needed() == (8 * n * b, 8 * n * b)
        with pytest.raises(fftc.FFTCError) as e:
            p.execute(x, y)
        assert e.value.status == 1
        with pytest.raises(fftc.FFTCError):
            p.execute(y, x)
        with pytest.raises(fftc.FFTCError):
            p.execute_batch(y[: 2 * n - 1], y, 2)
        p.execute_batch(y[: 2 * n], x[: 2 * n], 2)  # exactly large enough
    # a planar layout with gaps: each array must reach the last element
    with fftc.plan_layout(n, b, FWD, "c64", (1, n + 3, 1), None) as p:
        assert p.bytes_needed() == (4 * ((b - 1) * (n + 3) + n), 8 * n * b)
        re = torch.zeros((b - 1) * (n + 3) + n - 1, device="cuda")
        with pytest.raises(fftc.FFTCError):
            fftc.execute_layout(p, re, re, y, None)
    torch.cuda.synchronize()


def test_unusable_tensors_refused_before_launch():
    """Host tensors, non-contiguous views, under-sized batch slices of a
    layout plan and under-sized copy operands raise before any launch."""
    n, b = 256, 4
    y = torch.zeros(n * b, dtype=torch.complex64, device="cuda")
    big = torch.zeros(2 * n * b, dtype=torch.complex64, device="cuda")
    with fftc.Plan(n, b, FWD, "c64") as p:
        with pytest.raises(fftc.FFTCError) as e:
            p.execute(torch.zeros(n * b, dtype=torch.complex64), y)       # host memory
        assert e.value.status == 1
        with pytest.raises(fftc.FFTCError):
            p.execute(big[::2], y)                                           # spans enough, not dense
        with pytest.raises(fftc.FFTCError):
            p.execute_batch(y, big.view(2, n * b).t(), 1)                 # transposed view
    # layout plan: each batch slice must reach its own last element
    lay = (1, n + 8, 0)
    with fftc.plan_layout(n, b, FWD, "c64", lay, lay) as p:
        need2 = (2 - 1) * (n + 8) + n
        assert p.bytes_needed(2) == (8 * need2, 8 * need2)
        with pytest.raises(fftc.FFTCError):
            p.execute_batch(big[: need2 - 1], big[: need2], 2)
        p.execute_batch(y[: need2], big[: need2], 2)
    with pytest.raises(fftc.FFTCError):
        fftc.copy(y[: n - 2], big, 8 * n)                                    # source too short
    with pytest.raises(fftc.FFTCError):
        fftc.copy(big, y[: n - 2], 8 * n)                                    # destination too short
    torch.cuda.synchronize()


def test_injected_device_allocation_faults():
    """FFTC_FAULT's counter from code: the k-th device allocation of a plan
    fails with FFTC_ERR_OUT_OF_MEMORY before any HIP call, the partial plan
    is freed, and the next plan works."""
    from paper_2207_06803_amd import server as srv
    free0 = torch.cuda.mem_get_info()[0]
    try:
        for n, k in ((1024, 1), (1 << 20, 1), (1 << 20, 2), (1 << 20, 3)):
            srv.fault_set(k)
            with pytest.raises(fftc.FFTCError) as e:
                fftc.Plan(n, 4, FWD, "c64")
            assert e.value.status == 3 and "injected" in str(e.value), (n, k)
        srv.fault_set(0)
        with fftc.Plan(1 << 20, 4, FWD, "c64") as p:
            assert p.describe()["variant"] == "two_pass"
        torch.cuda.synchronize()
        assert abs(torch.cuda.mem_get_info()[0] - free0) < (64 << 20)
    finally:
        srv.fault_set(0)
