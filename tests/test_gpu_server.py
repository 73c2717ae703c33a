"""Serving runtime on the GPU: results in the mix equal results alone, a small
budget forces queueing without exceeding it, and timestamps are ordered."""
import time

import numpy as np
import pytest

import oracle
from gpu_util import rel_l2, say, tol_for
from paper_2207_06803_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2207_06803_amd import fftc  # noqa: E402
from paper_2207_06803_amd import server as srv  # noqa: E402


def _collect(expected, outputs, timeout=60.0):
    got = {}
    t0 = time.time()
    while len(got) < expected and time.time() - t0 < timeout:
        for c in srv.poll():
            assert c["status"] == 0, c
            n, b = c["n"], c["batch"]
            # copy the output out of the arena, then give the memory back
            outputs[c["tag"]] = (c, _read_device(c["out"], n * b))
            srv.release(c["out"])
            got[c["tag"]] = c
        time.sleep(0.0002)
    return got


def _read_device(ptr, count):
    """Copy `count` complex64 values at a device address to a host array."""
    import ctypes
    host = np.empty(count, np.complex64)
    hip = ctypes.CDLL("libamdhip64.so.7")  # the runtime torch already loaded
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    rc = hip.hipMemcpy(host.ctypes.data, ctypes.c_void_p(ptr), count * 8, 2)  # device to host
    assert rc == 0
    return host


@pytest.fixture
def gpu_server():
    started = []

    def _start(budget, **kw):
        srv.start(budget, **kw)
        started.append(True)
    yield _start
    if started:
        try:
            srv.stop(drain=False)
        except fftc.FFTCError:
            pass


@pytest.mark.parametrize("fuse,hold_at", [(False, 0), (True, 0), (True, 4)])
def test_results_in_the_mix_equal_results_alone(gpu_server, fuse, hold_at):
    # hold_at = 4: rounds admitted while 4 or more requests run wait and
    # launch together (larger fused steps); every result must still equal the
    # same request run alone, bit for bit
    gpu_server(1 << 30, n_streams=4, max_inflight=32, fuse=fuse, hold_at=hold_at)
    g = synth.rng(5, 1)
    pool = torch.from_numpy(synth.uniform_complex(g, (1 << 21,), np.complex64)).to("cuda")
    reqs = []
    for tag in range(120):
        n = int(1 << g.integers(6, 17))
        b = int(g.integers(1, min(16, (1 << 21) // n) + 1))
        d = int(g.choice([fftc.FORWARD, fftc.INVERSE]))
        off = int(g.integers(0, (1 << 21) - n * b + 1))
        reqs.append((tag, n, b, d, off))
    for n in sorted({r[1] for r in reqs}):
        for d in (fftc.FORWARD, fftc.INVERSE):
            srv.prepare(n, d, "c64", 16)
    outputs = {}
    for tag, n, b, d, off in reqs:
        assert srv.submit(n, b, d, pool.data_ptr() + 8 * off, tag) == 0
    got = _collect(len(reqs), outputs)
    assert len(got) == len(reqs)
    host_pool = pool.cpu().numpy()
    for tag, n, b, d, off in reqs:
        c, y = outputs[tag]
        assert c["arrival_ns"] <= c["admit_ns"] <= c["start_ns"] <= c["done_ns"]
        x = host_pool[off:off + n * b]
        # alone: the same request through a plain plan
        with fftc.Plan(n, b, d, "c64") as p:
            xd = torch.from_numpy(x).to("cuda")
            yd = torch.empty_like(xd)
            p.execute(xd, yd)
            torch.cuda.synchronize()
        assert np.array_equal(y, yd.cpu().numpy()), (tag, n, b, d)
        if tag % 10 == 0:   # sampled requests against the oracle
            rows = x.reshape(b, n)[:2]
            if n <= 16384:
                err = rel_l2(y.reshape(b, n)[:len(rows)], oracle.dft(rows, d))
                assert err.max() <= tol_for(n, "c64"), (tag, n, err.max())
            else:
                ks = np.array([0, 1, n // 3, n - 1])
                ref = oracle.dft_points(rows[0], ks, d)
                scale = np.sqrt(n * (np.abs(rows[0].astype(np.complex128)) ** 2).sum())
                assert np.linalg.norm(y[:n][ks] - ref) / (scale * np.sqrt(len(ks) / n)) <= tol_for(n, "c64")
    st = srv.stats()
    say("served", len(reqs), "fuse", fuse, "stats", st)
    if fuse:  # a burst of 120 requests over 11 lengths: some steps run several requests
        assert st["fused_launches"] > 0 and st["fused_requests"] >= 2 * st["fused_launches"]
    else:
        assert st["fused_launches"] == 0


def test_small_budget_queues_and_holds(gpu_server):
    budget = 16 << 20
    gpu_server(budget, n_streams=2, max_inflight=8)
    pool = torch.randn(1 << 20, dtype=torch.complex64, device="cuda")
    total = 0
    for tag in range(64):
        n, b = 4096, 256        # 8 MiB each: at most two fit
        total += n * b * 8
        assert srv.submit(n, b, fftc.FORWARD, pool.data_ptr(), tag) == 0
    outputs = {}
    got = _collect(64, outputs)
    st = srv.stats()
    say("small budget stats", st, "total MiB", total >> 20)
    assert len(got) == 64
    assert st["peak_bytes"] <= budget
    assert total > 10 * budget
