"""Serving runtime logic on the CPU, with the mock executor (no device use,
no computation): admission against the budget, FIFO order, slots, errors,
shutdown."""
import time

import numpy as np
import pytest

from paper_2207_06803_amd import fftc
from paper_2207_06803_amd import server as srv

FAKE_IN = 0x10000  # never dereferenced by the mock executor


@pytest.fixture
def mock_server():
    def _start(budget, max_inflight=8, ns_per_mb=20000, streams=2):
        srv.start(budget, n_streams=streams, max_inflight=max_inflight,
                  executor=srv.EXECUTOR_MOCK, mock_ns_per_mb=ns_per_mb)
    yield _start
    try:
        srv.stop(drain=False)
    except fftc.FFTCError:
        pass


def _drain(expected, release=True, timeout=20.0):
    got = []
    t0 = time.time()
    while len(got) < expected and time.time() - t0 < timeout:
        for c in srv.poll():
            got.append(c)
            if release and c["status"] == 0:
                srv.release(c["out"])
        time.sleep(0.0005)
    return got


def test_budget_never_exceeded_and_all_complete(mock_server):
    budget = 8 << 20
    mock_server(budget, max_inflight=6)
    g = np.random.default_rng(1)
    reqs = []
    for tag in range(300):
        n = int(1 << g.integers(6, 14))
        b = int(g.integers(1, max(2, (budget // 8) // n // 2)))
        reqs.append((n, b))
        assert srv.submit(n, b, fftc.FORWARD, FAKE_IN, tag) == 0
    got = _drain(len(reqs))
    st = srv.stats()
    assert len(got) == len(reqs) and all(c["status"] == 0 for c in got)
    assert st["peak_bytes"] <= budget
    assert st["max_inflight_seen"] <= 6
    assert st["completed"] == 300 and st["bytes_in_use"] == 0


def test_admission_is_fifo_and_times_are_ordered(mock_server):
    mock_server(4 << 20, max_inflight=3)
    for tag in range(120):
        assert srv.submit(256, int(1 + tag % 100), fftc.INVERSE, FAKE_IN, tag) == 0
    got = _drain(120)
    by_tag = sorted(got, key=lambda c: c["tag"])
    admits = [c["admit_ns"] for c in by_tag]
    assert admits == sorted(admits)  # admitted in arrival order
    for c in got:
        assert c["arrival_ns"] <= c["admit_ns"] <= c["start_ns"] <= c["done_ns"]


def test_large_request_is_not_starved(mock_server):
    budget = 4 << 20
    mock_server(budget, max_inflight=8)
    n = 1024
    big_batch = (budget // 8) // n  # the whole budget
    for tag in range(20):
        srv.submit(n, 16, fftc.FORWARD, FAKE_IN, tag)
    assert srv.submit(n, big_batch, fftc.FORWARD, FAKE_IN, 999) == 0
    for tag in range(20, 40):
        srv.submit(n, 16, fftc.FORWARD, FAKE_IN, tag)
    got = _drain(41)
    tags = [c["tag"] for c in sorted(got, key=lambda c: c["admit_ns"])]
    assert len(got) == 41
    # the big one is admitted after the 20 ahead of it and before those behind
    assert tags.index(999) == 20


def test_too_large_and_bad_requests(mock_server):
    mock_server(1 << 20)
    assert srv.submit(1024, 1024, fftc.FORWARD, FAKE_IN, 1) == 4  # 8 MiB > 1 MiB
    assert srv.submit(11, 1, fftc.FORWARD, FAKE_IN, 2) == 2
    assert srv.submit(64, 0, fftc.FORWARD, FAKE_IN, 3) == 1
    assert srv.submit(64, 1, 0, FAKE_IN, 4) == 1
    assert srv.submit(64, 1, fftc.FORWARD, 0, 5) == 1
    assert srv.stats()["rejected"] == 1
    with pytest.raises(fftc.FFTCError) as e:
        srv.release(0x1234)
    assert e.value.status == 1
    with pytest.raises(fftc.FFTCError):
        srv.start(1 << 20, executor=srv.EXECUTOR_MOCK)  # already running


def test_stop_without_drain_cancels_queue(mock_server):
    mock_server(1 << 20, max_inflight=1, ns_per_mb=2_000_000)  # slow: queue builds up
    for tag in range(50):
        srv.submit(1024, 64, fftc.FORWARD, FAKE_IN, tag)
    time.sleep(0.01)
    srv.stop(drain=False)
    with pytest.raises(fftc.FFTCError) as e:
        srv.poll()
    assert e.value.status == 6


def test_stop_with_drain_completes_queue():
    srv.start(64 << 20, n_streams=2, max_inflight=4, executor=srv.EXECUTOR_MOCK, mock_ns_per_mb=1000)
    for tag in range(40):
        srv.submit(512, 32, fftc.FORWARD, FAKE_IN, tag)
    got = []
    # releases are not needed: the budget holds everything
    srv.stop(drain=True)
    assert len(got) == 0  # completions went away with the server; no hang


def test_calls_without_server():
    with pytest.raises(fftc.FFTCError) as e:
        srv.stats()
    assert e.value.status == 6
    assert srv.submit(64, 1, fftc.FORWARD, FAKE_IN, 0) == 6


def test_injected_arena_fault_fails_one_request_and_serving_continues(mock_server):
    """fftc_fault_set(k): the k-th arena allocation fails that request with
    FFTC_ERR_OUT_OF_MEMORY; nothing leaks and later requests are served."""
    mock_server(8 << 20, max_inflight=2)
    srv.fault_set(3)
    try:
        for tag in range(6):
            assert srv.submit(256, 4, fftc.FORWARD, FAKE_IN, tag) == 0
        got = _drain(6)
        assert len(got) == 6
        assert sorted(c["status"] for c in got) == [0, 0, 0, 0, 0, 3]
        failed = [c for c in got if c["status"] == 3][0]
        assert failed["tag"] == 2 and failed["out"] == 0        # admission order: the third request
        st = srv.stats()
        assert st["failed"] == 1 and st["completed"] == 6 and st["bytes_in_use"] == 0
        assert srv.fault_count() >= 6
        for tag in range(6, 12):
            assert srv.submit(1024, 2, fftc.INVERSE, FAKE_IN, tag) == 0
        got = _drain(6)
        assert len(got) == 6 and all(c["status"] == 0 for c in got)
        assert srv.stats()["bytes_in_use"] == 0
    finally:
        srv.fault_set(0)


def test_fault_and_log_environment_in_a_fresh_process(tmp_path):
    """FFTC_FAULT=2 and FFTC_LOG=1 set in the environment of a new process."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys, time; sys.path.insert(0, %r)\n"
        "from paper_2207_06803_amd import fftc, server as srv\n"
        "srv.start(1 << 20, n_streams=1, max_inflight=1, executor=srv.EXECUTOR_MOCK, mock_ns_per_mb=1000)\n"
        "for t in range(3): assert srv.submit(64, 2, fftc.FORWARD, 0x10000, t) == 0\n"
        "got = []\n"
        "t0 = time.time()\n"
        "while len(got) < 3 and time.time() - t0 < 20:\n"
        "    for c in srv.poll():\n"
        "        got.append(c)\n"
        "        if c['status'] == 0: srv.release(c['out'])\n"
        "srv.stop(drain=True)\n"
        "print(sorted((c['tag'], c['status']) for c in got))\n" % root)
    env = dict(os.environ, FFTC_FAULT="2", FFTC_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "[(0, 0), (1, 3), (2, 0)]"
    assert "fftc: server start" in r.stderr and "fftc: injected allocation failure" in r.stderr
    assert "fftc: server stop" in r.stderr


def test_server_config_tune_db(tmp_path):
    """fftc_server_config.tune_db is merged into the tuning database at start;
    an unreadable file fails the start."""
    fftc.tune_clear()
    db = tmp_path / "tune.txt"
    db.write_text(f"{fftc.tune_key()} c64 1024 16,4,16 0.010\n")
    try:
        srv.start(1 << 20, executor=srv.EXECUTOR_MOCK, tune_db=str(db))
        srv.stop(drain=True)
        assert fftc.factorize(1024)[0] == [16, 4, 16]
        with pytest.raises(fftc.FFTCError) as e:
            srv.start(1 << 20, executor=srv.EXECUTOR_MOCK, tune_db=str(tmp_path / "missing.txt"))
        assert e.value.status == 1
    finally:
        fftc.tune_clear()


@pytest.mark.parametrize("hold_at", [0, 2])
def test_hold_at_launches_held_rounds_when_the_device_drains(hold_at):
    """hold_at = k: requests admitted while k or more are running wait and
    start once fewer than k run; hold_at = 0 starts every request at
    admission.  Two 1 MiB requests run 50 ms each (mock executor); two more
    arrive 10 ms later."""
    srv.start(64 << 20, n_streams=2, max_inflight=16, executor=srv.EXECUTOR_MOCK,
              mock_ns_per_mb=50_000_000, hold_at=hold_at)
    try:
        for tag in (0, 1):
            assert srv.submit(1024, 128, fftc.FORWARD, FAKE_IN, tag) == 0
        time.sleep(0.010)
        for tag in (2, 3):
            assert srv.submit(1024, 128, fftc.FORWARD, FAKE_IN, tag) == 0
        got = {c["tag"]: c for c in _drain(4)}
        assert sorted(got) == [0, 1, 2, 3] and all(c["status"] == 0 for c in got.values())
        first_done = min(got[0]["done_ns"], got[1]["done_ns"])
        late = [got[2]["start_ns"], got[3]["start_ns"]]
        if hold_at:
            assert min(late) >= first_done
        else:
            assert max(late) < first_done
        for c in got.values():
            assert c["arrival_ns"] <= c["admit_ns"] <= c["start_ns"] <= c["done_ns"]
    finally:
        srv.stop(drain=True)
