"""Python binding of the fftc serving API (argument marshalling only)."""
from __future__ import annotations

import ctypes

from . import fftc
from .fftc import _i64, _int, _vp, check

EXECUTOR_GPU = 0
EXECUTOR_MOCK = 1


class Config(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("n_streams", _int), ("max_inflight", _int),
                ("executor", _int), ("mock_ns_per_mb", _i64), ("fuse", _int), ("tune_db", ctypes.c_char_p),
                ("hold_at", _int)]


class Request(ctypes.Structure):
    _fields_ = [("n", _i64), ("batch", _i64), ("direction", _int), ("dtype", _int), ("in_", _vp),
                ("tag", ctypes.c_uint64), ("arrival_ns", _i64)]


class Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", _int), ("out", _vp), ("arrival_ns", _i64),
                ("admit_ns", _i64), ("start_ns", _i64), ("done_ns", _i64), ("n", _i64), ("batch", _i64)]


class Stats(ctypes.Structure):
    _fields_ = [("submitted", _i64), ("admitted", _i64), ("completed", _i64), ("rejected", _i64),
                ("cancelled", _i64), ("failed", _i64), ("budget_bytes", ctypes.c_size_t),
                ("bytes_in_use", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t), ("pending", _int),
                ("inflight", _int), ("max_inflight_seen", _int), ("fused_launches", _i64),
                ("fused_requests", _i64), ("plan_bytes", ctypes.c_size_t)]


fftc.register("fftc_now_ns", _i64, [])
fftc.register("fftc_server_start", _int, [ctypes.POINTER(Config)])
fftc.register("fftc_server_prepare", _int, [_i64, _int, _int, _i64])
fftc.register("fftc_submit", _int, [ctypes.POINTER(Request)])
fftc.register("fftc_poll", _int, [ctypes.POINTER(Completion), _int, ctypes.POINTER(_int)])
fftc.register("fftc_release", _int, [_vp])
fftc.register("fftc_server_stats_get", _int, [ctypes.POINTER(Stats)])
fftc.register("fftc_server_stop", _int, [_int])
fftc.register("fftc_fault_set", _int, [_i64])
fftc.register("fftc_fault_count", _i64, [])

lib = fftc.lib


def now_ns() -> int:
    return int(lib.fftc_now_ns())


def start(budget_bytes: int, n_streams: int = 64, max_inflight: int = 256,
          executor: int = EXECUTOR_GPU, mock_ns_per_mb: int = 0, fuse: bool = False, tune_db: str = None,
          hold_at: int = 0) -> None:
    cfg = Config(budget_bytes, n_streams, max_inflight, executor, mock_ns_per_mb, 1 if fuse else 0,
                 tune_db.encode() if tune_db else None, hold_at)
    check(lib.fftc_server_start(ctypes.byref(cfg)), "fftc_server_start")


def fault_set(k: int) -> None:
    """Fail the k-th device or arena allocation from now on (k <= 0: off)."""
    check(lib.fftc_fault_set(int(k)), "fftc_fault_set")


def fault_count() -> int:
    return int(lib.fftc_fault_count())


def prepare(n: int, direction: int, dtype="c64", max_batch: int = 1) -> None:
    check(lib.fftc_server_prepare(n, direction, fftc.dtype_code(dtype), max_batch), "fftc_server_prepare")


def submit(n: int, batch: int, direction: int, in_ptr, tag: int, arrival_ns: int | None = None,
           dtype="c64") -> int:
    """Queue a request; returns the status code (0 OK, 4 too large, ...)."""
    r = Request(n, batch, direction, fftc.dtype_code(dtype), fftc.ptr(in_ptr), tag,
                now_ns() if arrival_ns is None else arrival_ns)
    return int(lib.fftc_submit(ctypes.byref(r)))


_poll_buf = (Completion * 256)()


def poll(max_items: int = 256):
    """Finished requests as a list of dicts."""
    k = _int()
    check(lib.fftc_poll(_poll_buf, min(max_items, 256), ctypes.byref(k)), "fftc_poll")
    out = []
    for i in range(k.value):
        c = _poll_buf[i]
        out.append({"tag": c.tag, "status": c.status, "out": c.out or 0, "arrival_ns": c.arrival_ns,
                    "admit_ns": c.admit_ns, "start_ns": c.start_ns, "done_ns": c.done_ns,
                    "n": c.n, "batch": c.batch})
    return out


def release(out_ptr: int) -> None:
    check(lib.fftc_release(out_ptr), "fftc_release")


def stats() -> dict:
    s = Stats()
    check(lib.fftc_server_stats_get(ctypes.byref(s)), "fftc_server_stats_get")
    return {f: getattr(s, f) for f, _ in Stats._fields_}


def stop(drain: bool = True) -> None:
    check(lib.fftc_server_stop(1 if drain else 0), "fftc_server_stop")
