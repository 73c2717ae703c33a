"""Python binding of the fftc C ABI (include/fftc.h).

Argument marshalling only: every transform runs in the HIP kernels of
libfftc.so.  PyTorch is used by callers for device memory and streams; this
module accepts anything with a `data_ptr()` (a torch tensor) or a raw integer
device address.  If libfftc.so is missing the import fails loudly -- there is
no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfftc.so")

FORWARD = -1
INVERSE = +1
C64 = 0
C128 = 1
C64_SPLIT_F16 = 2
C64_SPLIT_BF16 = 3
C64_SPLIT3_BF16 = 4
C64_F16 = 5
DTYPES = {"c64": C64, "complex64": C64, C64: C64, "c128": C128, "complex128": C128, C128: C128,
          "split_f16": C64_SPLIT_F16, C64_SPLIT_F16: C64_SPLIT_F16,
          "split_bf16": C64_SPLIT_BF16, C64_SPLIT_BF16: C64_SPLIT_BF16,
          "split3_bf16": C64_SPLIT3_BF16, C64_SPLIT3_BF16: C64_SPLIT3_BF16,
          "f16": C64_F16, C64_F16: C64_F16}

VARIANT_NAMES = {0: "single_specialised", 1: "single_generic", 2: "two_pass", 3: "mixed_persistent",
                 4: "split_mfma", 5: "formula", 6: "order"}

# factorisation orders
ORDER_STOCKHAM = 0
ORDER_CT = 1
ORDER_PEASE = 2
ORDER_FOURSTEP = 3
ORDER_WAVE = 4
ORDER_NAMES = {0: "stockham", 1: "ct", 2: "pease", 3: "fourstep", 4: "wave"}
MIXED_LAUNCH_GRAPH = 0
MIXED_LAUNCH_DIRECT = 1

# formula plan flags
FORMULA_NO_FOLD = 1
FORMULA_EQ2 = 2
FORMULA_HBM_PASSES = 4

STATUS = {0: "FFTC_OK", 1: "FFTC_ERR_INVALID_ARG", 2: "FFTC_ERR_UNSUPPORTED_SIZE",
          3: "FFTC_ERR_OUT_OF_MEMORY", 4: "FFTC_ERR_TOO_LARGE", 5: "FFTC_ERR_HIP",
          6: "FFTC_ERR_SHUTDOWN", 7: "FFTC_ERR_INTERNAL"}


class FFTCError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")


class Layout(ctypes.Structure):
    _fields_ = [("stride", ctypes.c_int64), ("dist", ctypes.c_int64), ("planar", ctypes.c_int)]


class PlanDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("batch", ctypes.c_int64), ("direction", ctypes.c_int),
                ("dtype", ctypes.c_int), ("variant", ctypes.c_int), ("nradices", ctypes.c_int),
                ("radices", ctypes.c_int * 16), ("threads_per_transform", ctypes.c_int),
                ("transforms_per_group", ctypes.c_int), ("split_m", ctypes.c_int64),
                ("split_k", ctypes.c_int64), ("twiddle_bytes", ctypes.c_size_t),
                ("scratch_bytes", ctypes.c_size_t), ("mixed_transforms", ctypes.c_int64),
                ("mixed_elements", ctypes.c_int64), ("mixed_classes", ctypes.c_int),
                ("mixed_items", ctypes.c_int), ("persistent_groups", ctypes.c_int),
                ("formula_passes", ctypes.c_int), ("formula_folded", ctypes.c_int),
                ("formula_lds", ctypes.c_int), ("formula_fold_n", ctypes.c_int64),
                ("formula_fold_p", ctypes.c_int64), ("formula_kernels", ctypes.c_int),
                ("has_layout", ctypes.c_int), ("layout_in", Layout), ("layout_out", Layout),
                ("order", ctypes.c_int), ("order_radix", ctypes.c_int)]


_i64, _int, _vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
_SIGNATURES = {
    "fftc_plan": (_int, [_i64, _i64, _int, _int, ctypes.POINTER(_vp)]),
    "fftc_plan_radices": (_int, [_i64, _i64, _int, _int, ctypes.POINTER(_int), _int, ctypes.POINTER(_vp)]),
    "fftc_execute": (_int, [_vp, _vp, _vp, _vp]),
    "fftc_execute_batch": (_int, [_vp, _vp, _vp, _i64, _vp]),
    "fftc_destroy_plan": (_int, [_vp]),
    "fftc_plan_describe": (_int, [_vp, ctypes.POINTER(PlanDesc)]),
    "fftc_factorize": (_int, [_i64, _int, ctypes.POINTER(_int), _int, ctypes.POINTER(_int),
                              ctypes.POINTER(_i64)]),
    "fftc_max_single_n": (_i64, [_int]),
    "fftc_copy": (_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "fftc_compiled_count": (_int, [_int]),
    "fftc_compiled_entry": (_int, [_int, _int, ctypes.POINTER(_i64), ctypes.POINTER(_int), _int,
                                   ctypes.POINTER(_int)]),
    "fftc_candidates": (_int, [_i64, ctypes.POINTER(_int), ctypes.POINTER(_int), _int, ctypes.POINTER(_int)]),
    "fftc_plan_mixed": (_int, [ctypes.POINTER(_i64), _i64, _int, _int, ctypes.POINTER(_vp)]),
    "fftc_plan_mixed_set_launch": (_int, [_vp, _int]),
    "fftc_autotune": (_int, [_i64, _i64, _int, _int, ctypes.POINTER(_int), _int, ctypes.POINTER(_int),
                             ctypes.POINTER(ctypes.c_double)]),
    "fftc_tune_load": (_int, [ctypes.c_char_p, ctypes.POINTER(_int)]),
    "fftc_tune_save": (_int, [ctypes.c_char_p, ctypes.POINTER(_int)]),
    "fftc_tune_clear": (_int, []),
    "fftc_tune_key": (ctypes.c_char_p, []),
    "fftc_plan_formula": (_int, [ctypes.c_char_p, _i64, _int, _int, _int, ctypes.POINTER(_vp)]),
    "fftc_formula_lower": (_int, [ctypes.c_char_p, _int, _int, ctypes.POINTER(_i64), ctypes.c_char_p,
                                  ctypes.c_size_t]),
    "fftc_formula_max_lds_dim": (_i64, [_int]),
    "fftc_plan_layout": (_int, [_i64, _i64, _int, _int, ctypes.POINTER(Layout), ctypes.POINTER(Layout),
                                ctypes.POINTER(_vp)]),
    "fftc_execute_layout": (_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "fftc_plan_order": (_int, [_i64, _i64, _int, _int, _int, _int, ctypes.POINTER(_vp)]),
    "fftc_order_count": (_int, [_int]),
    "fftc_order_entry": (_int, [_int, _int, ctypes.POINTER(_i64), ctypes.POINTER(_int), ctypes.POINTER(_int)]),
    "fftc_autotune_orders": (_int, [_i64, _i64, _int, _int, ctypes.POINTER(_int), ctypes.POINTER(_int),
                                    ctypes.POINTER(ctypes.c_double), _int, ctypes.POINTER(_int),
                                    ctypes.POINTER(_int)]),
    "fftc_execute_static": (_int, [_i64, _i64, _int, _int, _vp, _vp, _vp]),
    "fftc_static_scratch_bytes": (ctypes.c_size_t, []),
    "fftc_status_string": (ctypes.c_char_p, [_int]),
    "fftc_last_error": (ctypes.c_char_p, []),
}


def _load() -> ctypes.CDLL:
    # PyTorch-ROCm carries its own HIP runtime (libamdhip64.so.7).  Import it
    # first so libfftc.so binds to that same runtime (same soname) and the
    # process holds one HIP runtime shared by torch's allocations/streams and
    # fftc's launches.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950); there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


class _Declared:
    """The library with only its declared entry points visible: ctypes would
    pass undeclared arguments as 32-bit ints (truncating device pointers)."""

    def __init__(self, so: ctypes.CDLL):
        self._so = so
        self._fns = {name: getattr(so, name) for name in _SIGNATURES}

    def declare(self, name: str, restype, argtypes) -> None:
        fn = getattr(self._so, name)
        fn.restype = restype
        fn.argtypes = argtypes
        self._fns[name] = fn

    def __getattr__(self, name):
        try:
            return self.__dict__["_fns"][name]
        except KeyError:
            raise AttributeError(f"{name} has no declared signature; call fftc.register first") from None


lib = _Declared(_load())


def register(name: str, restype, argtypes) -> None:
    """Declare the signature of a further C entry point of the library."""
    lib.declare(name, restype, argtypes)


def last_error() -> str:
    return (lib.fftc_last_error() or b"").decode()


def check(status: int, where: str) -> None:
    if status != 0:
        raise FFTCError(status, where, last_error())


def ptr(x) -> int:
    """Device address of a tensor (data_ptr()) or an integer address."""
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def check_extent(t, nbytes: int, what: str, device=None) -> None:
    """Refuse a tensor the kernels cannot use as a dense device buffer of at
    least `nbytes` (integer addresses are the caller's responsibility): a host
    tensor, one on another GPU than the plan's, a non-contiguous view (the
    kernels ignore torch strides and would read and write the storage between
    its elements), or one smaller than what the launch touches (the kernels
    cannot see a buffer's size, and an access past its end faults the GPU)."""
    if t is None or isinstance(t, int):
        return
    dev = getattr(t, "device", None)
    if dev is not None:
        if getattr(dev, "type", "cuda") != "cuda":
            raise FFTCError(1, f"{what} buffer", f"{what} tensor is on {dev}, not on a GPU")
        if device is not None and dev.index is not None and dev.index != device:
            raise FFTCError(1, f"{what} buffer", f"{what} tensor is on {dev}, the plan on cuda:{device}")
    try:
        contiguous = t.is_contiguous()
        have = t.nbytes
    except AttributeError:  # not a tensor: an object with data_ptr() only
        return
    if not contiguous:
        raise FFTCError(1, f"{what} buffer", f"{what} tensor is a non-contiguous view")
    if have < nbytes:
        raise FFTCError(1, f"{what} buffer",  # FFTC_ERR_INVALID_ARG
                        f"{what} tensor spans {have} bytes, the plan touches {nbytes}")


def _current_device():
    """Index of the GPU plans are created on (HIP's current device, which
    torch's current device sets), or None without a usable torch."""
    try:
        import torch
        return int(torch.cuda.current_device()) if torch.cuda.is_available() else None
    except Exception:
        return None


def stream_handle(stream) -> int:
    """hipStream_t of a torch stream, an int handle, or torch's current stream."""
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def dtype_code(dtype) -> int:
    if dtype in DTYPES:
        return DTYPES[dtype]
    s = str(dtype).replace("torch.", "")
    if s in DTYPES:
        return DTYPES[s]
    raise ValueError(f"unsupported dtype {dtype!r}")


class Plan:
    """Owns an fftc_plan_t; destroyed by close() or garbage collection."""

    def __init__(self, n: int, batch: int, direction: int = FORWARD, dtype="c64", radices=None,
                 _handle=None):
        code = dtype_code(dtype)
        self.device = _current_device()
        if _handle is not None:
            self._h = _handle
            self.n, self.batch, self.direction, self.dtype = n, batch, direction, code
            return
        h = _vp()
        if radices is None:
            check(lib.fftc_plan(n, batch, direction, code, ctypes.byref(h)), "fftc_plan")
        else:
            arr = (_int * max(1, len(radices)))(*radices)
            check(lib.fftc_plan_radices(n, batch, direction, code, arr, len(radices), ctypes.byref(h)),
                  "fftc_plan_radices")
        self._h = h
        self.n, self.batch, self.direction, self.dtype = n, batch, direction, code

    @property
    def handle(self) -> int:
        return self._h.value or 0

    def bytes_needed(self, batch=None) -> tuple:
        """(input bytes, output bytes) one execute of the first `batch`
        transforms (default: the plan's batch) reads and writes; a layout side
        counts from its first to its last element (per array when planar)."""
        d = self.__dict__.get("_desc")
        if d is None:
            d = self._desc = self.describe()
        cs = 16 if d["dtype"] == C128 else 8
        if d["variant"] == "mixed_persistent":
            return (d["mixed_elements"] * cs,) * 2
        b = d["batch"] if batch is None else int(batch)
        if b <= 0:
            return (0, 0)
        if d["has_layout"]:
            def side(layout):
                stride, dist, planar = layout
                last = (b - 1) * dist + (d["n"] - 1) * stride
                return (last + 1) * (cs // 2 if planar else cs)
            return (side(d["layout_in"]), side(d["layout_out"]))
        return (d["n"] * b * cs,) * 2

    def execute(self, x, y, stream=None) -> None:
        """Enqueue y = DFT(x) on the stream (default: torch's current stream)."""
        nin, nout = self.bytes_needed()
        check_extent(x, nin, "input", self.device)
        check_extent(y, nout, "output", self.device)
        check(lib.fftc_execute(self._h, ptr(x), ptr(y), stream_handle(stream)), "fftc_execute")

    def execute_batch(self, x, y, batch: int, stream=None) -> None:
        """Enqueue the first `batch` transforms (1 <= batch <= the plan's batch;
        the library refuses any other count before touching memory)."""
        if self.batch and 0 < int(batch) <= self.batch:
            nin, nout = self.bytes_needed(batch)
            check_extent(x, nin, "input", self.device)
            check_extent(y, nout, "output", self.device)
        check(lib.fftc_execute_batch(self._h, ptr(x), ptr(y), int(batch), stream_handle(stream)),
              "fftc_execute_batch")

    def set_mixed_launch(self, mode: int) -> None:
        """Mixed plans: MIXED_LAUNCH_GRAPH (replay the plan's hipGraph, the
        default) or MIXED_LAUNCH_DIRECT (launch the same kernel on the stream)."""
        check(lib.fftc_plan_mixed_set_launch(self._h, int(mode)), "fftc_plan_mixed_set_launch")

    def describe(self) -> dict:
        d = PlanDesc()
        check(lib.fftc_plan_describe(self._h, ctypes.byref(d)), "fftc_plan_describe")
        return {"n": d.n, "batch": d.batch, "direction": d.direction, "dtype": d.dtype,
                "variant": VARIANT_NAMES.get(d.variant, d.variant),
                "radices": list(d.radices[:d.nradices]),
                "threads_per_transform": d.threads_per_transform,
                "transforms_per_group": d.transforms_per_group,
                "split_m": d.split_m, "split_k": d.split_k,
                "twiddle_bytes": d.twiddle_bytes, "scratch_bytes": d.scratch_bytes,
                "mixed_transforms": d.mixed_transforms, "mixed_elements": d.mixed_elements,
                "mixed_classes": d.mixed_classes, "mixed_items": d.mixed_items,
                "persistent_groups": d.persistent_groups,
                "formula_passes": d.formula_passes, "formula_folded": bool(d.formula_folded),
                "formula_lds": bool(d.formula_lds), "formula_fold_n": d.formula_fold_n,
                "formula_fold_p": d.formula_fold_p, "formula_kernels": d.formula_kernels,
                "has_layout": bool(d.has_layout),
                "layout_in": (d.layout_in.stride, d.layout_in.dist, d.layout_in.planar),
                "layout_out": (d.layout_out.stride, d.layout_out.dist, d.layout_out.planar),
                "order": ORDER_NAMES.get(d.order, d.order), "order_radix": d.order_radix}

    def close(self) -> None:
        if self._h is not None and self._h.value:
            check(lib.fftc_destroy_plan(self._h), "fftc_destroy_plan")
        self._h = _vp()

    def __del__(self):
        try:
            if self._h is not None and self._h.value:
                lib.fftc_destroy_plan(self._h)
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def plan_mixed(lengths, direction: int = FORWARD, dtype="c64") -> Plan:
    """One persistent-launch plan for transforms of the given lengths, packed
    back to back in that order."""
    lens = [int(v) for v in lengths]
    arr = (_i64 * len(lens))(*lens)
    h = _vp()
    check(lib.fftc_plan_mixed(arr, len(lens), direction, dtype_code(dtype), ctypes.byref(h)),
          "fftc_plan_mixed")
    p = Plan(0, len(lens), direction, dtype, _handle=h)
    p.lengths = lens
    return p


def plan_formula(formula: str, batch: int, direction: int = FORWARD, dtype="c64", flags: int = 0) -> Plan:
    """Plan applying a Kronecker-product formula (the DSL of the paper's
    Section IV-A) to `batch` contiguous vectors of its size."""
    h = _vp()
    check(lib.fftc_plan_formula(formula.encode(), batch, direction, dtype_code(dtype), flags,
                                ctypes.byref(h)), "fftc_plan_formula")
    d = PlanDesc()
    check(lib.fftc_plan_describe(h, ctypes.byref(d)), "fftc_plan_describe")
    p = Plan(int(d.n), batch, direction, dtype, _handle=h)
    p.formula = formula
    return p


def formula_lower(formula: str, flags: int = 0, dtype="c64"):
    """Host only: (size, lowering text) of a formula -- the folded formula and
    its pass list; raises FFTCError on a syntax or shape error."""
    dim = _i64()
    buf = ctypes.create_string_buffer(1 << 16)
    check(lib.fftc_formula_lower(formula.encode(), flags, dtype_code(dtype), ctypes.byref(dim), buf,
                                 len(buf)), "fftc_formula_lower")
    return dim.value, buf.value.decode()


def formula_max_lds_dim(dtype="c64") -> int:
    return int(lib.fftc_formula_max_lds_dim(dtype_code(dtype)))


def plan_layout(n: int, batch: int, direction: int = FORWARD, dtype="c64", in_layout=None, out_layout=None) -> Plan:
    """Plan reading and writing planar and/or strided data.  A layout is
    (stride, dist, planar) in elements; None = interleaved contiguous."""
    def mk(l):
        return None if l is None else ctypes.byref(Layout(int(l[0]), int(l[1]), int(l[2])))
    h = _vp()
    check(lib.fftc_plan_layout(n, batch, direction, dtype_code(dtype), mk(in_layout), mk(out_layout),
                               ctypes.byref(h)), "fftc_plan_layout")
    return Plan(n, batch, direction, dtype, _handle=h)


def execute_layout(plan: Plan, in_re, in_im, out_re, out_im, stream=None) -> None:
    """Run a layout plan: planar sides give (re, im), interleaved sides (array, None)."""
    nin, nout = plan.bytes_needed()
    for t, n, what in ((in_re, nin, "input"), (in_im, nin, "input (im)"), (out_re, nout, "output"),
                       (out_im, nout, "output (im)")):
        check_extent(t, n, what, plan.device)
    check(lib.fftc_execute_layout(plan._h, ptr(in_re), ptr(in_im) or None, ptr(out_re), ptr(out_im) or None,
                                  stream_handle(stream)), "fftc_execute_layout")


def plan_order(n: int, batch: int, direction: int = FORWARD, dtype="c64", order=ORDER_CT, radix: int = 2) -> Plan:
    """Plan running an alternative factorisation order (ORDER_CT / ORDER_PEASE / ORDER_FOURSTEP /
    ORDER_WAVE)."""
    h = _vp()
    check(lib.fftc_plan_order(n, batch, direction, dtype_code(dtype), int(order), int(radix), ctypes.byref(h)),
          "fftc_plan_order")
    return Plan(n, batch, direction, dtype, _handle=h)


def compiled_orders(dtype="c64"):
    """(n, order, radix) of every compiled alternative-order kernel."""
    code = dtype_code(dtype)
    out = []
    for i in range(lib.fftc_order_count(code)):
        n, o, r = _i64(), _int(), _int()
        check(lib.fftc_order_entry(code, i, ctypes.byref(n), ctypes.byref(o), ctypes.byref(r)), "fftc_order_entry")
        out.append((n.value, o.value, r.value))
    return out


def autotune_orders(n: int, batch: int, dtype="c64", reps: int = 10):
    """Time Stockham and every compiled order for n; returns ([(order, radix, us)], best index)."""
    m = 64
    orders, radices, us = (_int * m)(), (_int * m)(), (ctypes.c_double * m)()
    cnt, best = _int(), _int()
    check(lib.fftc_autotune_orders(n, batch, dtype_code(dtype), reps, orders, radices, us, m, ctypes.byref(cnt),
                                   ctypes.byref(best)), "fftc_autotune_orders")
    return [(ORDER_NAMES[orders[i]], radices[i], us[i]) for i in range(cnt.value)], best.value


def autotune(n: int, batch: int, dtype="c64", reps: int = 10):
    """Time every candidate radix list for n on the device; record and return
    the fastest (list, microseconds per launch)."""
    arr = (_int * 32)()
    cnt = _int()
    us = ctypes.c_double()
    check(lib.fftc_autotune(n, batch, dtype_code(dtype), reps, arr, 32, ctypes.byref(cnt),
                            ctypes.byref(us)), "fftc_autotune")
    return list(arr[:cnt.value]), us.value


def tune_load(path: str) -> int:
    k = _int()
    check(lib.fftc_tune_load(path.encode(), ctypes.byref(k)), "fftc_tune_load")
    return k.value


def tune_save(path: str) -> int:
    k = _int()
    check(lib.fftc_tune_save(path.encode(), ctypes.byref(k)), "fftc_tune_save")
    return k.value


def tune_key() -> str:
    """'<arch> <toolchain>' that a tuning-database line must start with."""
    return lib.fftc_tune_key().decode()


def tune_clear() -> None:
    check(lib.fftc_tune_clear(), "fftc_tune_clear")


def factorize(n: int, dtype="c64"):
    """Radix list the planner picks for n (host only), and the two-pass split m (0 if none)."""
    arr = (_int * 32)()
    cnt = _int()
    m = _i64()
    check(lib.fftc_factorize(n, dtype_code(dtype), arr, 32, ctypes.byref(cnt), ctypes.byref(m)),
          "fftc_factorize")
    return list(arr[:cnt.value]), m.value


def candidates(n: int):
    """Candidate radix lists for single-kernel length n, preference order."""
    flat = (_int * (16 * 12))()
    lens = (_int * 12)()
    cnt = _int()
    check(lib.fftc_candidates(n, flat, lens, 12, ctypes.byref(cnt)), "fftc_candidates")
    return [list(flat[i * 16:i * 16 + lens[i]]) for i in range(min(cnt.value, 12))]


def compiled_lists(dtype="c64"):
    """(n, radix list) of every specialised kernel compiled for dtype."""
    code = dtype_code(dtype)
    out = []
    for i in range(lib.fftc_compiled_count(code)):
        n = _i64()
        arr = (_int * 16)()
        cnt = _int()
        check(lib.fftc_compiled_entry(code, i, ctypes.byref(n), arr, 16, ctypes.byref(cnt)),
              "fftc_compiled_entry")
        out.append((n.value, list(arr[:cnt.value])))
    return out


def copy(x, y, nbytes: int, stream=None) -> None:
    """Device copy of nbytes from x to y with 16-byte nontemporal accesses
    (the library's bandwidth reference)."""
    check_extent(x, int(nbytes), "copy source")
    check_extent(y, int(nbytes), "copy destination")
    check(lib.fftc_copy(ptr(x), ptr(y), int(nbytes), stream_handle(stream)), "fftc_copy")


def execute_static(n: int, batch: int, x, y, direction: int = FORWARD, dtype="c64", stream=None) -> None:
    """Plan and run `batch` transforms of length n in one call that allocates
    no device memory (tables and any in-place intermediate in the library's
    static device array); calls overlapping in time on one GPU race."""
    code = dtype_code(dtype)
    nbytes = int(n) * int(batch) * (16 if code == C128 else 8)
    dev = _current_device()
    check_extent(x, nbytes, "input", dev)
    check_extent(y, nbytes, "output", dev)
    check(lib.fftc_execute_static(int(n), int(batch), int(direction), code, ptr(x), ptr(y), stream_handle(stream)),
          "fftc_execute_static")


def static_scratch_bytes() -> int:
    return int(lib.fftc_static_scratch_bytes())


def max_single_n(dtype="c64") -> int:
    return int(lib.fftc_max_single_n(dtype_code(dtype)))


def status_string(code: int) -> str:
    return lib.fftc_status_string(code).decode()
