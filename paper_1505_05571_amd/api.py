"""ctypes binding to ``libexsum.so`` (the C ABI of ``include/exsum.h``).

Argument marshalling only: every step of every sum runs in the library's HIP
kernels.  Tensors must be CUDA (HIP) tensors; results are written into device
tensors on the caller's current stream.  There is no CPU fallback: if the
library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

__all__ = [
    "ExsumError", "ExsumConfig", "library_path", "load_library",
    "exsum_f64", "exsum_f64_noalloc", "exsum_segmented_f64", "exsum_check_offsets", "exsum_inexact_f64",
    "exsum_f64_cfg",
    "exsum_get_config", "exsum_set_config", "exsum_release", "exsum_status_string",
    "exsum_autotune", "exsum_load_tuning", "exsum_large_variants",
    "ServerConfig", "Server", "exsum_server_default_config", "exsum_server_plan", "exsum_serial_replay",
    "exsum_sqnorm_f64", "exsum_dot_f64", "exsum_mean_f64", "exsum_f32", "exsum_dot_f32", "Accumulator",
    "EXSUM_ACC_BYTES",
    "EXPORTED_SYMBOLS",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libexsum.so")
_lock = threading.Lock()
_lib = None

EXSUM_OK, EXSUM_EINVAL, EXSUM_ENOMEM, EXSUM_EDEVICE = 0, 1, 2, 3

# every function include/exsum.h declares
EXPORTED_SYMBOLS = [
    "exsum_status_string", "exsum_f64", "exsum_segmented_f64", "exsum_inexact_f64",
    "exsum_get_config", "exsum_set_config", "exsum_f64_cfg", "exsum_release",
    "exsum_server_default_config", "exsum_server_create", "exsum_server_destroy", "exsum_server_submit",
    "exsum_server_step", "exsum_server_poll", "exsum_server_drain", "exsum_server_pending",
    "exsum_server_replay", "exsum_serial_replay", "exsum_server_plan",
    "exsum_sqnorm_f64", "exsum_dot_f64", "exsum_mean_f64", "exsum_f32",
    "exsum_acc_zero", "exsum_acc_add_f64", "exsum_acc_merge", "exsum_acc_round_f64",
    "exsum_autotune", "exsum_load_tuning", "exsum_dot_f32", "exsum_check_offsets",
    "exsum_large_variants", "exsum_f64_noalloc",
]

EXSUM_ACC_BYTES = 576


class ExsumError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__("%s failed: %s (status %d)" % (what, _status_text(status), status))


class ExsumConfig(ctypes.Structure):
    _fields_ = [
        ("large_block", ctypes.c_int32),
        ("large_vec", ctypes.c_int32),
        ("large_depth", ctypes.c_int32),
        ("large_mode", ctypes.c_int32),
        ("large_grid", ctypes.c_int32),
        ("precombine", ctypes.c_int32),
        ("small_max", ctypes.c_int64),
        ("small_grid", ctypes.c_int32),
        ("seg_grid", ctypes.c_int32),
        ("seg_small_max", ctypes.c_int64),
        ("seg_mode", ctypes.c_int32),
        ("seg_block", ctypes.c_int32),
        ("seg_group", ctypes.c_int32),
        ("seg_pad", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("step_terms", ctypes.c_int64),
        ("piece_terms", ctypes.c_int64),
        ("short_max", ctypes.c_int64),
        ("max_slots", ctypes.c_int32),
        ("max_pieces", ctypes.c_int32),
        ("max_inflight", ctypes.c_int32),
        ("precombine", ctypes.c_int32),
        ("mem_budget", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libexsum.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("libexsum.so is not built (run __graft_entry__.build() or "
                               "python -m paper_1505_05571_amd.build); there is no fallback")
        # PyTorch first, so that the library and PyTorch share one HIP runtime
        # (PyTorch's): loaded the other way round, the library's first device
        # query can find no device
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(_LIB_PATH)
        P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.exsum_status_string.argtypes = [I32]
        lib.exsum_status_string.restype = ctypes.c_char_p
        lib.exsum_f64.argtypes = [P, I64, P, P]
        lib.exsum_f64_noalloc.argtypes = [P, I64, P, P]
        lib.exsum_f64_noalloc.restype = I32
        lib.exsum_f64.restype = I32
        lib.exsum_f64_cfg.argtypes = [P, I64, P, P, ctypes.POINTER(ExsumConfig)]
        lib.exsum_f64_cfg.restype = I32
        lib.exsum_segmented_f64.argtypes = [P, P, I64, P, P]
        lib.exsum_segmented_f64.restype = I32
        lib.exsum_inexact_f64.argtypes = [P, I64, P, P]
        lib.exsum_inexact_f64.restype = I32
        lib.exsum_get_config.argtypes = [ctypes.POINTER(ExsumConfig)]
        lib.exsum_get_config.restype = I32
        lib.exsum_set_config.argtypes = [ctypes.POINTER(ExsumConfig)]
        lib.exsum_set_config.restype = I32
        lib.exsum_release.argtypes = []
        lib.exsum_release.restype = I32
        PCFG = ctypes.POINTER(ServerConfig)
        PI64 = ctypes.POINTER(ctypes.c_int64)
        lib.exsum_server_default_config.argtypes = [PCFG]
        lib.exsum_server_create.argtypes = [PCFG, P, ctypes.POINTER(P)]
        lib.exsum_server_destroy.argtypes = [P]
        lib.exsum_server_submit.argtypes = [P, P, I64, P, PI64]
        lib.exsum_server_step.argtypes = [P, PI64]
        lib.exsum_server_poll.argtypes = [P, P, I64, PI64]
        lib.exsum_server_drain.argtypes = [P]
        lib.exsum_server_pending.argtypes = [P, PI64]
        lib.exsum_server_replay.argtypes = [P, P, P, P, P, I64, P, P, ctypes.POINTER(ctypes.c_double)]
        lib.exsum_serial_replay.argtypes = [P, P, P, P, I64, P, P, P, ctypes.POINTER(ctypes.c_double)]
        lib.exsum_server_plan.argtypes = [PCFG, P, I64, I64, P, P, P, P, P, P, PI64]
        lib.exsum_sqnorm_f64.argtypes = [P, I64, P, P]
        lib.exsum_dot_f64.argtypes = [P, P, I64, P, P]
        lib.exsum_mean_f64.argtypes = [P, I64, P, P]
        lib.exsum_f32.argtypes = [P, I64, P, P]
        lib.exsum_dot_f32.argtypes = [P, P, I64, P, P]
        lib.exsum_dot_f32.restype = I32
        lib.exsum_check_offsets.argtypes = [P, I64, I64, P, P]
        lib.exsum_check_offsets.restype = I32
        lib.exsum_acc_zero.argtypes = [P, P]
        lib.exsum_acc_add_f64.argtypes = [P, P, I64, P]
        lib.exsum_acc_merge.argtypes = [P, P, P]
        lib.exsum_acc_round_f64.argtypes = [P, P, P]
        lib.exsum_autotune.argtypes = [ctypes.c_char_p, ctypes.c_char_p, I64, P]
        lib.exsum_autotune.restype = I32
        lib.exsum_large_variants.argtypes = [P, I64, ctypes.POINTER(I64)]
        lib.exsum_large_variants.restype = I32
        lib.exsum_load_tuning.argtypes = [ctypes.c_char_p]
        lib.exsum_load_tuning.restype = I32
        for name in ("exsum_sqnorm_f64", "exsum_dot_f64", "exsum_mean_f64", "exsum_f32", "exsum_acc_zero",
                     "exsum_acc_add_f64", "exsum_acc_merge", "exsum_acc_round_f64"):
            getattr(lib, name).restype = I32
        for name in ("exsum_server_default_config", "exsum_server_create", "exsum_server_destroy",
                     "exsum_server_submit", "exsum_server_step", "exsum_server_poll", "exsum_server_drain",
                     "exsum_server_pending", "exsum_server_replay", "exsum_serial_replay", "exsum_server_plan"):
            getattr(lib, name).restype = I32
        _lib = lib
        return lib


def _status_text(status: int) -> str:
    try:
        return load_library().exsum_status_string(status).decode()
    except Exception:  # library missing while formatting an error
        return "status %d" % status


def exsum_status_string(status: int) -> str:
    return load_library().exsum_status_string(int(status)).decode()


def _check(status: int, what: str):
    if status != EXSUM_OK:
        raise ExsumError(status, what)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _dev_f64(x, name="x"):
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("%s must be a device (HIP) tensor" % name)
    if x.dtype != torch.float64:
        raise TypeError("%s must be float64" % name)
    if not x.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return x


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t.numel() else ctypes.c_void_p(t.data_ptr() or 0)


def _out1(x, out):
    import torch
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=x.device)
    return _dev_f64(out, "out")


def exsum_f64(x, out=None, stream=None):
    """Correctly rounded exact sum of a float64 device tensor -> 1-element tensor."""
    x = _dev_f64(x)
    out = _out1(x, out)
    _check(load_library().exsum_f64(_ptr(x), x.numel(), _ptr(out), _stream_handle(stream)), "exsum_f64")
    return out


def exsum_f64_noalloc(x, out, stream=None):
    """exsum_f64 through the entry point that allocates nothing (a static
    per-device scratch accumulator); `out` must be given, so that no
    allocation happens here either."""
    x = _dev_f64(x)
    out = _dev_f64(out, "out")
    _check(load_library().exsum_f64_noalloc(_ptr(x), x.numel(), _ptr(out), _stream_handle(stream)),
           "exsum_f64_noalloc")
    return out


def exsum_f64_cfg(x, cfg: ExsumConfig, out=None, stream=None):
    """exsum_f64 with an explicit launch configuration for this call."""
    x = _dev_f64(x)
    out = _out1(x, out)
    _check(load_library().exsum_f64_cfg(_ptr(x), x.numel(), _ptr(out), _stream_handle(stream),
                                         ctypes.byref(cfg)), "exsum_f64_cfg")
    return out


def exsum_inexact_f64(x, out=None, stream=None):
    """Ordinary (inexact) float64 tree sum over the same load path."""
    x = _dev_f64(x)
    out = _out1(x, out)
    _check(load_library().exsum_inexact_f64(_ptr(x), x.numel(), _ptr(out), _stream_handle(stream)),
           "exsum_inexact_f64")
    return out


def exsum_check_offsets(offsets, n=None, stream=None):
    """Validate segment offsets on the device: a 1-element int64 device tensor
    holding -1 when offsets[0] >= 0, the offsets do not decrease and (if n is
    given) offsets[-1] <= n, else the first segment index that breaks them."""
    import torch
    if not isinstance(offsets, torch.Tensor) or not offsets.is_cuda or offsets.dtype != torch.int64:
        raise TypeError("offsets must be an int64 device tensor")
    offsets = offsets.contiguous()
    nseg = max(offsets.numel() - 1, 0)
    first_bad = torch.empty(1, dtype=torch.int64, device=offsets.device)
    _check(load_library().exsum_check_offsets(_ptr(offsets), nseg, -1 if n is None else int(n), _ptr(first_bad),
                                               _stream_handle(stream)), "exsum_check_offsets")
    return first_bad


def exsum_segmented_f64(x, offsets, out=None, stream=None, check=True):
    """Exact sum of each segment x[offsets[i]:offsets[i+1]] (offsets: int64 device tensor).

    With ``check`` (the default) the offsets are first validated on the device
    against x's length (exsum_check_offsets) and a bad one raises ValueError
    before the sums run: the library itself trusts its offsets, and offsets
    past the end of x would read outside it.  The check waits for the stream;
    pass ``check=False`` for offsets known to be good, in timed loops and under
    HIP graph capture."""
    import torch
    x = _dev_f64(x)
    if not isinstance(offsets, torch.Tensor) or not offsets.is_cuda or offsets.dtype != torch.int64:
        raise TypeError("offsets must be an int64 device tensor")
    offsets = offsets.contiguous()
    nseg = max(offsets.numel() - 1, 0)
    if out is None:
        out = torch.empty(nseg, dtype=torch.float64, device=x.device)
    out = _dev_f64(out, "out")
    if out.numel() < nseg:
        raise ValueError("out is too small")
    if check and nseg > 0:
        bad = int(exsum_check_offsets(offsets, n=x.numel(), stream=stream).cpu()[0])
        if bad >= 0:
            raise ValueError("offsets of segment %d are out of order or outside x (%d terms)" % (bad, x.numel()))
    _check(load_library().exsum_segmented_f64(_ptr(x), _ptr(offsets), nseg, _ptr(out),
                                               _stream_handle(stream)), "exsum_segmented_f64")
    return out


def _dev_f32(x, name="x"):
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("%s must be a device (HIP) tensor" % name)
    if x.dtype != torch.float32:
        raise TypeError("%s must be float32" % name)
    if not x.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return x


def exsum_sqnorm_f64(x, out=None, stream=None):
    """Exact sum of x[i]*x[i] (products rounded to binary64), rounded once."""
    x = _dev_f64(x)
    out = _out1(x, out)
    _check(load_library().exsum_sqnorm_f64(_ptr(x), x.numel(), _ptr(out), _stream_handle(stream)),
           "exsum_sqnorm_f64")
    return out


def exsum_dot_f64(x, y, out=None, stream=None):
    """Exact sum of x[i]*y[i] (products rounded to binary64), rounded once."""
    x = _dev_f64(x)
    y = _dev_f64(y, "y")
    if y.numel() != x.numel():
        raise ValueError("x and y differ in length")
    out = _out1(x, out)
    _check(load_library().exsum_dot_f64(_ptr(x), _ptr(y), x.numel(), _ptr(out), _stream_handle(stream)),
           "exsum_dot_f64")
    return out


def exsum_mean_f64(x, out=None, stream=None):
    """Exact sum of x divided by its length, rounded once (n = 0 gives +0)."""
    x = _dev_f64(x)
    out = _out1(x, out)
    _check(load_library().exsum_mean_f64(_ptr(x), x.numel(), _ptr(out), _stream_handle(stream)),
           "exsum_mean_f64")
    return out


def exsum_f32(x, out=None, stream=None):
    """Exact sum of a float32 device tensor, rounded once to binary32."""
    import torch
    x = _dev_f32(x)
    if out is None:
        out = torch.empty(1, dtype=torch.float32, device=x.device)
    out = _dev_f32(out, "out")
    _check(load_library().exsum_f32(_ptr(x), x.numel(), _ptr(out), _stream_handle(stream)), "exsum_f32")
    return out


def exsum_dot_f32(x, y, out=None, stream=None):
    """Exact dot product of two float32 device tensors (products exact in
    binary64), rounded once to binary32."""
    import torch
    x = _dev_f32(x)
    y = _dev_f32(y, "y")
    if y.numel() != x.numel():
        raise ValueError("x and y differ in length")
    if out is None:
        out = torch.empty(1, dtype=torch.float32, device=x.device)
    out = _dev_f32(out, "out")
    _check(load_library().exsum_dot_f32(_ptr(x), _ptr(y), x.numel(), _ptr(out), _stream_handle(stream)),
           "exsum_dot_f32")
    return out


class Accumulator:
    """A device-resident exact accumulator (EXSUM_ACC_BYTES of device memory):
    add terms in any number of calls, merge accumulators, round at any time."""

    def __init__(self, device="cuda:0", stream=None):
        import torch
        self.state = torch.empty(EXSUM_ACC_BYTES // 8, dtype=torch.int64, device=device)
        self._stream = stream
        self.zero()

    def _h(self):
        return ctypes.c_void_p(self.state.data_ptr())

    def zero(self):
        _check(load_library().exsum_acc_zero(self._h(), _stream_handle(self._stream)), "exsum_acc_zero")
        return self

    def add(self, x):
        x = _dev_f64(x)
        _check(load_library().exsum_acc_add_f64(self._h(), _ptr(x), x.numel(), _stream_handle(self._stream)),
               "exsum_acc_add_f64")
        return self

    def merge(self, other: "Accumulator"):
        _check(load_library().exsum_acc_merge(self._h(), other._h(), _stream_handle(self._stream)),
               "exsum_acc_merge")
        return self

    def round(self, out=None):
        import torch
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.state.device)
        out = _dev_f64(out, "out")
        _check(load_library().exsum_acc_round_f64(self._h(), _ptr(out), _stream_handle(self._stream)),
               "exsum_acc_round_f64")
        return out


def exsum_large_variants():
    """The large kernel's built (block, vec, depth, mode) shapes, as tuples."""
    lib = load_library()
    n = ctypes.c_int64(0)
    _check(lib.exsum_large_variants(None, 0, ctypes.byref(n)), "exsum_large_variants")
    buf = (ctypes.c_int32 * (4 * n.value))()
    _check(lib.exsum_large_variants(buf, n.value, ctypes.byref(n)), "exsum_large_variants")
    return [tuple(buf[4 * k:4 * k + 4]) for k in range(n.value)]


def exsum_get_config() -> ExsumConfig:
    cfg = ExsumConfig()
    _check(load_library().exsum_get_config(ctypes.byref(cfg)), "exsum_get_config")
    return cfg


def exsum_set_config(cfg: ExsumConfig) -> None:
    _check(load_library().exsum_set_config(ctypes.byref(cfg)), "exsum_set_config")


def exsum_autotune(cache_path: str | None = None, stream=None) -> dict:
    """Time candidate launch configurations on the current device, make the
    fastest the process configuration and return the tuner's JSON report
    (also written to cache_path if given)."""
    import json
    buf = ctypes.create_string_buffer(1 << 16)
    path = cache_path.encode() if cache_path else None
    st = load_library().exsum_autotune(path, buf, len(buf), _stream_handle(stream))
    if st != EXSUM_OK:
        detail = json.loads(buf.value.decode() or "{}").get("error", "")
        raise ExsumError(st, "exsum_autotune (%s)" % detail)
    return json.loads(buf.value.decode())


def exsum_load_tuning(cache_path: str) -> None:
    """Make the configuration stored by exsum_autotune() the process
    configuration (same kind of device only)."""
    _check(load_library().exsum_load_tuning(cache_path.encode()), "exsum_load_tuning")


def exsum_release() -> None:
    _check(load_library().exsum_release(), "exsum_release")


# ---------------------------------------------------------------------------
# serving loop
# ---------------------------------------------------------------------------

def _host_array(a, dtype, name):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, ctypes.c_void_p(a.ctypes.data if a.size else 0)


def exsum_server_default_config() -> ServerConfig:
    cfg = ServerConfig()
    _check(load_library().exsum_server_default_config(ctypes.byref(cfg)), "exsum_server_default_config")
    return cfg


def exsum_server_plan(lens, cfg: ServerConfig = None):
    """The server's plan for requests of the given lengths, all submitted at
    once (host only).  Returns a dict of numpy arrays: req, off, len, step,
    slot, expected (0xFFFFFFFF for pieces of steps that do not complete their
    request)."""
    import numpy as np
    lens, lp = _host_array(lens, np.int64, "lens")
    lib = load_library()
    cfgp = ctypes.byref(cfg) if cfg is not None else None
    count = ctypes.c_int64(0)
    _check(lib.exsum_server_plan(cfgp, lp, lens.size, 0, None, None, None, None, None, None,
                                 ctypes.byref(count)), "exsum_server_plan")
    n = count.value
    out = {k: np.zeros(n, dtype=t) for k, t in (("req", np.int64), ("off", np.int64), ("len", np.int64),
                                                   ("step", np.int64), ("slot", np.int32),
                                                   ("expected", np.uint32))}
    ptr = {k: ctypes.c_void_p(v.ctypes.data) for k, v in out.items()}
    _check(lib.exsum_server_plan(cfgp, lp, lens.size, n, ptr["req"], ptr["off"], ptr["len"], ptr["step"],
                                 ptr["slot"], ptr["expected"], ctypes.byref(count)), "exsum_server_plan")
    return out


class Server:
    """Continuous-batching exact-sum server on one stream (see exsum.h)."""

    def __init__(self, cfg: ServerConfig = None, stream=None):
        lib = load_library()
        self._lib = lib
        self._h = ctypes.c_void_p(0)
        self._stream = _stream_handle(stream)
        cfgp = ctypes.byref(cfg) if cfg is not None else None
        _check(lib.exsum_server_create(cfgp, self._stream, ctypes.byref(self._h)), "exsum_server_create")
        self._keep = {}                      # tensors of requests in flight

    def close(self):
        if self._h:
            st = self._lib.exsum_server_destroy(self._h)
            self._h = ctypes.c_void_p(0)
            self._keep.clear()
            _check(st, "exsum_server_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, x, out, out_index: int = 0) -> int:
        """Queue the exact sum of the float64 device tensor x into
        out[out_index]; returns the request id."""
        x = _dev_f64(x)
        out = _dev_f64(out, "out")
        if not 0 <= out_index < out.numel():
            raise IndexError("out_index out of range")
        rid = ctypes.c_int64(0)
        optr = ctypes.c_void_p(out.data_ptr() + 8 * out_index)
        _check(self._lib.exsum_server_submit(self._h, _ptr(x), x.numel(), optr, ctypes.byref(rid)),
               "exsum_server_submit")
        self._keep[rid.value] = (x, out)
        return rid.value

    def step(self) -> int:
        n = ctypes.c_int64(0)
        _check(self._lib.exsum_server_step(self._h, ctypes.byref(n)), "exsum_server_step")
        return n.value

    def poll(self, max_ids: int = 4096):
        import numpy as np
        ids = np.zeros(max_ids, dtype=np.int64)
        n = ctypes.c_int64(0)
        _check(self._lib.exsum_server_poll(self._h, ctypes.c_void_p(ids.ctypes.data), max_ids, ctypes.byref(n)),
               "exsum_server_poll")
        done = [int(i) for i in ids[:n.value]]
        for i in done:
            self._keep.pop(i, None)
        return done

    def drain(self):
        _check(self._lib.exsum_server_drain(self._h), "exsum_server_drain")

    def pending(self) -> int:
        n = ctypes.c_int64(0)
        _check(self._lib.exsum_server_pending(self._h, ctypes.byref(n)), "exsum_server_pending")
        return n.value

    def replay(self, pool, starts, lens, arrival_s, out):
        """Real-time replay of a trace (see exsum_server_replay).  Returns
        (latency_s numpy array, makespan_s)."""
        import numpy as np
        pool = _dev_f64(pool, "pool")
        out = _dev_f64(out, "out")
        starts, sp = _host_array(starts, np.int64, "starts")
        lens, lp = _host_array(lens, np.int64, "lens")
        arr, ap = _host_array(arrival_s, np.float64, "arrival_s")
        if not (starts.size == lens.size == arr.size) or out.numel() < lens.size:
            raise ValueError("trace arrays disagree in length")
        if lens.size and int((starts + lens).max()) > pool.numel():
            raise ValueError("a request runs past the end of the pool")
        lat = np.zeros(lens.size, dtype=np.float64)
        mk = ctypes.c_double(0.0)
        _check(self._lib.exsum_server_replay(self._h, _ptr(pool), sp, lp, ap, lens.size, _ptr(out),
                                             ctypes.c_void_p(lat.ctypes.data), ctypes.byref(mk)),
               "exsum_server_replay")
        return lat, mk.value


def exsum_serial_replay(pool, starts, lens, arrival_s, out, stream=None):
    """The same trace served by one exsum_f64 call per request, in arrival
    order on one stream.  Returns (latency_s, makespan_s)."""
    import numpy as np
    pool = _dev_f64(pool, "pool")
    out = _dev_f64(out, "out")
    starts, sp = _host_array(starts, np.int64, "starts")
    lens, lp = _host_array(lens, np.int64, "lens")
    arr, ap = _host_array(arrival_s, np.float64, "arrival_s")
    if not (starts.size == lens.size == arr.size) or out.numel() < lens.size:
        raise ValueError("trace arrays disagree in length")
    if lens.size and int((starts + lens).max()) > pool.numel():
        raise ValueError("a request runs past the end of the pool")
    lat = np.zeros(lens.size, dtype=np.float64)
    mk = ctypes.c_double(0.0)
    _check(load_library().exsum_serial_replay(_ptr(pool), sp, lp, ap, lens.size, _ptr(out), _stream_handle(stream),
                                               ctypes.c_void_p(lat.ctypes.data), ctypes.byref(mk)),
           "exsum_serial_replay")
    return lat, mk.value
