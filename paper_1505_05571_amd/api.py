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
    "exsum_f64", "exsum_segmented_f64", "exsum_inexact_f64", "exsum_f64_cfg",
    "exsum_get_config", "exsum_set_config", "exsum_release", "exsum_status_string",
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
]


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
        lib = ctypes.CDLL(_LIB_PATH)
        P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.exsum_status_string.argtypes = [I32]
        lib.exsum_status_string.restype = ctypes.c_char_p
        lib.exsum_f64.argtypes = [P, I64, P, P]
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


def exsum_segmented_f64(x, offsets, out=None, stream=None):
    """Exact sum of each segment x[offsets[i]:offsets[i+1]] (offsets: int64 device tensor)."""
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
    _check(load_library().exsum_segmented_f64(_ptr(x), _ptr(offsets), nseg, _ptr(out),
                                               _stream_handle(stream)), "exsum_segmented_f64")
    return out


def exsum_get_config() -> ExsumConfig:
    cfg = ExsumConfig()
    _check(load_library().exsum_get_config(ctypes.byref(cfg)), "exsum_get_config")
    return cfg


def exsum_set_config(cfg: ExsumConfig) -> None:
    _check(load_library().exsum_set_config(ctypes.byref(cfg)), "exsum_set_config")


def exsum_release() -> None:
    _check(load_library().exsum_release(), "exsum_release")
