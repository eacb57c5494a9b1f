"""CPU oracle for exact summation -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports it and
shares no code with it.

The arithmetic lives in ``exsum_oracle.c`` (plain C, wide-integer fixed point
in units of the smallest denormal, explicit round to nearest with ties to
even).  This module compiles it with gcc when the shared object is missing
and exposes thin ctypes wrappers that return result *bit patterns* (numpy
``uint64``/``uint32``) so NaN payloads and signed zeros survive intact.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "exsum_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
               "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.exo_sum_f64.argtypes = [P, I64]
        lib.exo_sum_f64.restype = ctypes.c_uint64
        lib.exo_segmented_f64.argtypes = [P, P, I64, P]
        lib.exo_segmented_f64.restype = None
        lib.exo_sum_ranges_f64.argtypes = [P, P, P, I64, P]
        lib.exo_sum_ranges_f64.restype = None
        lib.exo_mean_f64.argtypes = [P, I64]
        lib.exo_mean_f64.restype = ctypes.c_uint64
        lib.exo_dot_f64.argtypes = [P, P, I64]
        lib.exo_dot_f64.restype = ctypes.c_uint64
        lib.exo_sqnorm_f64.argtypes = [P, I64]
        lib.exo_sqnorm_f64.restype = ctypes.c_uint64
        lib.exo_sum_f32.argtypes = [P, I64]
        lib.exo_sum_f32.restype = ctypes.c_uint32
        lib.exo_dot_f32.argtypes = [P, P, I64]
        lib.exo_dot_f32.restype = ctypes.c_uint32
        lib.exo_ranges_by_prefix_f64.argtypes = [P, I64, P, P, I64, I64, ctypes.c_int, P]
        lib.exo_ranges_by_prefix_f64.restype = ctypes.c_int
        lib.exo_sum_f64_mt.argtypes = [P, I64, ctypes.c_int]
        lib.exo_sum_f64_mt.restype = ctypes.c_uint64
        _lib = lib
        return lib


def _f64(x) -> np.ndarray:
    a = np.ascontiguousarray(x, dtype=np.float64)
    return a


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def sum_f64(x) -> np.uint64:
    """Bits of the correctly rounded exact sum of binary64 values."""
    a = _f64(x)
    return np.uint64(_load().exo_sum_f64(_ptr(a), a.size))


def sum_f64_mt(x, nthreads: int) -> np.uint64:
    """As sum_f64, split over host threads (timing of the CPU baseline)."""
    a = _f64(x)
    return np.uint64(_load().exo_sum_f64_mt(_ptr(a), a.size, int(nthreads)))


def segmented_f64(x, offsets) -> np.ndarray:
    """Bits of the exact sum of each segment x[offsets[i]:offsets[i+1]]."""
    a = _f64(x)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    nseg = off.size - 1
    out = np.zeros(max(nseg, 0), dtype=np.uint64)
    if nseg > 0:
        _load().exo_segmented_f64(_ptr(a), _ptr(off), nseg, _ptr(out))
    return out


def sum_ranges_f64(x, starts, lens) -> np.ndarray:
    """Bits of the exact sum of x[starts[r]:starts[r]+lens[r]] for each r."""
    a = _f64(x)
    st = np.ascontiguousarray(starts, dtype=np.int64)
    ln = np.ascontiguousarray(lens, dtype=np.int64)
    out = np.zeros(st.size, dtype=np.uint64)
    if st.size:
        _load().exo_sum_ranges_f64(_ptr(a), _ptr(st), _ptr(ln), st.size, _ptr(out))
    return out


def ranges_by_prefix_f64(x, starts, lens, stride: int = 1 << 16, nthreads: int = 1) -> np.ndarray:
    """The same bits as sum_ranges_f64, through exact prefix sums every
    `stride` terms (a finite pool only): each range costs at most about
    2*stride terms, so long traces of slices of one pool are checked in full."""
    a = _f64(x)
    st = np.ascontiguousarray(starts, dtype=np.int64)
    ln = np.ascontiguousarray(lens, dtype=np.int64)
    out = np.zeros(st.size, dtype=np.uint64)
    rc = _load().exo_ranges_by_prefix_f64(_ptr(a), a.size, _ptr(st), _ptr(ln), st.size, int(stride),
                                          int(nthreads), _ptr(out))
    if rc == -1:
        raise ValueError("the pool holds an infinity or NaN; prefix sums need a finite pool")
    if rc != 0:
        raise ValueError("a range lies outside the pool, or stride < 1")
    return out


def mean_f64(x) -> np.uint64:
    """Bits of the correctly rounded exact mean (exact sum / n, one rounding)."""
    a = _f64(x)
    return np.uint64(_load().exo_mean_f64(_ptr(a), a.size))


def dot_f64(x, y) -> np.uint64:
    """Bits of the exact sum of the binary64-rounded products x[i]*y[i]."""
    a = _f64(x)
    b = _f64(y)
    assert a.size == b.size
    return np.uint64(_load().exo_dot_f64(_ptr(a), _ptr(b), a.size))


def sqnorm_f64(x) -> np.uint64:
    """Bits of the exact sum of the binary64-rounded squares x[i]*x[i]."""
    a = _f64(x)
    return np.uint64(_load().exo_sqnorm_f64(_ptr(a), a.size))


def sum_f32(x) -> np.uint32:
    """Bits of the correctly rounded (binary32) exact sum of binary32 values."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    return np.uint32(_load().exo_sum_f32(_ptr(a), a.size))


def dot_f32(x, y) -> np.uint32:
    """Bits of the exact dot product of two binary32 vectors, rounded once to
    binary32 (the products are exact in binary64)."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    b = np.ascontiguousarray(y, dtype=np.float32)
    assert a.size == b.size
    return np.uint32(_load().exo_dot_f32(_ptr(a), _ptr(b), a.size))


def bits_to_f64(b) -> float:
    return float(np.array([b], dtype=np.uint64).view(np.float64)[0])


def f64_to_bits(v) -> np.uint64:
    return np.array([v], dtype=np.float64).view(np.uint64)[0]
