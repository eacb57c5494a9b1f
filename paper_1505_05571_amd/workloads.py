"""Seeded synthetic inputs for exact summation.

This module only *draws* inputs; it holds none of the summation arithmetic.
Every value is built exactly (bit assembly or ``np.ldexp`` of a double by an
integer power of two), so generation itself never rounds.  The same arrays
feed the GPU library and the CPU oracle.

Workloads (sizes are the benchmark's; every function takes smaller sizes too):

* ``small_normal``      n=1000: sign uniform +-1, |N(0,1)| * 2^k, k uniform
                        integer in [-20, 20].  Small-accumulator-only size.
* ``uniform_exponent``  n=10^8: sign uniform, mantissa uniform [1, 2),
                        exponent uniform integer in [-300, 300].  Touches
                        1202 (sign, exponent) chunks.
* ``adversarial``       n=2^27: first half uniform [1, 2) all positive (one
                        hot chunk); second half x, -x pairs with
                        x = N(0,1) 2^40, every position = 999 (mod 1000) a
                        tiny N(0,1) 2^-60, and 1% of all terms near DBL_MAX
                        as +-y pairs (or all +y in the overflow variant).
* ``segments``          65536 segments, lengths lognormal(median 1000,
                        sigma 2) clipped to [1, 10^6]; values +-|N(0,1)| 2^k,
                        k uniform integer in [-30, 30].
* ``serve_trace``       request lengths log-uniform in [10, 10^8], each a
                        slice of one resident pool drawn like
                        ``uniform_exponent``.
* ``mirrored``          the timing distribution of the paper's Performance
                        evaluations section: first half U1 exp(30 U2), second
                        half the negated mirror image, so the exact sum is 0.
"""
from __future__ import annotations

import numpy as np

MANT_MASK = np.uint64((1 << 52) - 1)


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def small_normal(n: int = 1000, seed: int = 0, kmin: int = -20, kmax: int = 20) -> np.ndarray:
    """sign uniform, magnitude |N(0,1)| * 2^k with k uniform in [kmin, kmax]."""
    rng = _rng(seed)
    s = rng.integers(0, 2, size=n)
    k = rng.integers(kmin, kmax + 1, size=n)
    mag = np.abs(rng.standard_normal(n))
    x = np.ldexp(mag, k)
    return np.where(s == 1, -x, x)


def uniform_exponent(n: int = 10 ** 8, seed: int = 0, kmin: int = -300, kmax: int = 300,
                     chunk: int = 1 << 24) -> np.ndarray:
    """bits = s<<63 | (k+1023)<<52 | f, s uniform bit, k uniform integer in
    [kmin, kmax], f uniform 52-bit fraction (mantissa uniform in [1, 2)).
    Drawn in chunks of ``chunk`` terms to bound host memory; the draw order
    per chunk is s, k, f."""
    rng = _rng(seed)
    out = np.empty(n, dtype=np.uint64)
    for lo in range(0, n, chunk):
        m = min(chunk, n - lo)
        s = rng.integers(0, 2, size=m, dtype=np.uint64)
        k = rng.integers(kmin + 1023, kmax + 1023 + 1, size=m, dtype=np.uint64)
        f = rng.integers(0, 1 << 52, size=m, dtype=np.uint64)
        out[lo:lo + m] = (s << np.uint64(63)) | (k << np.uint64(52)) | f
    return out.view(np.float64)


def adversarial(n: int = 1 << 27, seed: int = 0, overflow: bool = False) -> np.ndarray:
    """The adversarial layout (n must be even and >= 2000).

    * positions [0, n/2): bits 0x3FF<<52 | f, f uniform 52-bit (all in the
      single chunk of sign +, exponent 0);
    * positions n/2 + i with i = 999 (mod 1000): N(0,1) * 2^-60;
    * the remaining second-half positions, in order, hold pairs (x, -x) with
      x = N(0,1) * 2^40;
    * 1% of n (rounded down to an even count) are near DBL_MAX:
      RNG-chosen whole pairs become (y, -y) with
      y = bits 0x7FE<<52 | (2^52 - 1 - u), u uniform in [0, 2^42);
      with ``overflow=True`` both members are +y, so the exact sum overflows.
    """
    assert n % 2 == 0 and n >= 2000
    rng = _rng(seed)
    half = n // 2
    out = np.empty(n, dtype=np.float64)
    f = rng.integers(0, 1 << 52, size=half, dtype=np.uint64)
    out[:half] = ((np.uint64(0x3FF) << np.uint64(52)) | f).view(np.float64)

    i = np.arange(half)
    tiny_mask = (i % 1000) == 999
    ntiny = int(tiny_mask.sum())
    rest = half - ntiny
    npairs = rest // 2                     # an odd leftover slot (small n only) holds +0.0
    t = np.ldexp(rng.standard_normal(ntiny), -60)
    x = np.ldexp(rng.standard_normal(npairs), 40)
    pairs = np.zeros(rest, dtype=np.float64)
    pairs[0:2 * npairs:2] = x
    pairs[1:2 * npairs:2] = -x

    nbig = (n // 100) & ~1
    nbig_pairs = nbig // 2
    which = rng.choice(npairs, size=nbig_pairs, replace=False)
    u = rng.integers(0, 1 << 42, size=nbig_pairs, dtype=np.uint64)
    y = ((np.uint64(0x7FE) << np.uint64(52)) | (MANT_MASK - u)).view(np.float64)
    pairs[2 * which] = y
    pairs[2 * which + 1] = y if overflow else -y

    second = np.empty(half, dtype=np.float64)
    second[tiny_mask] = t
    second[~tiny_mask] = pairs
    out[half:] = second
    return out


def segment_lengths(nseg: int = 65536, seed: int = 0, median: float = 1000.0,
                    sigma: float = 2.0, lo: int = 1, hi: int = 10 ** 6) -> np.ndarray:
    """Lengths clip(rint(exp(N(ln median, sigma))), lo, hi) as int64."""
    rng = _rng(seed)
    L = np.rint(np.exp(rng.normal(np.log(median), sigma, size=nseg)))
    return np.clip(L, lo, hi).astype(np.int64)


def segments(nseg: int = 65536, seed: int = 0, sigma: float = 2.0, median: float = 1000.0,
             hi: int = 10 ** 6, kmin: int = -30, kmax: int = 30):
    """Returns (x, offsets): offsets int64[nseg+1] is the exclusive prefix of
    the lengths; values are s * |N(0,1)| * 2^k, k uniform in [kmin, kmax]."""
    L = segment_lengths(nseg, seed, median=median, sigma=sigma, hi=hi)
    offsets = np.zeros(nseg + 1, dtype=np.int64)
    np.cumsum(L, out=offsets[1:])
    n = int(offsets[-1])
    x = small_normal(n, seed=seed + 1000003, kmin=kmin, kmax=kmax)
    return x, offsets


def serve_trace(nreq: int = 20000, seed: int = 1, pool_n: int = 10 ** 8,
                lmin: float = 10.0, lmax: float = 1e8):
    """Request lengths rint(10^U(log10 lmin, log10 lmax)) (clipped to the
    pool), start offsets uniform in [0, pool_n - L], and unit-rate
    exponential inter-arrival gaps (scale by 1/lambda to get seconds)."""
    rng = _rng(seed)
    L = np.rint(10.0 ** rng.uniform(np.log10(lmin), np.log10(lmax), size=nreq)).astype(np.int64)
    L = np.clip(L, 1, pool_n)
    starts = np.floor(rng.uniform(0.0, 1.0, size=nreq) * (pool_n - L + 1)).astype(np.int64)
    gaps = rng.exponential(1.0, size=nreq)
    return starts, L, gaps


def mirrored(n: int, seed: int = 0) -> np.ndarray:
    """First half U1 * exp(30 U2); element n-1-i is the negation of element i."""
    rng = _rng(seed)
    h = n // 2
    u1 = rng.uniform(0.0, 1.0, size=h)
    u2 = rng.uniform(0.0, 1.0, size=h)
    first = u1 * np.exp(30.0 * u2)
    out = np.zeros(n, dtype=np.float64)
    out[:h] = first
    out[n - h:] = -first[::-1]
    return out


def special_grid() -> np.ndarray:
    """Boundary binary64 values: zeros, denormal extremes, normal extremes,
    values around 1, powers of two near the top, DBL_MAX, infinities."""
    vals = [
        0.0, -0.0,
        5e-324, -5e-324,                                     # 2^-1074
        np.float64(2.2250738585072009e-308),                # largest denormal
        -np.float64(2.2250738585072009e-308),
        2.2250738585072014e-308, -2.2250738585072014e-308,  # smallest normal
        1.0, -1.0, np.nextafter(1.0, 2.0), np.nextafter(1.0, 0.0),
        2.0 ** 52, 2.0 ** 53, -(2.0 ** 53), 2.0 ** 970, 2.0 ** 1023, -(2.0 ** 1023),
        np.finfo(np.float64).max, -np.finfo(np.float64).max,
        0.1, -0.1, 3.0, 1e15, -1e15,
    ]
    return np.array(vals, dtype=np.float64)


def random_bits(n: int, seed: int, finite_only: bool = True) -> np.ndarray:
    """Uniformly random 64-bit patterns (optionally with infinities/NaNs
    replaced by their finite neighbours)."""
    rng = _rng(seed)
    b = rng.integers(0, np.iinfo(np.uint64).max, size=n, dtype=np.uint64, endpoint=True)
    if finite_only:
        e = (b >> np.uint64(52)) & np.uint64(2047)
        b = np.where(e == 2047, b ^ np.uint64(1 << 52), b)
    return b.view(np.float64)
