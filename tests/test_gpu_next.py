"""GPU parity of the further reductions over the same path: squared norm and
dot product (products rounded to binary64, then summed exactly), the exact
mean, binary32 sums, and the streaming accumulator -- bit for bit against
the oracle, on the small-only and the large path."""
import math

import numpy as np
import pytest

import oracle
from paper_1505_05571_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NAN_A = np.array([0x7FF0000000000001], dtype=np.uint64).view(np.float64)[0]


@pytest.fixture(scope="module")
def ex():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1505_05571_amd as ex
    ex.load_library()
    base = ex.exsum_get_config()
    yield ex
    ex.exsum_set_config(base)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def u64(t):
    torch.cuda.synchronize()
    return int(t.cpu().numpy().view(np.uint64)[0])


def u32(t):
    torch.cuda.synchronize()
    return int(t.cpu().numpy().view(np.uint32)[0])


def paths(ex):
    """Run the body on the default path choice, small-only and large-only."""
    base = ex.exsum_get_config()
    for small_max in (None, 10 ** 12, 0):
        c = ex.exsum_get_config()
        for k, _ in c._fields_:
            setattr(c, k, getattr(base, k))
        if small_max is not None:
            c.small_max = small_max
        ex.exsum_set_config(c)
        yield small_max
    ex.exsum_set_config(base)


SIZES = [0, 1, 2, 3, 63, 1000, 4096, 4097, 100003, 1000003]


def operands(n, seed):
    x = W.uniform_exponent(n, seed=seed, kmin=-250, kmax=250)
    y = W.uniform_exponent(n, seed=seed + 1, kmin=-250, kmax=250)
    return x, y


def test_sqnorm_and_dot(ex):
    for n in SIZES:
        x, y = operands(n, n)
        want_sq, want_dot = int(oracle.sqnorm_f64(x)), int(oracle.dot_f64(x, y))
        xt, yt = dev(x), dev(y)
        for p in paths(ex):
            assert u64(ex.exsum_sqnorm_f64(xt)) == want_sq, (n, p)
            assert u64(ex.exsum_dot_f64(xt, yt)) == want_dot, (n, p)


def test_dot_with_operands_of_different_alignment(ex):
    x, y = operands(300007, 11)
    xt, yt = dev(x), dev(y)
    for (a, b, L) in [(0, 1, 300000), (1, 0, 300000), (1, 1, 300001), (3, 6, 250000), (1, 2, 5)]:
        want = int(oracle.dot_f64(x[a:a + L], y[b:b + L]))
        for p in paths(ex):
            assert u64(ex.exsum_dot_f64(xt[a:a + L], yt[b:b + L])) == want, (a, b, L, p)


def test_products_that_underflow_overflow_or_are_special(ex):
    rng = np.random.default_rng(12)
    n = 20000
    x = np.ldexp(rng.standard_normal(n), rng.integers(-560, 560, size=n))
    y = np.ldexp(rng.standard_normal(n), rng.integers(-560, 560, size=n))
    with np.errstate(over="ignore"):
        keep = np.isfinite(x * y)                                   # drop products that overflow
    x, y = x[keep], y[keep]
    want = int(oracle.dot_f64(x, y))
    for p in paths(ex):
        assert u64(ex.exsum_dot_f64(dev(x), dev(y))) == want, p
    base = W.uniform_exponent(5000, seed=13, kmin=-10, kmax=10)
    for xs, ys in (([math.inf], [0.0]), ([math.inf], [2.0]), ([NAN_A], [3.0]), ([1e200], [1e200]),
                   ([1e200, -1e200], [1e200, 1e200]), ([-math.inf, 4.0], [1.0, math.inf])):
        x = base.copy()
        y = base.copy()
        x[[10, 4000][:len(xs)]] = xs
        y[[10, 4000][:len(ys)]] = ys
        want = int(oracle.dot_f64(x, y))
        for p in paths(ex):
            assert u64(ex.exsum_dot_f64(dev(x), dev(y))) == want, (xs, ys, p)


def test_mean(ex):
    for n in SIZES:
        x = W.uniform_exponent(n, seed=n + 5)
        want = int(oracle.mean_f64(x))
        xt = dev(x)
        for p in paths(ex):
            assert u64(ex.exsum_mean_f64(xt)) == want, (n, p)
    dmax = np.finfo(np.float64).max
    cases = [
        [1e15, -1e15, 0.1],                      # the worked example: the mean is fl(0.1/3)
        [dmax, dmax, dmax],                      # the sum overflows, the mean does not
        [5e-324, 0.0, 0.0],                      # 2^-1074 / 3 rounds to zero: +0
        [5e-324, 5e-324, 0.0],                   # 2^-1075 * 4/3 rounds to 2^-1074
        [-3.0, 1.0],
        [1.0] * 7 + [2.0 ** -60],
        [5e-324, 0.0],                           # 2^-1075: a tie between 0 and 2^-1074 -> +0
        [3 * 5e-324, 0.0],                       # 1.5 units: a tie -> 2 units (even)
        [1.0 + 2.0 ** -52, 2.0 ** -53, 0.0, 0.0],            # quotient needs its low bits (sticky)
        [2.0 ** 1000, 2.0 ** 1000 * (1 + 2.0 ** -52), 2.0 ** -1000],   # long quotient, tiny remainder
        list(np.ldexp(np.arange(1, 12, dtype=np.float64), 900)) + [-(2.0 ** -1070)],
    ]
    for vals in cases:
        x = np.array(vals, dtype=np.float64)
        want = int(oracle.mean_f64(x))
        for p in paths(ex):
            assert u64(ex.exsum_mean_f64(dev(x))) == want, (vals, p)
    assert int(oracle.mean_f64(np.array(cases[0]))) == int(np.array([0.1 / 3]).view(np.uint64)[0])


def f32_bits(n, seed):
    rng = np.random.default_rng(seed)
    b = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    e = (b >> np.uint32(23)) & np.uint32(255)
    b = np.where(e == 255, b ^ np.uint32(1 << 23), b)         # finite only
    return b.view(np.float32)


def test_f32(ex):
    for n in SIZES:
        for x in (f32_bits(n, n), (W.small_normal(n, seed=n)).astype(np.float32)):
            want = int(oracle.sum_f32(x))
            xt = dev(x)
            for p in paths(ex):
                assert u32(ex.exsum_f32(xt)) == want, (n, p)
    fmax = np.finfo(np.float32).max
    tiny = np.float32(1e-45)
    nan_a = np.array([0x7F800001], dtype=np.uint32).view(np.float32)[0]
    nan_b = np.array([0xFFC01234], dtype=np.uint32).view(np.float32)[0]
    cases = [
        [fmax, fmax, -fmax],                     # overflowing partial sums, finite result
        [fmax, fmax],                            # overflow to +Inf
        [tiny] * 5,                              # denormal sums
        [np.float32(1.0), tiny],                 # rounds back to 1
        [np.float32(np.inf), np.float32(-np.inf)],
        [nan_a, nan_b, np.float32(2.0)],
        [np.float32(-0.0), np.float32(-0.0)],    # exact zero: +0
    ]
    for vals in cases:
        x = np.array(vals, dtype=np.float32)
        big = np.zeros(50001, dtype=np.float32)
        big[::50001 // x.size][:x.size] = x
        want = int(oracle.sum_f32(x))
        assert int(oracle.sum_f32(big)) == want
        for p in paths(ex):
            assert u32(ex.exsum_f32(dev(x))) == want, (vals, p)
            assert u32(ex.exsum_f32(dev(big))) == want, (vals, p)
    x = f32_bits(300003, 7)
    xt = dev(x)
    for lo, hi in [(1, 300003), (2, 299999), (3, 300000), (1, 4)]:
        assert u32(ex.exsum_f32(xt[lo:hi])) == int(oracle.sum_f32(x[lo:hi])), (lo, hi)


def with_config(ex, **kw):
    c = ex.exsum_get_config()
    for k, v in kw.items():
        setattr(c, k, v)
    ex.exsum_set_config(c)


def test_f32_large_accumulator(ex):
    """The binary32 large path's own cases: whole tiles in one chunk, chunk
    totals past 2^48, subnormals (added at the weight of exponent field 1),
    zeros of both signs among normal terms (the fast path's unread chunks),
    grids with empty or tiny ranges; the pre-combine setting must not
    matter."""
    rng = np.random.default_rng(41)
    one_chunk = (1.0 + rng.random(2_000_003)).astype(np.float32)            # all in [1, 2)
    heavy = np.full((1 << 25) + 7, np.array([0x3FFFFFFF], dtype=np.uint32).view(np.float32)[0])
    sub_b = rng.integers(0, 1 << 24, size=1_000_003, dtype=np.uint64).astype(np.uint32)
    sub_b |= (rng.integers(0, 2, size=sub_b.size, dtype=np.uint64).astype(np.uint32) << np.uint32(31))
    subnormal_and_e1 = sub_b.view(np.float32)                               # exponent field 0 or 1
    mixed = f32_bits(100003, 43)
    few = f32_bits(5, 44)                                                   # most ranges empty at grid 1000
    with_zeros = rng.standard_normal(1_000_003).astype(np.float32)
    with_zeros[rng.random(with_zeros.size) < 0.5] = 0.0
    with_zeros[rng.random(with_zeros.size) < 0.1] = -0.0
    base = ex.exsum_get_config()
    try:
        for x in (one_chunk, heavy, subnormal_and_e1, mixed, with_zeros, few):
            want = int(oracle.sum_f32(x))
            xt = dev(x)
            for pre in (base.precombine, 0):
                for grid in (0, 1, 3, 1000):
                    with_config(ex, small_max=0, precombine=pre, large_grid=grid)
                    assert u32(ex.exsum_f32(xt)) == want, (x.size, pre, grid)
            ex.exsum_set_config(base)
    finally:
        ex.exsum_set_config(base)


def test_dot_f32_large_accumulator(ex):
    """The binary32 dot product's large path: products split into two 24-bit
    halves 24 exponents apart.  Cases: every product in one chunk, products
    of the largest significands many times over, subnormal operands, zeros of
    both signs, operands at the exponent extremes, y misaligned against x,
    grids with empty or tiny ranges."""
    rng = np.random.default_rng(45)
    n = 1_000_003
    one = ((1.0 + rng.random(n)).astype(np.float32), (1.0 + rng.random(n)).astype(np.float32))
    big_m = np.array([0x3FFFFFFF], dtype=np.uint32).view(np.float32)[0]
    heavy = (np.full((1 << 25) + 5, big_m), np.full((1 << 25) + 5, -big_m))
    sub = rng.integers(1, 1 << 23, size=n, dtype=np.uint64).astype(np.uint32).view(np.float32)
    subnormal = (sub, f32_bits(n, 46))
    zx = rng.standard_normal(n).astype(np.float32)
    zx[rng.random(n) < 0.4] = 0.0
    zx[rng.random(n) < 0.1] = -0.0
    zeros = (zx, rng.standard_normal(n).astype(np.float32))
    ext_e = rng.choice(np.array([1, 2, 253, 254], dtype=np.uint32), size=(2, n))
    ext_b = (ext_e << np.uint32(23)) | rng.integers(0, 1 << 23, size=(2, n), dtype=np.uint64).astype(np.uint32)
    ext_b |= rng.integers(0, 2, size=(2, n), dtype=np.uint64).astype(np.uint32) << np.uint32(31)
    extremes = (ext_b[0].view(np.float32), ext_b[1].view(np.float32))
    base = ex.exsum_get_config()
    try:
        for x, y in (one, heavy, subnormal, zeros, extremes, (f32_bits(7, 47), f32_bits(7, 48))):
            want = int(oracle.dot_f32(x, y))
            xt, yt = dev(x), dev(y)
            for grid in (0, 1, 3, 1000):
                with_config(ex, small_max=0, large_grid=grid)
                assert u32(ex.exsum_dot_f32(xt, yt)) == want, (x.size, grid)
            with_config(ex, small_max=0, large_grid=0)
            yb = dev(np.concatenate([[np.float32(0)], y]))
            assert u32(ex.exsum_dot_f32(xt, yb[1:])) == want, "y misaligned"
            ex.exsum_set_config(base)
    finally:
        ex.exsum_set_config(base)


def test_accumulator_add_merge_round(ex):
    parts = [W.uniform_exponent(n, seed=20 + n) for n in (0, 1, 1000, 4097, 300001)]
    parts.append(W.adversarial(4000, seed=21))
    whole = np.concatenate(parts)
    want = int(oracle.sum_f64(whole))
    for p in paths(ex):
        a = ex.Accumulator()
        b = ex.Accumulator()
        running = []
        for i, part in enumerate(parts):
            (a if i % 2 == 0 else b).add(dev(part))
            running.append(u64(a.round()))
        assert running[-1] == int(oracle.sum_f64(np.concatenate(parts[0::2]))), p
        a.merge(b)
        assert u64(a.round()) == want, p
        assert u64(a.round()) == want                  # rounding leaves the state as it was
        a.zero()
        assert u64(a.round()) == 0


def test_accumulator_many_updates_and_specials(ex):
    dmax = np.finfo(np.float64).max
    a = ex.Accumulator()
    chunk = np.array([dmax, -dmax / 2, 2.0 ** -1074], dtype=np.float64)
    ct = dev(chunk)
    for _ in range(300):
        a.add(ct)
    want = int(oracle.sum_f64(np.tile(chunk, 300)))
    assert u64(a.round()) == want                      # +Inf: the exact sum overflows
    b = ex.Accumulator().add(dev(np.array([-dmax / 2] * 300, dtype=np.float64)))
    a.merge(b)
    want = int(oracle.sum_f64(np.concatenate([np.tile(chunk, 300), [-dmax / 2] * 300])))
    assert u64(a.round()) == want                      # back to 300 * 2^-1074
    c = ex.Accumulator().add(dev(np.array([1.0, NAN_A])))
    a.merge(c)
    assert u64(a.round()) == int(oracle.sum_f64(np.array([NAN_A])))


def test_dot_f32(ex):
    # random bit patterns (denormals included) and normal-only values, every path
    for n in SIZES:
        for x, y in ((f32_bits(n, n + 11), f32_bits(n, n + 12)),
                     (W.small_normal(n, seed=n).astype(np.float32), W.small_normal(n, seed=n + 1).astype(np.float32))):
            want = int(oracle.dot_f32(x, y))
            xt, yt = dev(x), dev(y)
            for p in paths(ex):
                assert u32(ex.exsum_dot_f32(xt, yt)) == want, (n, p)
    # y at another alignment than x (four 4-byte loads per position)
    x, y = f32_bits(300005, 21), f32_bits(300005, 22)
    xt, yt = dev(x), dev(y)
    for lo, hi, d in [(0, 300000, 1), (1, 300001, 2), (3, 299999, 1), (2, 5, 3)]:
        want = int(oracle.dot_f32(x[lo:hi], y[lo + d:hi + d]))
        for p in paths(ex):
            assert u32(ex.exsum_dot_f32(xt[lo:hi], yt[lo + d:hi + d])) == want, (lo, hi, d, p)
    # closed forms from the oracle's pins, alone and buried in zeros
    t, u = np.float32(2.0 ** -75), np.float32(2.0 ** -100)
    fmax = np.finfo(np.float32).max
    inf = np.float32(np.inf)
    q = np.array([0x7FC01234], dtype=np.uint32).view(np.float32)[0]
    cases = [
        ([t, t, t], [t, t, t], 2),                                  # 3 * 2^-150 -> 2 units
        ([t], [t], 0),                                              # half a unit, ties to even -> +0
        ([t, u], [t, u], 1),                                        # just above half a unit
        ([3.0, -3.0, u], [5.0, 5.0, u], 0),                         # 2^-200 -> +0
        ([-t], [t], 0),                                             # -(half a unit) -> +0, not -0
        ([-3.0, 3.0, -u], [5.0, 5.0, u], 0),                        # -2^-200 -> +0, not -0
        ([-t, -u], [t, u], 0x80000001),                             # just below minus half a unit
        ([1.0, 2.0 ** -12, u], [1.0, 2.0 ** -12, u], 0x3F800001),   # just above a tie
        ([fmax, fmax], [2.0, -1.0], int(np.array([fmax]).view(np.uint32)[0])),
        ([fmax], [2.0], 0x7F800000),
        ([inf, 1.0], [1.0, 2.0], 0x7F800000),
        ([inf, inf], [1.0, -1.0], 0x7FC00000),
        ([q, 1.0], [2.0, 3.0], 0x7FC01234),
    ]
    for xs, ys, want in cases:
        x = np.array(xs, dtype=np.float32)
        y = np.array(ys, dtype=np.float32)
        assert int(oracle.dot_f32(x, y)) == want
        bx = np.zeros(50003, dtype=np.float32)
        by = np.zeros(50003, dtype=np.float32)
        pos = np.arange(x.size) * (50003 // x.size)
        bx[pos], by[pos] = x, y
        assert int(oracle.dot_f32(bx, by)) == want
        for p in paths(ex):
            assert u32(ex.exsum_dot_f32(dev(x), dev(y))) == want, (xs, p)
            assert u32(ex.exsum_dot_f32(dev(bx), dev(by))) == want, (xs, p)
