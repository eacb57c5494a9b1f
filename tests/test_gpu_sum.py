"""GPU parity: the HIP library (through the C ABI) against the CPU oracle, bit
for bit (0 ulp), on seeded inputs of the benchmark's shapes plus edge cases.
Every launch configuration must give the same bits."""
import math

import numpy as np
import pytest

import oracle
from chain_cases import long_chain_cases
from paper_1505_05571_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ex():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1505_05571_amd as ex
    ex.load_library()
    return ex


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def gbits(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def run(ex, x, cfg=None):
    xt = dev(x) if isinstance(x, np.ndarray) else x
    out = ex.exsum_f64(xt) if cfg is None else ex.exsum_f64_cfg(xt, cfg)
    return int(gbits(out)[0])


def cfg_with(ex, **kw):
    c = ex.exsum_get_config()
    for k, v in kw.items():
        setattr(c, k, v)
    return c


# pre-combine thresholds cycled over the built variants, so that every
# variant runs with and without the pre-combine across the test grid
PRECOMBINES = (16, 0, 32, 1, 8)


def large_variants(ex):
    """Every large-kernel shape the library is built with (the library's own
    list, which the CPU tests check against the header and the configuration
    checks), each with a pre-combine threshold."""
    out = []
    for k, (b, v, d, m) in enumerate(ex.exsum_large_variants()):
        out.append(dict(large_block=b, large_vec=v, large_depth=d, large_mode=m,
                        precombine=PRECOMBINES[k % len(PRECOMBINES)]))
    return out


def all_paths(ex):
    """Small-only path and several large-path configurations (and grids)."""
    cfgs = [cfg_with(ex, small_max=10 ** 12)]
    for v in large_variants(ex):
        for grid in (0, 1, 7, 300):
            cfgs.append(cfg_with(ex, small_max=0, large_grid=grid, **v))
    return cfgs


def test_small_normal_1000(ex):
    x = W.small_normal(1000, seed=0)
    want = int(oracle.sum_f64(x))
    assert run(ex, x) == want
    for c in all_paths(ex):
        assert run(ex, x, c) == want


@pytest.mark.parametrize("n", [0, 1, 2, 3, 31, 64, 65, 127, 1000, 2047, 2048, 2049, 4095, 4096, 4097,
                               10000, 65537, 262147, 1000003])
def test_sizes_and_paths(ex, n):
    for gen in (lambda m: W.uniform_exponent(m, seed=n), lambda m: W.small_normal(m, seed=n + 1)):
        x = gen(n)
        want = int(oracle.sum_f64(x))
        assert run(ex, x) == want, n
        if n <= 70000:
            for c in all_paths(ex):
                assert run(ex, x, c) == want, (n, c.as_dict())


def test_misaligned_slices(ex):
    x = W.uniform_exponent(300001, seed=9)
    xt = dev(x)
    for lo, hi in [(1, 300001), (3, 299998), (1, 2), (5, 6), (7, 100000), (0, 299999)]:
        want = int(oracle.sum_f64(x[lo:hi]))
        assert run(ex, xt[lo:hi]) == want
        for c in all_paths(ex)[:6]:
            assert run(ex, xt[lo:hi], c) == want


def test_random_bit_patterns(ex):
    for seed in range(6):
        x = W.random_bits(200000 + seed, seed=seed)
        want = int(oracle.sum_f64(x))
        for c in all_paths(ex)[:8]:
            assert run(ex, x, c) == want


def test_hot_chunk_many_tiles(ex):
    # every term in one (sign, exponent) chunk: counts cross the transfer
    # threshold over and over; pre-combine on and off must agree
    rng = np.random.default_rng(3)
    f = rng.integers(0, 1 << 52, size=1 << 20, dtype=np.uint64)
    x = ((np.uint64(0x3FF) << np.uint64(52)) | f).view(np.float64)
    want = int(oracle.sum_f64(x))
    for c in all_paths(ex):
        assert run(ex, x, c) == want
    xneg = -x
    assert run(ex, xneg) == int(oracle.sum_f64(xneg))


def test_adversarial_small_scale(ex):
    for ovf in (False, True):
        x = W.adversarial(1 << 18, seed=4, overflow=ovf)
        want = int(oracle.sum_f64(x))
        if ovf:
            assert want == 0x7FF0000000000000
        for c in all_paths(ex)[:10]:
            assert run(ex, x, c) == want


def test_mirrored_is_zero(ex):
    for n in (10, 1001, 100000, 1000001):
        x = W.mirrored(n, seed=n)
        assert run(ex, x) == 0
        assert run(ex, np.random.default_rng(n).permutation(x)) == 0


def test_worked_example_and_closed_forms(ex):
    dmax = np.finfo(np.float64).max
    cases = [
        ([1e15, -1e15, 0.1], 0x3FB999999999999A),
        ([dmax, 2.0 ** 970], 0x7FF0000000000000),
        ([dmax, 2.0 ** 970, -5e-324], int(np.array([dmax]).view(np.uint64)[0])),
        ([2.0 ** 1023, 2.0 ** 1023, -(2.0 ** 1023)], int(np.array([2.0 ** 1023]).view(np.uint64)[0])),
        ([-0.0, -0.0], 0),
        ([], 0),
        ([5e-324] * 3, 3),
    ]
    for vals, want in cases:
        x = np.array(vals, dtype=np.float64)
        assert int(oracle.sum_f64(x)) == want
        for c in all_paths(ex)[:6]:
            assert run(ex, x, c) == want, vals
    # the same closed forms buried in a long array of cancelling pairs
    rng = np.random.default_rng(5)
    pairs = np.ldexp(rng.standard_normal(200000), rng.integers(-900, 900, size=200000))
    for vals, want in cases[:4]:
        x = np.concatenate([pairs, -pairs, np.array(vals)])
        rng.shuffle(x)
        assert int(oracle.sum_f64(x)) == want
        for c in all_paths(ex)[:6]:
            assert run(ex, x, c) == want


def test_special_values_anywhere(ex):
    rng = np.random.default_rng(6)
    base = W.uniform_exponent(100000, seed=6)
    nan_a = np.array([0x7FF0000000000001], dtype=np.uint64).view(np.float64)[0]
    nan_b = np.array([0xFFF80000000ABCDE], dtype=np.uint64).view(np.float64)[0]
    for specials in ([math.inf], [-math.inf], [math.inf, -math.inf], [nan_a], [nan_a, nan_b, math.inf]):
        x = base.copy()
        pos = rng.choice(x.size, size=len(specials), replace=False)
        x[pos] = specials
        want = int(oracle.sum_f64(x))
        for c in all_paths(ex)[:8]:
            assert run(ex, x, c) == want, specials


def test_denormals_and_extremes(ex):
    rng = np.random.default_rng(7)
    b = rng.integers(0, 1 << 53, size=300000, dtype=np.uint64)
    s = rng.integers(0, 2, size=300000, dtype=np.uint64) << np.uint64(63)
    x = (b | s).view(np.float64)
    want = int(oracle.sum_f64(x))
    for c in all_paths(ex)[:8]:
        assert run(ex, x, c) == want
    top = ((np.uint64(0x7FE) << np.uint64(52)) | rng.integers(0, 1 << 52, size=100000, dtype=np.uint64)).view(np.float64)
    top = np.concatenate([top, -top[:99990]])
    want = int(oracle.sum_f64(top))
    for c in all_paths(ex)[:8]:
        assert run(ex, top, c) == want


def test_long_carry_chains(ex):
    for x in long_chain_cases():
        want = int(oracle.sum_f64(x))
        for c in all_paths(ex)[:9]:
            assert run(ex, x, c) == want, (x, c.as_dict())
        # the same value spread over a long input (the large path proper)
        big = np.zeros(200003, dtype=np.float64)
        big[::200003 // x.size][:x.size] = x
        assert int(oracle.sum_f64(big)) == want
        for c in all_paths(ex)[:9]:
            assert run(ex, big, c) == want, (x, c.as_dict())


def test_permutation_invariance(ex):
    x = W.uniform_exponent(500000, seed=8)
    want = int(oracle.sum_f64(x))
    rng = np.random.default_rng(8)
    for _ in range(3):
        assert run(ex, rng.permutation(x)) == want


def test_repeated_calls_leave_workspace_clean(ex):
    xs = [W.uniform_exponent(n, seed=n) for n in (5000, 700000, 3, 123456)]
    wants = [int(oracle.sum_f64(x)) for x in xs]
    for _ in range(3):
        for x, w in zip(xs, wants):
            assert run(ex, x) == w


def test_inexact_comparator_is_close(ex):
    # any order of n-1 binary64 additions errs by at most (n-1) 2^-53 sum|x|
    # (first order); one or two terms are exact or one rounding
    x = W.small_normal(1000003, seed=3)
    xt = dev(x)
    for lo, hi in [(0, 1), (0, 2), (5, 8), (0, 1000003), (1, 1000003), (3, 999001), (0, 300001)]:
        part = x[lo:hi]
        got = float(ex.exsum_inexact_f64(xt[lo:hi]).cpu()[0])
        if part.size <= 2:
            assert got == float(np.float64(part[0]) + (np.float64(part[1]) if part.size == 2 else 0.0))
            continue
        exact = oracle.bits_to_f64(oracle.sum_f64(part))
        assert abs(got - exact) <= (part.size - 1) * 2.0 ** -53 * np.abs(part).sum() * 1.01, (lo, hi)
    assert float(ex.exsum_inexact_f64(xt[:0]).cpu()[0]) == 0.0


def test_bad_arguments(ex):
    import ctypes
    lib = ex.load_library()
    assert lib.exsum_f64(None, 5, None, None) == 1
    assert lib.exsum_f64(None, -1, None, None) == 1
    assert lib.exsum_segmented_f64(None, None, -1, None, None) == 1


@pytest.mark.parametrize("which", ["uniform_exponent_1e8"])
def test_full_size_uniform_exponent(ex, which):
    # the benchmark workload at full size, in its default launch configuration
    x = W.uniform_exponent(10 ** 8, seed=0)
    want = int(oracle.sum_f64_mt(x, 8))
    xt = dev(x)
    assert run(ex, xt) == want
    assert run(ex, xt) == want


def test_full_size_adversarial(ex):
    for ovf in (False, True):
        x = W.adversarial(1 << 27, seed=0, overflow=ovf)
        want = int(oracle.sum_f64_mt(x, 8))
        assert run(ex, dev(x)) == want


def test_beyond_32_bit_indices(ex):
    # 2^31 + 1000 terms (17 GB on the device, made there): every index and
    # offset path crosses 2^31.  Closed forms: a sum of ones is its count; a
    # few planted values change it by exactly their sum.
    n = (1 << 31) + 1000
    try:
        x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    except RuntimeError:
        pytest.skip("not enough device memory")
    assert run(ex, x) == int(np.array([float(n)]).view(np.uint64)[0])
    x[(1 << 31) + 3] = 2.0 ** 60
    x[5] = -(2.0 ** 60)
    x[n - 1] = 0.5
    want = float(n - 3) + 0.5                       # ones at 3 places replaced
    assert run(ex, x) == int(np.array([want]).view(np.uint64)[0])
    # segments across the boundary
    off = np.array([0, (1 << 31) - 5, (1 << 31) + 7, n - 1, n], dtype=np.int64)
    got = ex.exsum_segmented_f64(x, torch.from_numpy(off).to("cuda:0"))
    torch.cuda.synchronize()
    # segment 0 holds -2^60 and 2^31-6 ones, segment 1 holds 2^60 and 11
    # ones (each a single correctly rounded binary64 addition of exact
    # operands), segment 2 only ones, segment 3 the half
    seg = [-(2.0 ** 60) + float((1 << 31) - 6), 2.0 ** 60 + 11.0, float(n - 1 - ((1 << 31) + 7)), 0.5]
    want_bits = np.array(seg, dtype=np.float64).view(np.uint64)
    assert np.array_equal(got.cpu().numpy().view(np.uint64), want_bits)
    del x
    torch.cuda.empty_cache()
