"""Pins for the CPU oracle, against things other than the oracle itself.

* exact rational arithmetic (``fractions.Fraction``; CPython converts a
  Fraction to float with one correct rounding, raising OverflowError when
  the rounded value is not finite);
* ``math.fsum`` (a floating-point-expansion method, correctly rounded,
  numerically independent of any superaccumulator);
* IEEE hardware addition for two terms (the Discussion notes that sums of
  two terms are correctly rounded by ordinary addition) and identity for one;
* the worked example of the Introduction (``tests/golden``);
* closed-form sums of constructed cancellation sets, the paper's own
  mirror-negated timing distribution (exact sum zero), and invariants
  (order, negation, power-of-two scaling) that follow from exactness.
"""
import itertools
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1505_05571_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DBL_MAX = np.finfo(np.float64).max


def bits(v) -> int:
    return int(np.array([v], dtype=np.float64).view(np.uint64)[0])


def from_bits(b) -> float:
    return float(np.array([b], dtype=np.uint64).view(np.float64)[0])


def exact_round(values) -> int:
    """Bits of the correctly rounded exact sum via Fraction (finite inputs)."""
    s = sum((Fraction(float(v)) for v in values), Fraction(0))
    if s == 0:
        return 0  # exact zero is +0.0
    try:
        return bits(float(s))
    except OverflowError:
        return bits(math.inf if s > 0 else -math.inf)


def mixed_values(rng: random.Random, n: int):
    grid = list(W.special_grid())
    grid = [g for g in grid if math.isfinite(g)]
    out = []
    for _ in range(n):
        r = rng.random()
        if r < 0.3:
            out.append(rng.choice(grid))
        elif r < 0.5:  # denormals
            out.append(from_bits(rng.getrandbits(52)) * rng.choice([1, -1]))
        elif r < 0.7:  # near the top of the range
            out.append(from_bits((rng.randrange(2000, 2047) << 52) | rng.getrandbits(52))
                       * rng.choice([1, -1]))
        else:
            out.append(math.ldexp(rng.uniform(-1, 1), rng.randint(-1074, 1023)))
    return out


# ---- golden worked example -------------------------------------------------

def load_golden(name):
    terms, expect = [], {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, val = line.split()
            if key == "term":
                terms.append(from_bits(int(val, 16)))
            else:
                expect[key] = int(val, 16)
    return terms, expect


def test_worked_example_all_orders():
    terms, expect = load_golden("worked_example.txt")
    for perm in itertools.permutations(terms):
        assert int(oracle.sum_f64(list(perm))) == expect["sum"]
    # ordinary left-to-right addition depends on the order
    assert (1e15 + 0.1) - 1e15 == 0.125
    # the exact mean is the exact sum divided by 3 with one rounding, which
    # here is the IEEE quotient of the binary64 0.1 by 3
    assert int(oracle.mean_f64(terms)) == bits(0.1 / 3)


# ---- one and two terms -----------------------------------------------------

def test_single_term_identity():
    vals = [v for v in W.special_grid() if math.isfinite(v) and v != 0]
    vals += list(W.random_bits(20000, seed=11))
    for v in vals:
        if v == 0:
            continue
        assert int(oracle.sum_f64([v])) == bits(v), v


def test_zero_results_are_positive_zero():
    assert int(oracle.sum_f64([])) == 0
    assert int(oracle.sum_f64([-0.0])) == 0
    assert int(oracle.sum_f64([-0.0, -0.0, 0.0])) == 0
    assert int(oracle.sum_f64([1.5, -1.5])) == 0


def test_two_terms_match_hardware_addition():
    rng = random.Random(5)
    vals = list(W.special_grid()) + [math.inf, -math.inf]
    pairs = list(itertools.product(vals, vals))
    vals2 = mixed_values(rng, 4000)
    pairs += [(vals2[i], vals2[i + 1]) for i in range(0, len(vals2), 2)]
    rb = W.random_bits(40000, seed=3)
    pairs += [(rb[i], rb[i + 1]) for i in range(0, len(rb), 2)]
    for a, b in pairs:
        a, b = float(a), float(b)
        got = int(oracle.sum_f64([a, b]))
        hw = a + b
        if math.isnan(hw):
            assert math.isnan(from_bits(got))
            continue
        if hw == 0:
            assert got == 0  # +0 convention (hardware gives -0 for -0 + -0)
            continue
        assert got == bits(hw), (a, b)


# ---- brute force against exact rationals -----------------------------------

def test_bruteforce_small_random_sets():
    rng = random.Random(1234)
    for trial in range(6000):
        n = rng.randint(1, 8)
        vals = mixed_values(rng, n)
        assert int(oracle.sum_f64(vals)) == exact_round(vals), vals


def test_bruteforce_exhaustive_tiny_grid():
    grid = [v for v in W.special_grid() if math.isfinite(v)]
    for combo in itertools.combinations_with_replacement(grid, 3):
        assert int(oracle.sum_f64(list(combo))) == exact_round(combo), combo


def test_bruteforce_random_bit_patterns():
    for seed in range(40):
        vals = W.random_bits(64, seed=100 + seed)
        assert int(oracle.sum_f64(vals)) == exact_round(vals)


def test_bruteforce_near_ties():
    # x + tiny where tiny sits exactly at / just around half an ulp of x
    rng = random.Random(99)
    for _ in range(3000):
        e = rng.randint(-1000, 1000)
        m = rng.getrandbits(52) | (1 << 52)
        x = math.ldexp(m, e - 52)
        half = math.ldexp(1.0, e - 53)
        for tiny in (half, -half, half * (1 + 2 ** -40), half * (1 - 2 ** -40),
                     math.ldexp(1.0, e - 120)):
            if tiny == 0:
                continue
            vals = [x, tiny, math.ldexp(1.0, e - 200) * rng.choice([1, -1])]
            assert int(oracle.sum_f64(vals)) == exact_round(vals)


# ---- independent library: math.fsum ----------------------------------------

@pytest.mark.parametrize("seed", range(8))
def test_matches_fsum(seed):
    rng = np.random.default_rng(seed)
    n = 5000
    x = np.ldexp(rng.standard_normal(n), rng.integers(-400, 400, size=n))
    assert int(oracle.sum_f64(x)) == bits(math.fsum(x))
    y = W.small_normal(3001, seed=seed)
    assert int(oracle.sum_f64(y)) == bits(math.fsum(y))
    z = W.uniform_exponent(7777, seed=seed)
    assert int(oracle.sum_f64(z)) == bits(math.fsum(z))


def test_matches_fsum_denormal_heavy():
    rng = np.random.default_rng(77)
    b = rng.integers(0, 1 << 53, size=20000, dtype=np.uint64)  # e in {0,1}
    s = rng.integers(0, 2, size=20000, dtype=np.uint64) << np.uint64(63)
    x = (b | s).view(np.float64)
    got = from_bits(int(oracle.sum_f64(x)))
    assert got == math.fsum(x)


# ---- closed forms -------------------------------------------------------------

def test_mirrored_distribution_sums_to_zero():
    # the Performance evaluations distribution: exact sum is exactly 0
    for n in (10, 100, 1001, 100000):
        x = W.mirrored(n, seed=n)
        assert int(oracle.sum_f64(x)) == 0
        assert int(oracle.sum_f64(np.random.default_rng(n).permutation(x))) == 0


def test_k_copies():
    rng = random.Random(8)
    for _ in range(300):
        x = math.ldexp(rng.uniform(1, 2), rng.randint(-1070, 1000)) * rng.choice([1, -1])
        k = rng.randint(1, 5000)
        expect = Fraction(x) * k
        try:
            e = bits(float(expect))
        except OverflowError:
            e = bits(math.copysign(math.inf, x))
        assert int(oracle.sum_f64([x] * k)) == e


def test_integer_sums_are_exact():
    rng = np.random.default_rng(4)
    v = rng.integers(-(1 << 40), 1 << 40, size=4096)
    assert from_bits(int(oracle.sum_f64(v.astype(np.float64)))) == float(int(v.sum()))


def test_cancellation_pairs_leave_tiny_terms():
    rng = np.random.default_rng(12)
    x = np.ldexp(rng.standard_normal(5000), 40)
    K = rng.integers(-1000, 1000, size=500)
    t = np.ldexp(K.astype(np.float64), -60)  # integer multiples of 2^-60
    arr = np.concatenate([x, -x, t])
    rng.shuffle(arr)
    assert from_bits(int(oracle.sum_f64(arr))) == math.ldexp(float(int(K.sum())), -60)


def test_overflow_closed_forms():
    # the exact sum is representable => finite, even when naive sums overflow
    assert from_bits(int(oracle.sum_f64([DBL_MAX, 2.0 ** 970]))) == math.inf
    assert from_bits(int(oracle.sum_f64([DBL_MAX, 2.0 ** 970, -5e-324]))) == DBL_MAX
    assert from_bits(int(oracle.sum_f64([-DBL_MAX, -(2.0 ** 970), 5e-324]))) == -DBL_MAX
    assert from_bits(int(oracle.sum_f64([2.0 ** 1023, 2.0 ** 1023, -(2.0 ** 1023)]))) == 2.0 ** 1023
    # sums well beyond the top of the range (exponent field would be 2047 or more)
    assert from_bits(int(oracle.sum_f64([DBL_MAX, 2.0 ** 1023]))) == math.inf
    assert from_bits(int(oracle.sum_f64([-DBL_MAX] * 3))) == -math.inf
    assert from_bits(int(oracle.sum_f64([DBL_MAX] * 5000))) == math.inf
    assert (2.0 ** 1023 + 2.0 ** 1023) - 2.0 ** 1023 == math.inf
    big = [DBL_MAX] * 1000 + [-DBL_MAX] * 999
    assert from_bits(int(oracle.sum_f64(big))) == DBL_MAX


def test_denormal_sums_crossing_into_normals():
    d = from_bits((1 << 52) - 1)  # largest denormal
    assert int(oracle.sum_f64([d, 5e-324])) == 1 << 52
    assert int(oracle.sum_f64([d, d])) == bits(d * 2)
    assert int(oracle.sum_f64([5e-324] * 3)) == 3


# ---- invariants -----------------------------------------------------------------

def test_permutation_negation_scaling():
    rng = np.random.default_rng(21)
    x = W.uniform_exponent(20000, seed=21)
    s = int(oracle.sum_f64(x))
    for _ in range(3):
        assert int(oracle.sum_f64(rng.permutation(x))) == s
    neg = int(oracle.sum_f64(-x))
    assert neg == (s ^ (1 << 63) if s != 0 else 0)
    for k in (-5, 7, 100):
        assert from_bits(int(oracle.sum_f64(np.ldexp(x, k)))) == math.ldexp(from_bits(s), k)


def test_multithreaded_split_matches():
    x = W.uniform_exponent(100003, seed=5)
    s = oracle.sum_f64(x)
    for t in (1, 2, 3, 8):
        assert oracle.sum_f64_mt(x, t) == s


def test_segmented_matches_per_segment():
    x, off = W.segments(nseg=200, seed=3, hi=20000)
    seg = oracle.segmented_f64(x, off)
    for i in range(200):
        assert seg[i] == oracle.sum_f64(x[off[i]:off[i + 1]])
    starts = off[:-1]
    lens = np.diff(off)
    assert np.array_equal(oracle.sum_ranges_f64(x, starts, lens), seg)


def test_ranges_by_prefix_match_direct_sums():
    """Prefix-difference range sums (the served trace's full check) against
    the direct definition: ranges inside one stride, across strides, aligned
    to stride boundaries, empty and the whole pool, at several strides and
    thread counts; and, on tiny pools, against exact rationals."""
    x = W.uniform_exponent(50021, seed=9)
    rng = np.random.default_rng(9)
    st, ln = [], []
    for L in [0, 1, 2, 63, 64, 65, 127, 128, 129, 1000, 4096, 4097, 30000, 50021]:
        for a in (0, 1, 63, 64, 128, 50021 - L):
            if 0 <= a <= 50021 - L:
                st.append(a)
                ln.append(L)
    for _ in range(300):
        L = int(rng.integers(0, 50022))
        st.append(int(rng.integers(0, 50022 - L)))
        ln.append(L)
    st, ln = np.array(st, dtype=np.int64), np.array(ln, dtype=np.int64)
    want = oracle.sum_ranges_f64(x, st, ln)
    for stride, threads in ((64, 1), (1, 3), (4096, 4), (1 << 16, 2), (7, 1)):
        assert np.array_equal(oracle.ranges_by_prefix_f64(x, st, ln, stride=stride, nthreads=threads), want)
    # long cancellation: a prefix difference of huge partial sums leaves the tiny terms
    y = np.array([1e300, 3e-300, -1e300, 5e-310, 2.0 ** 1000, -(2.0 ** 1000), 7.0, -7.0, 1e-320], dtype=np.float64)
    rst = np.array([0, 0, 1, 2, 3, 4, 1], dtype=np.int64)
    rln = np.array([9, 3, 8, 7, 6, 5, 2], dtype=np.int64)
    for stride in (1, 2, 3, 4):
        got = oracle.ranges_by_prefix_f64(y, rst, rln, stride=stride)
        for r in range(rst.size):
            assert int(got[r]) == exact_round(y[rst[r]:rst[r] + rln[r]]), (stride, r)
    with pytest.raises(ValueError):
        oracle.ranges_by_prefix_f64(np.array([1.0, math.inf]), [0], [1])
    with pytest.raises(ValueError):
        oracle.ranges_by_prefix_f64(x, [50000], [22])


# ---- specials (conventions; the paper fixes only that they are side fields) -----

def test_special_values():
    nan1 = from_bits(0x7FF0000000000001)
    nan2 = from_bits(0xFFF8000000000123)
    assert int(oracle.sum_f64([1.0, math.inf])) == bits(math.inf)
    assert int(oracle.sum_f64([1.0, -math.inf, DBL_MAX, DBL_MAX])) == bits(-math.inf)
    assert int(oracle.sum_f64([math.inf, -math.inf])) == 0x7FF8000000000000
    # max payload with sign cleared, quiet bit set
    assert int(oracle.sum_f64([nan1, 2.0, nan2, math.inf])) == 0x7FF8000000000123
    assert int(oracle.sum_f64([nan1])) == 0x7FF8000000000001


# ---- mean, dot product, squared norm, binary32 -----------------------------------

def test_mean_bruteforce():
    rng = random.Random(17)
    for _ in range(3000):
        n = rng.randint(1, 9)
        vals = mixed_values(rng, n)
        s = sum((Fraction(v) for v in vals), Fraction(0)) / n
        if s == 0:
            e = 0
        else:
            try:
                e = bits(float(s))
            except OverflowError:
                e = bits(math.copysign(math.inf, s))
            if e & 0x7FFFFFFFFFFFFFFF == 0:
                e = 0
        assert int(oracle.mean_f64(vals)) == e, vals


def test_dot_and_sqnorm_bruteforce():
    rng = np.random.default_rng(31)
    for _ in range(200):
        n = int(rng.integers(1, 40))
        x = np.ldexp(rng.standard_normal(n), rng.integers(-500, 500, size=n))
        y = np.ldexp(rng.standard_normal(n), rng.integers(-500, 500, size=n))
        prods = [float(a) * float(b) for a, b in zip(x, y)]
        assert int(oracle.dot_f64(x, y)) == exact_round(prods)
        sq = [float(a) * float(a) for a in x]
        assert int(oracle.sqnorm_f64(x)) == exact_round(sq)


def test_f32_two_terms_hardware():
    rng = np.random.default_rng(8)
    b = rng.integers(0, 1 << 32, size=20000, dtype=np.uint64).astype(np.uint32)
    e = (b >> np.uint32(23)) & np.uint32(255)
    b = np.where(e == 255, b ^ np.uint32(1 << 23), b)
    x = b.view(np.float32)
    with np.errstate(over="ignore"):
        for i in range(0, x.size, 2):
            a, c = x[i], x[i + 1]
            hw = np.float32(a + c)  # binary32 RNE addition
            got = int(oracle.sum_f32([a, c]))
            if hw == 0:
                assert got == 0
            else:
                assert got == int(np.array([hw], dtype=np.float32).view(np.uint32)[0]), (a, c)


def test_f32_exact_in_double_sums():
    rng = np.random.default_rng(9)
    checked = 0
    for _ in range(400):
        n = int(rng.integers(1, 30))
        x = (rng.standard_normal(n) * np.exp2(rng.integers(-10, 10, size=n))).astype(np.float32)
        s = sum((Fraction(float(v)) for v in x), Fraction(0))
        if Fraction(float(s)) != s:
            continue  # the double would round; numpy's cast then double-rounds
        checked += 1
        exp = np.float32(float(s))
        got = int(oracle.sum_f32(x))
        assert got == (0 if exp == 0 else int(np.array([exp]).view(np.uint32)[0]))
    assert checked > 300


# ---- binary32 dot product --------------------------------------------------

def f32_round_bits(fr: Fraction) -> int:
    """Bits of a rational rounded to binary32, ties to even, written out from
    the format's definition (a result of magnitude zero is +0)."""
    if fr == 0:
        return 0
    s = 0x80000000 if fr < 0 else 0
    a = abs(fr)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    if Fraction(2) ** (e + 1) <= a:
        e += 1
    ulp = Fraction(2) ** (max(e, -126) - 23)
    q = a / ulp
    k = q.numerator // q.denominator
    rem = q - k
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and k % 2 == 1):
        k += 1
    if k == 0:
        return 0
    val = k * ulp
    if val >= Fraction(2) ** 128:
        return s | 0x7F800000
    return s | int(np.array([np.float32(float(val))]).view(np.uint32)[0])


def f32_words(rng, n):
    """Random binary32 values over the whole finite range, denormals included."""
    b = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    e = (b >> np.uint32(23)) & np.uint32(255)
    b = np.where(e == 255, b ^ np.uint32(1 << 23), b)
    return b.view(np.float32)


def test_f32_round_helper_matches_hardware_casts():
    # the test's own rounding, checked against numpy's binary64 -> binary32
    # cast on values that are exact in binary64 (one rounding only)
    rng = np.random.default_rng(40)
    d = np.ldexp(rng.standard_normal(5000), rng.integers(-160, 130, size=5000))
    with np.errstate(over="ignore"):
        for v in d:
            hw = np.float32(v)
            want = 0 if hw == 0 else int(np.array([hw]).view(np.uint32)[0])
            if math.isinf(hw):
                want = int(np.array([hw]).view(np.uint32)[0])
            assert f32_round_bits(Fraction(float(v))) == want, v


def test_dot_f32_bruteforce():
    rng = np.random.default_rng(41)
    for _ in range(600):
        n = int(rng.integers(1, 12))
        if rng.random() < 0.5:
            x, y = f32_words(rng, n), f32_words(rng, n)
        else:
            x = (rng.standard_normal(n) * np.exp2(rng.integers(-80, 80, size=n))).astype(np.float32)
            y = (rng.standard_normal(n) * np.exp2(rng.integers(-80, 80, size=n))).astype(np.float32)
        exact = sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0))
        assert int(oracle.dot_f32(x, y)) == f32_round_bits(exact), (x, y)


def test_dot_f32_single_products_and_cancellation():
    rng = np.random.default_rng(42)
    x, y = f32_words(rng, 3000), f32_words(rng, 3000)
    with np.errstate(over="ignore", under="ignore"):
        for a, b in zip(x, y):
            p = np.float32(np.float64(a) * np.float64(b))      # the exact product, rounded once
            want = int(np.array([p]).view(np.uint32)[0])
            if p == 0:
                want = 0
            assert int(oracle.dot_f32([a], [b])) == want, (a, b)
    # products that cancel exactly leave the small ones; all below binary32's
    # smallest denormal: the sum rounds to +0 or to the smallest denormal
    tiny = np.float32(2.0 ** -100)
    assert int(oracle.dot_f32([3.0, -3.0, tiny], [5.0, 5.0, tiny])) == 0          # 2^-200 -> +0
    assert int(oracle.dot_f32([tiny, -tiny], [tiny, tiny])) == 0                  # exact zero
    d = np.float32(2.0 ** -75)
    assert int(oracle.dot_f32([d] * 3, [d] * 3)) == 2                            # 3 * 2^-150 -> 2 units
    assert int(oracle.dot_f32([d], [d])) == 0                                    # half a unit, ties to even
    u = np.float32(2.0 ** -100)
    assert int(oracle.dot_f32([d, u], [d, u])) == 1                              # just above half a unit
    assert int(oracle.dot_f32([1.0, 2.0 ** -12, u], [1.0, 2.0 ** -12, u])) == 0x3F800001   # just above a tie
    assert int(oracle.dot_f32([1.0, 2.0 ** -12], [1.0, 2.0 ** -12])) == 0x3F800000         # the tie itself


def test_dot_f32_specials():
    inf, nan = np.float32(np.inf), np.float32(np.nan)
    assert int(oracle.dot_f32([inf, 1.0], [1.0, 2.0])) == 0x7F800000
    assert int(oracle.dot_f32([inf], [-1.0])) == 0xFF800000
    assert int(oracle.dot_f32([inf, inf], [1.0, -1.0])) == 0x7FC00000
    assert int(oracle.dot_f32([inf], [0.0])) == 0x7FC00000                   # inf * 0 is the default NaN
    q = np.array([0x7FC01234], dtype=np.uint32).view(np.float32)[0]
    assert int(oracle.dot_f32([q, 1.0], [2.0, 3.0])) == 0x7FC01234            # payload kept
    fmax = np.finfo(np.float32).max
    assert int(oracle.dot_f32([fmax, fmax], [2.0, -1.0])) == int(np.array([fmax]).view(np.uint32)[0])
    assert int(oracle.dot_f32([fmax], [2.0])) == 0x7F800000
