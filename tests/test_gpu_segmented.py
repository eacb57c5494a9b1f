"""GPU parity of the segmented (batched) exact sums against the oracle, bit
for bit, for several small/large thresholds and tile sizes."""
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
    if not DEFAULT:
        DEFAULT.append(ex.exsum_get_config())
    yield ex
    ex.exsum_set_config(DEFAULT[0])


DEFAULT = []


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def seg_bits(ex, xt, offt, **kw):
    if not DEFAULT:
        DEFAULT.append(ex.exsum_get_config())
    c = ex.exsum_get_config()
    base = DEFAULT[0]
    for k, _ in c._fields_:
        setattr(c, k, getattr(base, k))
    for k, v in kw.items():
        setattr(c, k, v)
    ex.exsum_set_config(c)
    out = ex.exsum_segmented_f64(xt, offt)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64)


VARIANTS = [
    dict(),
    dict(seg_mode=0),
    dict(seg_mode=0, seg_small_max=0),
    dict(seg_mode=0, seg_small_max=65536, seg_grid=37),
    dict(seg_mode=0, seg_small_max=100, seg_grid=5),
    dict(seg_mode=0, seg_small_max=2048, seg_grid=1),
    dict(seg_mode=0, seg_small_max=4096, seg_grid=1000),
    # one persistent launch: every workgroup shape, unit size and grid
    dict(seg_mode=1),
    dict(seg_mode=1, seg_block=256),
    dict(seg_mode=1, seg_block=1024, seg_group=64, seg_small_max=100),
    dict(seg_mode=1, seg_block=512, seg_grid=1, seg_group=1),
    dict(seg_mode=1, seg_block=256, seg_grid=37, seg_small_max=65536, seg_group=7),
    dict(seg_mode=1, seg_small_max=0, seg_grid=1000),
]


def test_mixed_lengths(ex):
    x, off = W.segments(nseg=3000, seed=1, hi=300000)
    want = oracle.segmented_f64(x, off)
    xt, offt = dev(x), dev(off)
    for v in VARIANTS:
        got = seg_bits(ex, xt, offt, **v)
        assert np.array_equal(got, want), v


def test_empty_and_tiny_segments(ex):
    rng = np.random.default_rng(2)
    L = rng.choice([0, 0, 1, 2, 3, 64, 65, 5000, 70000], size=2000)
    off = np.zeros(L.size + 1, dtype=np.int64)
    np.cumsum(L, out=off[1:])
    x = W.uniform_exponent(int(off[-1]), seed=2)
    want = oracle.segmented_f64(x, off)
    xt, offt = dev(x), dev(off)
    for v in VARIANTS:
        assert np.array_equal(seg_bits(ex, xt, offt, **v), want), v


def test_offsets_not_starting_at_zero_and_specials(ex):
    x = W.uniform_exponent(400000, seed=3)
    x[[10, 20000, 300001]] = [np.inf, np.nan, -np.inf]
    off = np.array([7, 7, 11, 25000, 25001, 300000, 300002, 399999], dtype=np.int64)
    want = oracle.segmented_f64(x, off)
    xt, offt = dev(x), dev(off)
    for v in VARIANTS:
        assert np.array_equal(seg_bits(ex, xt, offt, **v), want), v


def test_hot_chunk_segments(ex):
    rng = np.random.default_rng(4)
    f = rng.integers(0, 1 << 52, size=1 << 20, dtype=np.uint64)
    x = ((np.uint64(0x3FF) << np.uint64(52)) | f).view(np.float64)
    off = np.array([0, 1000, 300000, 300001, 1 << 20], dtype=np.int64)
    want = oracle.segmented_f64(x, off)
    xt, offt = dev(x), dev(off)
    for v in VARIANTS:
        assert np.array_equal(seg_bits(ex, xt, offt, **v), want), v


def test_long_carry_chain_segments(ex):
    # each case once as a short segment and once spread over a long one that
    # workgroup boundaries cut into pieces
    parts, lens = [], []
    for c in long_chain_cases():
        parts.append(c)
        lens.append(c.size)
        big = np.zeros(150001, dtype=np.float64)
        big[::150001 // c.size][:c.size] = c
        parts.append(big)
        lens.append(big.size)
    x = np.concatenate(parts)
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    want = oracle.segmented_f64(x, off)
    xt, offt = dev(x), dev(off)
    for v in VARIANTS:
        assert np.array_equal(seg_bits(ex, xt, offt, **v), want), v


@pytest.mark.parametrize("mode", [0, 1])
def test_repeated_calls_and_shrinking_batches(ex, mode):
    x, off = W.segments(nseg=5000, seed=5, hi=100000)
    xt = dev(x)
    for nseg in (5000, 17, 4999, 1):
        o = off[:nseg + 1]
        want = oracle.segmented_f64(x, o)
        assert np.array_equal(seg_bits(ex, xt, dev(o), seg_mode=mode), want), nseg


@pytest.mark.parametrize("mode", [0, 1])
def test_fewer_terms_than_workgroups(ex, mode):
    # the kernel caps its grid at the number of terms; a segment cut into
    # pieces must count exactly the workgroups that hold one
    x = W.uniform_exponent(300, seed=11)
    for off in ([0, 5, 9, 300], [0, 1], [3, 3, 3], [0, 0, 201, 201], [299, 300]):
        o = np.array(off, dtype=np.int64)
        want = oracle.segmented_f64(x, o)
        xt, offt = dev(x), dev(o)
        for grid in (0, 1, 2, 200, 1000, 8192):
            assert np.array_equal(seg_bits(ex, xt, offt, seg_grid=grid, seg_mode=mode), want), (off, grid)
            assert np.array_equal(seg_bits(ex, xt, offt, seg_grid=grid, seg_small_max=0, seg_mode=mode),
                                  want), (off, grid)


def test_full_size_batched_workload(ex):
    # 65536 segments, lognormal lengths (median 1000, sigma 2), both launch
    # modes, default shapes and every persistent workgroup size
    x, off = W.segments(nseg=65536, seed=0)
    want = oracle.segmented_f64(x, off)
    xt, offt = dev(x), dev(off)
    for kw in (dict(), dict(seg_mode=0), dict(seg_mode=1, seg_block=256), dict(seg_mode=1, seg_block=512),
               dict(seg_mode=1, seg_block=1024)):
        assert np.array_equal(seg_bits(ex, xt, offt, **kw), want), kw


def test_full_size_batched_workload_sigma_163(ex):
    # the same batch with sigma 1.63 (about 2.5e8 terms), at several
    # short/long thresholds: every threshold gives the same bits
    x, off = W.segments(nseg=65536, seed=0, sigma=1.63)
    want = oracle.segmented_f64(x, off)
    xt, offt = dev(x), dev(off)
    assert np.array_equal(seg_bits(ex, xt, offt), want)
    for mode in (0, 1):
        for sm in (0, 4096, 65536, 1 << 20):
            assert np.array_equal(seg_bits(ex, xt, offt, seg_small_max=sm, seg_mode=mode), want), (mode, sm)


def test_many_segments_count_partition(ex):
    # more segments than the weight partition takes (workgroups x 1024): the
    # short kernel splits them by count instead; same bits either way
    x, off = W.segments(nseg=300000, seed=8, median=20.0, sigma=1.5, hi=20000)
    want = oracle.segmented_f64(x, off)
    xt, offt = dev(x), dev(off)
    assert np.array_equal(seg_bits(ex, xt, offt), want)
    assert np.array_equal(seg_bits(ex, xt, offt, seg_small_max=64), want)
    assert np.array_equal(seg_bits(ex, xt, offt, seg_mode=1 - DEFAULT[0].seg_mode), want)
    # a slice below the threshold takes the weight partition
    sub = off[:200001] - off[0]
    assert np.array_equal(seg_bits(ex, dev(x[:int(sub[-1])]), dev(sub)), want[:200000])


def test_check_offsets(ex):
    """The offset validator: -1 for valid offsets, else the first segment
    whose bounds break them (a decrease, a negative start, an end past n)."""
    cases = [
        ([0, 3, 3, 10], 10, -1),
        ([5, 7, 9], None, -1),                 # offsets[0] need not be 0
        ([0], 0, -1),                          # no segments
        ([0, 4, 2, 6, 1], 6, 1),               # first decrease at segment 1
        ([-1, 2, 3], None, 0),                 # negative start
        ([0, 2, 11], 10, 1),                   # end past n
        ([0, 2, 11], None, -1),                # ... not checked without n
    ]
    for off, n, want in cases:
        t = torch.tensor(off, dtype=torch.int64, device="cuda:0")
        got = ex.exsum_check_offsets(t, n)
        torch.cuda.synchronize()
        assert int(got.item()) == want, (off, n)
    big = torch.arange(0, 3 * 300001, 3, dtype=torch.int64, device="cuda:0")
    assert int(ex.exsum_check_offsets(big, 3 * 300000).item()) == -1
    big[200000] = 1                                                   # segment 199999 now decreases
    assert int(ex.exsum_check_offsets(big, 3 * 300000).item()) == 199999


def test_wrapper_validates_offsets_and_empty_input(ex):
    """The binding checks offsets against x's length before the sums run
    (the summing kernels trust them, so no bad offset ever reaches them), and
    an empty x with only empty segments gives +0.0 for each."""
    x = dev(W.uniform_exponent(1000, seed=4))
    for off in ([0, 400, 300, 1000], [0, 500, 1001], [-2, 5, 9]):
        with pytest.raises(ValueError):
            ex.exsum_segmented_f64(x, torch.tensor(off, dtype=torch.int64, device="cuda:0"))
    empty = torch.empty(0, dtype=torch.float64, device="cuda:0")
    off = torch.zeros(6, dtype=torch.int64, device="cuda:0")
    out = torch.full((5,), np.nan, dtype=torch.float64, device="cuda:0")
    ex.exsum_segmented_f64(empty, off, out=out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint64), np.zeros(5, dtype=np.uint64))


def test_small_body_top_chunks(ex):
    """One-wave sums of 1023 to 30,000 terms whose pieces fall on the top
    chunks (terms of magnitude 2^1000 to 2^1024): the copies' final carry,
    folded into their sum, carries across the 64th chunk and into the top
    one.  Random signs, all positive (an exact sum above DBL_MAX rounds to
    +inf), and cancelling pairs with a small remainder, as short segments
    (default threshold, and 65536 so that a 30,000-term segment also gets
    the periodic carries) and as single sums; every result against the
    oracle."""
    rng = np.random.default_rng(11)

    def huge(n, sign):
        v = np.ldexp(rng.uniform(1, 2, n), rng.integers(1000, 1024, n))
        return v * (rng.choice([-1.0, 1.0], n) if sign else 1.0)

    parts = []
    for n in (1023, 1024, 1025, 2047, 4096, 8191, 12288):
        parts.append(huge(n, True))
        parts.append(huge(n, False))
        h = huge(n // 2, False)
        pair = np.empty(2 * h.size)
        pair[0::2], pair[1::2] = h, -h
        pair[rng.integers(0, pair.size, 3)] = [3.0, -0.5, 2.0 ** -1074]
        parts.append(rng.permutation(pair))
        # top chunks only just below overflow, with borrows from below
        m = np.full(n, np.finfo(np.float64).max) * rng.choice([-1.0, 1.0], n)
        m[::7] = -np.ldexp(1.0, 1000)
        parts.append(m)
    parts.append(huge(30000, True))
    parts.append(np.concatenate([huge(15000, False), -huge(15000, False), [1.0]]))
    lens = [p.size for p in parts]
    x = np.concatenate(parts)
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    want = oracle.segmented_f64(x, off)
    xt, offt = dev(x), dev(off)
    for sm in (12288, 65536):
        for mode in (0, 1):
            assert np.array_equal(seg_bits(ex, xt, offt, seg_small_max=sm, seg_mode=mode), want), (sm, mode)
    out = torch.empty(1, dtype=torch.float64, device="cuda:0")
    for k, p in enumerate(parts):
        if 1024 <= p.size <= 4096:
            ex.exsum_f64(dev(p), out=out)
            torch.cuda.synchronize()
            assert int(out.cpu().numpy().view(np.uint64)[0]) == int(oracle.sum_f64(p)), (k, p.size)


def test_small_window_edges(ex):
    """The small body's windowed finish: a sum whose terms' exponent fields
    span few small chunks adds only the copies' words of that window, and
    the accumulator must be clear everywhere else for the next sum.  Each
    class of values below hits one case of the window: 3, 4, 5 and 8 chunks
    (one round of lane groups, a partial second round, two full rounds, the
    limit with 16 copies), 9 and 18 chunks (the full finish with 16 copies;
    9 is still a window with 8), the top chunks (up to overflow), denormals
    (window from chunk 0), zeros (full finish), an infinity or NaN (full
    finish, side words cleared), exact cancellation, and rounding ties.
    Lengths cover edge-only ranges, ragged batches, the 1024-term boundary
    of the direct sum without carries and the longest range the window
    takes without carry steps (24,064 terms with 16 copies).  The segments
    are shuffled so that windowed and full finishes follow each other on
    the same wavefront; every result against the oracle, as segments, as
    single sums and as dot products."""
    rng = np.random.default_rng(23)

    def vals(n, e0, e1, sign=True):
        m = rng.integers(0, 1 << 52, n, dtype=np.uint64)
        e = rng.integers(e0, e1 + 1, n).astype(np.uint64)
        s = (rng.integers(0, 2, n).astype(np.uint64) << np.uint64(63)) if sign else np.uint64(0)
        return ((e << np.uint64(52)) | m | s).view(np.float64)

    classes = {
        "w3": (1024, 1055), "w4": (992, 1055), "w5": (960, 1055), "w8": (864, 1055),
        "w9": (832, 1055), "w18": (544, 1055), "top": (2016, 2046), "top2": (1984, 2046),
        "denorm": (0, 40),
    }
    parts = []
    for name, (e0, e1) in classes.items():
        for n in (1, 2, 3, 5, 64, 129, 511, 513, 1023, 1024, 1025, 2047, 4096, 12288):
            parts.append(vals(n, e0, e1))
        parts.append(vals(3000, e0, e1, sign=False))
    for n in (3, 1024, 5000):
        z = vals(n, 1024, 1055)
        z[rng.integers(0, n, max(1, n // 100))] = 0.0
        parts.append(z)
        sp = vals(n, 992, 1055)
        sp[rng.integers(0, n)] = [np.inf, -np.inf, np.nan][n % 3]
        parts.append(sp)
        h = vals(n, 960, 1055)
        pair = np.empty(2 * n)
        pair[0::2], pair[1::2] = h, -h
        parts.append(rng.permutation(pair))
    tie = np.ldexp(1.0, -53)
    one_up = 1.0 + np.ldexp(1.0, -52)
    for s in (1.0, -1.0):
        parts += [s * np.array([1.0, tie]), s * np.array([1.0, tie, np.ldexp(1.0, -100)]),
                  s * np.array([one_up, tie]), s * np.array([tie, 1.0, -np.ldexp(1.0, -100)])]
    # the longest windowed range, all terms on one chunk at full significand
    # (copy words near 2^62.5), and just past it
    for n in (24063, 24064, 24065):
        parts.append(np.full(n, np.ldexp(2.0 - 2.0 ** -52, 31)))
        parts.append(vals(n, 960, 1055))
    order = rng.permutation(len(parts))
    parts = [parts[i] for i in order]
    lens = [p.size for p in parts]
    x = np.concatenate(parts)
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    want = oracle.segmented_f64(x, off)
    xt, offt = dev(x), dev(off)
    for sm in (12288, 65536):
        for mode in (0, 1):
            got = seg_bits(ex, xt, offt, seg_small_max=sm, seg_mode=mode)
            bad = np.nonzero(got != want)[0]
            assert bad.size == 0, (sm, mode, bad[:5], [lens[i] for i in bad[:5]])
    out = torch.empty(1, dtype=torch.float64, device="cuda:0")
    two = np.ldexp(np.ones(4096), rng.integers(-3, 4, 4096))
    for k, p in enumerate(parts):
        if p.size <= 4096:
            ex.exsum_f64(dev(p), out=out)
            torch.cuda.synchronize()
            assert int(out.cpu().numpy().view(np.uint64)[0]) == int(oracle.sum_f64(p)), (k, p.size)
            if p.size >= 64 and k % 3 == 0:
                y = two[:p.size]
                ex.exsum_dot_f64(dev(p), dev(y), out=out)
                torch.cuda.synchronize()
                assert int(out.cpu().numpy().view(np.uint64)[0]) == int(oracle.dot_f64(p, y)), (k, p.size)


def test_long_range_split_edges(ex):
    """The long-segment kernel's term ranges shrink along the dispatch order
    (range w of G starts at floor(N f(w) / 5G^2), f(w) = w (5G + 4(G - w)))
    once N (G - 4) >= 5 G^2, and are equal otherwise (G capped at N).  Batches
    of N terms just below, at and above that bound for several grids, made of
    segments longer than the small/large threshold so that many are cut into
    pieces over several ranges (merged by ticket), and larger batches; every
    result against the oracle, with the grid and threshold varied."""
    rng = np.random.default_rng(29)
    for G in (5, 6, 37, 64, 300):
        bound = -(-5 * G * G // (G - 4))          # smallest N with N (G - 4) >= 5 G^2
        for N in sorted({bound - 1, bound, bound + 1, 5 * G + 3, 40 * G + 7}):
            if N < 1:
                continue
            lens = []
            left = N
            while left > 0:
                k = int(min(left, rng.integers(1, 3 * max(1, N // G) + 2)))
                lens.append(k)
                left -= k
            x = np.ldexp(rng.uniform(1, 2, N), rng.integers(-40, 40, N)) * rng.choice([-1.0, 1.0], N)
            off = np.zeros(len(lens) + 1, dtype=np.int64)
            np.cumsum(lens, out=off[1:])
            want = oracle.segmented_f64(x, off)
            xt, offt = dev(x), dev(off)
            for sm in (0, 2, 16):
                got = seg_bits(ex, xt, offt, seg_grid=G, seg_small_max=sm, seg_mode=0)
                assert np.array_equal(got, want), (G, N, sm)
