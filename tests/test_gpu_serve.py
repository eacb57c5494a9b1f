"""GPU parity of the serving loop: every request's bits, served in a mix
through continuous batching (split across pieces, steps and accumulator
slots), equal the bits of the request summed alone and the oracle's."""
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


def bits(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def tiny_cfg(ex, **kw):
    c = ex.exsum_server_default_config()
    c.step_terms, c.piece_terms, c.short_max, c.max_slots, c.max_pieces, c.max_inflight = (
        1 << 16, 1 << 13, 1024, 3, 40, 2)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


LENS = [0, 1, 2, 63, 64, 65, 1000, 1024, 1025, 4096, 8191, 8192, 8193, 50000, 65536, 65537, 300001, 2000003]


def pool_and_requests(seed, n_pool=3_000_000):
    pool = W.uniform_exponent(n_pool, seed=seed)
    rng = np.random.default_rng(seed)
    lens = np.array(LENS + list(rng.integers(0, 20000, size=40)), dtype=np.int64)
    starts = np.array([rng.integers(0, n_pool - L + 1) for L in lens], dtype=np.int64)
    return pool, starts, lens


@pytest.mark.parametrize("cfg_kw", [dict(), dict(short_max=0), dict(short_max=1 << 13, max_inflight=1),
                                    dict(max_slots=1, max_pieces=5), "default"])
def test_mixed_requests_match_alone_and_oracle(ex, cfg_kw):
    pool, starts, lens = pool_and_requests(1)
    want = oracle.sum_ranges_f64(pool, starts, lens)
    pt = torch.from_numpy(pool).to("cuda:0")
    out = torch.full((lens.size,), np.nan, dtype=torch.float64, device="cuda:0")
    cfg = ex.exsum_server_default_config() if cfg_kw == "default" else tiny_cfg(ex, **cfg_kw)
    with ex.Server(cfg) as srv:
        ids = [srv.submit(pt[s:s + L], out, i) for i, (s, L) in enumerate(zip(starts, lens))]
        assert ids == list(range(lens.size))
        srv.drain()
        done = srv.poll(10000)
        assert sorted(done) == ids
        assert srv.pending() == 0
    got = bits(out)
    assert np.array_equal(got, want)
    alone = torch.empty(1, dtype=torch.float64, device="cuda:0")
    for i in (0, 5, 13, 17, 20):
        ex.exsum_f64(pt[starts[i]:starts[i] + lens[i]], out=alone)
        assert bits(alone)[0] == got[i]


def test_interleaved_submit_step_poll(ex):
    pool, starts, lens = pool_and_requests(2)
    want = oracle.sum_ranges_f64(pool, starts, lens)
    pt = torch.from_numpy(pool).to("cuda:0")
    out = torch.full((lens.size,), np.nan, dtype=torch.float64, device="cuda:0")
    seen = []
    with ex.Server(tiny_cfg(ex)) as srv:
        order = np.random.default_rng(2).permutation(lens.size)
        for k, i in enumerate(order):
            srv.submit(pt[starts[i]:starts[i] + lens[i]], out, int(i))
            if k % 3 == 0:
                srv.step()
            seen += srv.poll()
        srv.drain()
        seen += srv.poll()
    assert sorted(seen) == list(range(lens.size))
    assert np.array_equal(bits(out), want)


def test_specials_and_long_chains_through_the_server(ex):
    parts = []
    for c in long_chain_cases():
        big = np.zeros(20001, dtype=np.float64)
        big[::20001 // c.size][:c.size] = c
        parts += [c, big]
    base = W.uniform_exponent(30000, seed=5)
    for sp in ([np.inf], [-np.inf], [np.inf, -np.inf], [np.nan]):
        y = base.copy()
        y[[7, 29000][:len(sp)]] = sp
        parts.append(y)
    lens = np.array([p.size for p in parts], dtype=np.int64)
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    pool = np.concatenate(parts)
    want = oracle.sum_ranges_f64(pool, starts, lens)
    pt = torch.from_numpy(pool).to("cuda:0")
    out = torch.empty(lens.size, dtype=torch.float64, device="cuda:0")
    with ex.Server(tiny_cfg(ex, piece_terms=1 << 11, step_terms=1 << 13)) as srv:
        for i, (s, L) in enumerate(zip(starts, lens)):
            srv.submit(pt[s:s + L], out, i)
        srv.drain()
    assert np.array_equal(bits(out), want)


def test_replays_batched_and_serial(ex):
    rng = np.random.default_rng(3)
    n_pool = 2_000_000
    pool = W.uniform_exponent(n_pool, seed=3)
    nreq = 300
    lens = np.rint(10.0 ** rng.uniform(1, 6, size=nreq)).astype(np.int64)
    starts = np.floor(rng.uniform(0, 1, size=nreq) * (n_pool - lens + 1)).astype(np.int64)
    arrival = np.cumsum(rng.exponential(20e-6, size=nreq))
    want = oracle.sum_ranges_f64(pool, starts, lens)
    pt = torch.from_numpy(pool).to("cuda:0")
    out = torch.full((nreq,), np.nan, dtype=torch.float64, device="cuda:0")
    with ex.Server() as srv:
        lat, mk = srv.replay(pt, starts, lens, arrival, out)
    assert np.array_equal(bits(out), want)
    assert np.all(lat > 0) and mk >= arrival[-1]
    out2 = torch.full((nreq,), np.nan, dtype=torch.float64, device="cuda:0")
    lat2, mk2 = ex.exsum_serial_replay(pt, starts, lens, arrival, out2)
    assert np.array_equal(bits(out2), want)
    assert np.all(lat2 > 0) and mk2 >= arrival[-1]


def test_replay_2000_requests_every_result_against_the_oracle(ex):
    """A served trace of 2,000 requests (lengths log-uniform in [10, 10^6],
    slices of one resident pool), replayed in real time through the batching
    server at about twice the serial service rate and then serially: every
    request's bits equal the oracle's (exact prefix sums of the pool)."""
    n_pool = 8_000_000
    pool = W.uniform_exponent(n_pool, seed=7)
    rng = np.random.default_rng(7)
    nreq = 2000
    lens = np.rint(10.0 ** rng.uniform(1, 6, size=nreq)).astype(np.int64)
    starts = np.floor(rng.uniform(0, 1, size=nreq) * (n_pool - lens + 1)).astype(np.int64)
    want = oracle.ranges_by_prefix_f64(pool, starts, lens, stride=1 << 14, nthreads=8)
    # spacing of arrivals: about half the mean serial service time
    arrival = np.cumsum(rng.exponential(10e-6, size=nreq))
    pt = torch.from_numpy(pool).to("cuda:0")
    out = torch.full((nreq,), np.nan, dtype=torch.float64, device="cuda:0")
    with ex.Server() as srv:
        lat, mk = srv.replay(pt, starts, lens, arrival, out)
    got = bits(out)
    assert int((got != want).sum()) == 0
    assert np.all(lat > 0) and mk >= arrival[-1]
    out2 = torch.full((nreq,), np.nan, dtype=torch.float64, device="cuda:0")
    ex.exsum_serial_replay(pt, starts, lens, arrival, out2)
    assert np.array_equal(bits(out2), want)


def test_inputs_written_on_the_stream_are_seen(ex):
    """The server's steps run in order on its stream: inputs filled with NaN
    and then overwritten by a copy on that stream, submitted without any
    synchronisation, are summed from the copy."""
    pool, starts, lens = pool_and_requests(4)
    want = oracle.sum_ranges_f64(pool, starts, lens)
    src = torch.from_numpy(pool).to("cuda:0")
    out = torch.full((lens.size,), np.nan, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        buf = torch.full_like(src, np.nan)
        with ex.Server(tiny_cfg(ex), stream=side) as srv:
            for rep in range(3):
                buf.fill_(np.nan)
                buf.copy_(src)
                for i, (s0, L) in enumerate(zip(starts, lens)):
                    srv.submit(buf[s0:s0 + L], out, i)
                srv.drain()
                assert np.array_equal(bits(out), want), rep
