"""HIP graph capture of the library calls: after one call on a stream has
allocated that stream's workspace, exsum_f64, exsum_segmented_f64 and the
further reductions can be captured on it and replayed; every replay must give
the oracle's bits, with eager work between replays and with input changed
between replays (the graph reads the buffers live)."""
import numpy as np
import pytest

import oracle
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
    return t.cpu().numpy().view(np.uint64)


def test_capture_and_replay(ex):
    s = torch.cuda.Stream()
    x1 = W.uniform_exponent(2_000_003, seed=31)
    x2 = W.uniform_exponent(2_000_003, seed=33)
    xs, off = W.segments(nseg=3000, seed=32, hi=40000)
    y = W.uniform_exponent(2_000_003, seed=34, kmin=-200, kmax=200)
    with torch.cuda.stream(s):
        xt = torch.from_numpy(x1).to("cuda:0")
        yt = torch.from_numpy(y).to("cuda:0")
        xst = torch.from_numpy(xs).to("cuda:0")
        offt = torch.from_numpy(off).to("cuda:0")
        out = torch.empty(4, dtype=torch.float64, device="cuda:0")
        outs = torch.empty(off.size - 1, dtype=torch.float64, device="cuda:0")
        # first calls on this stream: allocate its workspace outside the capture
        ex.exsum_f64(xt, out=out[0:1], stream=s)
        ex.exsum_segmented_f64(xst, offt, out=outs, stream=s, check=False)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ex.exsum_f64(xt, out=out[0:1], stream=s)
        ex.exsum_segmented_f64(xst, offt, out=outs, stream=s, check=False)
        ex.exsum_dot_f64(xt, yt, out=out[1:2], stream=s)
        ex.exsum_mean_f64(xt, out=out[2:3], stream=s)
    want_seg = oracle.segmented_f64(xs, off)
    for rep in range(4):
        xv = x1 if rep % 2 == 0 else x2
        # eager work between replays: new input, poisoned outputs, another sum
        xt.copy_(torch.from_numpy(xv))
        out.fill_(float("nan"))
        outs.fill_(float("nan"))
        ex.exsum_f64(yt, out=out[3:4])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = bits(out)
        assert got[0] == int(oracle.sum_f64(xv)), rep
        assert got[1] == int(oracle.dot_f64(xv, y)), rep
        assert got[2] == int(oracle.mean_f64(xv)), rep
        assert got[3] == int(oracle.sum_f64(y)), rep
        assert np.array_equal(bits(outs), want_seg), rep


def test_capture_binary32(ex):
    """The binary32 sum and dot product (the narrow kernel) captured and
    replayed, with the input changed and the outputs poisoned between
    replays."""
    rng = np.random.default_rng(35)

    def draws(n, kmax):
        b = ((rng.integers(0, 2, size=n, dtype=np.uint32) << np.uint32(31))
             | (rng.integers(127 - kmax, 127 + kmax + 1, size=n, dtype=np.uint32) << np.uint32(23))
             | rng.integers(0, 1 << 23, size=n, dtype=np.uint32))
        return b.view(np.float32)

    n = 3_000_017
    x1, x2, y = draws(n, 60), draws(n, 60), draws(n, 40)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        xt = torch.from_numpy(x1).to("cuda:0")
        yt = torch.from_numpy(y).to("cuda:0")
        out = torch.empty(2, dtype=torch.float32, device="cuda:0")
        ex.exsum_f32(xt, out=out[0:1], stream=s)              # allocates this stream's workspace
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ex.exsum_f32(xt, out=out[0:1], stream=s)
        ex.exsum_dot_f32(xt, yt, out=out[1:2], stream=s)
    for rep in range(4):
        xv = x1 if rep % 2 == 0 else x2
        xt.copy_(torch.from_numpy(xv))
        out.fill_(float("nan"))
        ex.exsum_f32(yt)                                      # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint32)
        assert int(got[0]) == int(oracle.sum_f32(xv)), rep
        assert int(got[1]) == int(oracle.dot_f32(xv, y)), rep


@pytest.mark.parametrize("mode", [0, 1])
def test_capture_segmented_both_modes(ex, mode):
    """The segmented call in either launch mode (two launches, or the
    persistent launch whose device cursors its last wave resets) captured and
    replayed several times, with eager segmented calls on another stream and
    poisoned outputs between replays: every replay gives the oracle's bits."""
    base = ex.exsum_get_config()
    c = ex.exsum_get_config()
    c.seg_mode = mode
    ex.exsum_set_config(c)
    try:
        s = torch.cuda.Stream()
        xs, off = W.segments(nseg=20000, seed=36, hi=100000)
        want = oracle.segmented_f64(xs, off)
        with torch.cuda.stream(s):
            xst = torch.from_numpy(xs).to("cuda:0")
            offt = torch.from_numpy(off).to("cuda:0")
            outs = torch.empty(off.size - 1, dtype=torch.float64, device="cuda:0")
            ex.exsum_segmented_f64(xst, offt, out=outs, stream=s, check=False)   # this stream's workspace
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            ex.exsum_segmented_f64(xst, offt, out=outs, stream=s, check=False)
        other = torch.empty_like(outs)
        for rep in range(4):
            outs.fill_(float("nan"))
            ex.exsum_segmented_f64(xst, offt, out=other, check=False)          # eager, current stream
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(bits(outs), want), rep
            assert np.array_equal(bits(other), want), rep
    finally:
        ex.exsum_set_config(base)
