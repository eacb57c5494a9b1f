"""The allocation-free single sum (exsum_f64_noalloc, a static per-device
scratch accumulator instead of the per-stream workspace) through the C ABI:
its bits equal exsum_f64's and the oracle's, call after call, with a smaller
input following a larger one (the scratch is shared and must be left clean),
on the large and the small-only path."""
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


def u64(t):
    torch.cuda.synchronize()
    return int(t.cpu().numpy().view(np.uint64)[0])


def test_noalloc_matches_exsum_f64_on_consecutive_calls(ex):
    dev = "cuda:0"
    cases = [
        ("uniform_exponent", W.uniform_exponent(3_000_017, seed=11)),      # large path, full grid
        ("small_normal", W.small_normal(100_003, seed=12)),                # large path, fewer workgroups
        ("adversarial", W.adversarial(1 << 20, seed=13)),                  # hot chunk, cancellation, near-max
        ("small_only", W.small_normal(4000, seed=14)),                     # small-only kernel
        ("tiny", W.small_normal(37, seed=15)),
        ("empty", np.zeros(0, dtype=np.float64)),
    ]
    out_a = torch.full((1,), np.nan, dtype=torch.float64, device=dev)
    out_b = torch.full((1,), np.nan, dtype=torch.float64, device=dev)
    for name, x in cases:
        xt = torch.from_numpy(x).to(dev)
        want = int(oracle.sum_f64(x))
        # two calls in a row: the whole input, then a smaller prefix of it
        for part in (xt, xt[: xt.numel() // 3]):
            ex.exsum_f64_noalloc(part, out_a)
            got = u64(out_a)
            ex.exsum_f64(part, out=out_b)
            assert got == u64(out_b), (name, part.numel())
            if part.numel() == xt.numel():
                assert got == want, name
            else:
                assert got == int(oracle.sum_f64(x[: x.size // 3])), name


def test_noalloc_back_to_back_on_one_stream(ex):
    """Several calls queued on one stream without a host wait between them:
    each reads the scratch the previous one left cleared."""
    dev = "cuda:0"
    xs = [W.uniform_exponent(n, seed=20 + k) for k, n in enumerate((2_000_000, 700_001, 5000, 1_500_000, 10))]
    outs = torch.full((len(xs),), np.nan, dtype=torch.float64, device=dev)
    xts = [torch.from_numpy(x).to(dev) for x in xs]
    torch.cuda.synchronize()
    for k, xt in enumerate(xts):
        ex.exsum_f64_noalloc(xt, outs[k:k + 1])
    torch.cuda.synchronize()
    got = outs.cpu().numpy().view(np.uint64)
    for k, x in enumerate(xs):
        assert int(got[k]) == int(oracle.sum_f64(x)), k


def test_noalloc_host_checks(ex):
    import ctypes
    lib = ex.load_library()
    P = ctypes.c_void_p
    assert lib.exsum_f64_noalloc(None, -1, P(8), None) == 1
    assert lib.exsum_f64_noalloc(None, 10, P(8), None) == 1
    assert lib.exsum_f64_noalloc(P(8), 10, None, None) == 1
    assert lib.exsum_f64_noalloc(P(8), 1 << 40, P(8), None) == 1
