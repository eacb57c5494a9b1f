"""The launch-configuration tuner on the GPU: it returns a valid
configuration, makes it the process configuration, writes a cache that
loads back on the same device and is refused for another, and sums under the
tuned configuration still match the oracle bit for bit."""
import json

import numpy as np
import pytest

import oracle
from paper_1505_05571_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FIELDS = ("large_block", "large_vec", "large_depth", "large_mode", "large_grid", "precombine", "small_max",
          "small_grid", "seg_grid", "seg_small_max", "seg_mode", "seg_block", "seg_group")


@pytest.fixture(scope="module")
def ex():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1505_05571_amd as ex
    ex.load_library()
    base = ex.exsum_get_config()
    yield ex
    ex.exsum_set_config(base)


def as_dict(c):
    return {k: int(getattr(c, k)) for k in FIELDS}


def test_autotune_and_cache(ex, tmp_path):
    base = ex.exsum_get_config()
    path = str(tmp_path / "tuning.json")
    rep = ex.exsum_autotune(path)
    assert set(rep["config"]) == set(FIELDS)
    assert as_dict(ex.exsum_get_config()) == rep["config"]
    assert json.loads(open(path).read())["config"] == rep["config"]
    assert rep["cus"] > 0 and "gfx" in rep["arch"]
    # the segmented launch was chosen among both modes on both batch shapes
    seg = rep["measured"]["segmented"]
    assert {r["mode"] for r in seg} == {0, 1} and all(len(r["us"]) == 2 for r in seg)
    best = min(seg, key=lambda r: r["score"])
    assert best["score"] >= 1.0
    cfg = rep["config"]
    assert (cfg["seg_mode"], cfg["seg_small_max"], cfg["seg_grid"]) == (best["mode"], best["small_max"], best["grid"])
    if best["mode"] == 1:
        assert (cfg["seg_block"], cfg["seg_group"]) == (best["block"], best["group"])
    # back to the defaults, then the cache restores the tuned configuration
    ex.exsum_set_config(base)
    ex.exsum_load_tuning(path)
    assert as_dict(ex.exsum_get_config()) == rep["config"]
    # results under the tuned configuration
    for n in (0, 1, 1000, 5000, 100003, 3000017):
        x = W.uniform_exponent(n, seed=n)
        out = ex.exsum_f64(torch.from_numpy(x).to("cuda:0"))
        assert int(out.cpu().numpy().view(np.uint64)[0]) == int(oracle.sum_f64(x)), n
    xs, off = W.segments(nseg=4000, seed=3, hi=200000)
    got = ex.exsum_segmented_f64(torch.from_numpy(xs).to("cuda:0"), torch.from_numpy(off).to("cuda:0"))
    assert np.array_equal(got.cpu().numpy().view(np.uint64), oracle.segmented_f64(xs, off))
    # the full sigma 1.63 batch under the tuned segmented configuration
    xs, off = W.segments(nseg=65536, seed=0, sigma=1.63)
    got = ex.exsum_segmented_f64(torch.from_numpy(xs).to("cuda:0"), torch.from_numpy(off).to("cuda:0"))
    assert np.array_equal(got.cpu().numpy().view(np.uint64), oracle.segmented_f64(xs, off))
    # a cache from another kind of device is refused and changes nothing
    d = json.loads(open(path).read())
    d["cus"] = d["cus"] + 1
    other = str(tmp_path / "other.json")
    open(other, "w").write(json.dumps(d))
    ex.exsum_set_config(base)
    with pytest.raises(ex.ExsumError):
        ex.exsum_load_tuning(other)
    assert as_dict(ex.exsum_get_config()) == as_dict(base)
