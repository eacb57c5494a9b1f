"""The C ABI without a GPU: the library loads, exports every function
include/exsum.h declares, and rejects bad arguments on the host before any
device work (no compute call is made here)."""
import ctypes
import os
import re

import pytest

import paper_1505_05571_amd as ex

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "exsum.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(exsum_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ex.library_path()):
        from paper_1505_05571_amd import build
        build.build()
    return ex.load_library()


def test_header_declares_expected_entry_points():
    names = declared_functions()
    assert "exsum_f64" in names and "exsum_segmented_f64" in names
    assert set(names) == set(ex.EXPORTED_SYMBOLS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = os.popen("nm -D --defined-only %s" % ex.library_path()).read()
    for name in declared_functions():
        assert re.search(r"\bT %s\b" % name, out), name


def test_status_strings(lib):
    assert ex.exsum_status_string(0) == "ok"
    assert ex.exsum_status_string(1) == "invalid argument"
    assert ex.exsum_status_string(99) == "unknown status"


def test_host_side_argument_checks(lib):
    P = ctypes.c_void_p
    assert lib.exsum_f64(None, -1, P(8), None) == 1
    assert lib.exsum_f64(None, 10, P(8), None) == 1          # x NULL with work to do
    assert lib.exsum_f64(P(8), 10, None, None) == 1          # out NULL
    assert lib.exsum_f64(P(8), 1 << 40, P(8), None) == 1     # too many terms
    assert lib.exsum_inexact_f64(None, -5, P(8), None) == 1
    assert lib.exsum_segmented_f64(None, None, -1, None, None) == 1
    assert lib.exsum_segmented_f64(None, None, 0, None, None) == 0   # nothing to do
    assert lib.exsum_segmented_f64(P(8), None, 3, P(8), None) == 1   # offsets NULL
    assert lib.exsum_segmented_f64(P(8), P(8), 3, None, None) == 1   # out NULL
    assert lib.exsum_f64_cfg(P(8), 4, P(8), None, None) == 1


def test_config_roundtrip_and_validation(lib):
    c0 = ex.exsum_get_config()
    try:
        c = ex.exsum_get_config()
        c.large_block, c.large_vec, c.large_depth, c.large_mode = 512, 3, 2, 0
        ex.exsum_set_config(c)
        assert ex.exsum_get_config().large_vec == 3
        c.large_block, c.large_vec, c.large_depth, c.large_mode = 1024, 4, 2, 1
        ex.exsum_set_config(c)
        assert ex.exsum_get_config().large_mode == 1
        for field, bad in [("large_vec", 8), ("large_block", 128), ("precombine", -1), ("large_mode", 2),
                           ("seg_small_max", 1 << 21), ("large_grid", -3)]:
            c = ex.exsum_get_config()
            setattr(c, field, bad)
            with pytest.raises(ex.ExsumError):
                ex.exsum_set_config(c)
    finally:
        ex.exsum_set_config(c0)


def header_variant_list():
    """The (block, vec, depth, mode) shapes the header documents as built."""
    text = open(HEADER).read()
    m = re.search(r"Built \(block, vec, depth, mode\):(.*?)\.\s*\n", text, flags=re.S)
    assert m, "variant list not found in exsum.h"
    return [tuple(int(v) for v in t.split(",")) for t in re.findall(r"\((\d+,\d+,\d+,\d)\)", m.group(1))]


def test_built_variants_match_header_and_config_checks(lib):
    """One table: the variants the library reports as built are the ones the
    header documents and exactly the shapes exsum_set_config accepts; the GPU
    parity tests run every one of them (tests/test_gpu_sum.py reads the same
    list from the library)."""
    built = ex.exsum_large_variants()
    assert len(built) == len(set(built)) == 10
    assert sorted(built) == sorted(header_variant_list())
    c0 = ex.exsum_get_config()
    try:
        for block in (64, 128, 256, 512, 768, 1024):
            for vec in range(1, 9):
                for depth in range(1, 6):
                    for mode in (0, 1):
                        c = ex.exsum_get_config()
                        c.large_block, c.large_vec, c.large_depth, c.large_mode = block, vec, depth, mode
                        ok = True
                        try:
                            ex.exsum_set_config(c)
                        except ex.ExsumError:
                            ok = False
                        assert ok == ((block, vec, depth, mode) in built), (block, vec, depth, mode)
    finally:
        ex.exsum_set_config(c0)


# ---- serving loop: the scheduler's plan (host only) and host-side checks ----

def plan_invariants(lens, cfg, plan):
    """Check a plan against the scheduling rules stated in exsum.h."""
    import numpy as np
    lens = np.asarray(lens, dtype=np.int64)
    req, off, ln, st, sl, exp = (plan[k] for k in ("req", "off", "len", "step", "slot", "expected"))
    NOT_FINAL = 0xFFFFFFFF
    # every request covered exactly once, in order, in pieces of at most piece_terms
    for r in range(lens.size):
        idx = np.nonzero(req == r)[0]
        assert idx.size >= 1, r
        assert np.all(np.diff(st[idx]) >= 0)
        o, l = off[idx], ln[idx]
        assert o[0] == 0 and np.all(o[1:] == (o + l)[:-1]) and (o + l)[-1] == lens[r], r
        assert np.all(l <= cfg.piece_terms)
        last_step = st[idx].max()
        if lens[r] <= cfg.piece_terms:
            # never split: one piece, rounded where it is summed, no slot
            assert idx.size == 1 and exp[idx[0]] == 1 and sl[idx[0]] == -1, r
        else:
            assert idx.size >= 2 and np.all(sl[idx] == sl[idx[0]]) and 0 <= sl[idx[0]] < cfg.max_slots
            fin = st[idx] == last_step
            assert np.all(exp[idx][fin] == idx.size), r
            assert np.all(exp[idx][~fin] == NOT_FINAL), r
    # per step: term budget and piece cap
    for s in np.unique(st):
        m = st == s
        assert ln[m].sum() <= cfg.step_terms
        assert m.sum() <= cfg.max_pieces
    # a slot is held by at most one request at a time, and at most max_slots are held
    spans = {}
    for r in np.unique(req[sl >= 0]):
        idx = np.nonzero(req == r)[0]
        spans[int(r)] = (int(sl[idx[0]]), int(st[idx].min()), int(st[idx].max()))
    for s in range(int(st.max()) + 1 if st.size else 0):
        held = [v[0] for v in spans.values() if v[1] <= s <= v[2]]
        assert len(held) == len(set(held)) and len(held) <= cfg.max_slots


def small_cfg(**kw):
    c = ex.exsum_server_default_config()
    c.step_terms, c.piece_terms, c.max_slots, c.max_pieces = 1 << 12, 1 << 9, 3, 64
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_server_plan_invariants(lib):
    import numpy as np
    rng = np.random.default_rng(0)
    cases = [
        [0, 1, 512, 513, 1024, 5000, 0, 3, 100000],
        list(np.rint(10.0 ** rng.uniform(0, 5.3, size=300)).astype(np.int64)),
        [1 << 12] * 7 + [1] * 50,
        [],
    ]
    for lens in cases:
        for cfg in (small_cfg(), small_cfg(max_slots=1, max_pieces=3), small_cfg(step_terms=1 << 9),
                    ex.exsum_server_default_config()):
            plan = ex.exsum_server_plan(lens, cfg)
            plan_invariants(lens, cfg, plan)


def test_server_plan_lays_out_a_requests_pieces_in_a_row(lib):
    """Within a step, the pieces of one request after its first come in one
    contiguous block of the list, in the order of its terms, so that the
    piece kernel's workgroups meet them as runs (summed in one accumulator
    and merged once)."""
    import numpy as np
    rng = np.random.default_rng(9)
    lens = list(np.rint(10.0 ** rng.uniform(2, 5.5, size=60)).astype(np.int64))
    for cfg in (small_cfg(step_terms=1 << 14), small_cfg(step_terms=1 << 16, max_pieces=400),
                ex.exsum_server_default_config()):
        plan = ex.exsum_server_plan(lens, cfg)
        for s in np.unique(plan["step"]):
            idx = np.nonzero(plan["step"] == s)[0]
            req, off = plan["req"][idx], plan["off"][idx]
            for r in np.unique(req):
                pos = np.nonzero(req == r)[0]
                rest = pos[1:]
                assert np.all(np.diff(rest) == 1), (s, r)
                assert np.all(np.diff(off[pos]) > 0), (s, r)


def test_server_plan_shares_steps_fairly(lib):
    import numpy as np
    # a short request behind a long one is served in the first step
    cfg = small_cfg()
    plan = ex.exsum_server_plan([1 << 20, 10], cfg)
    assert plan["step"][plan["req"] == 1][0] == 0
    # every step of a lone long request uses the whole budget but the last
    plan = ex.exsum_server_plan([10 * cfg.step_terms + 7], cfg)
    per_step = np.bincount(plan["step"], weights=plan["len"])
    assert np.all(per_step[:-1] == cfg.step_terms) and per_step[-1] == 7


def test_server_plan_admits_by_memory_budget(lib):
    """With a memory budget of two slots (576 B each) plus a few piece
    descriptors (32 B), at most two requests that are cut into pieces hold a
    slot at once, even with many free slots; the others wait, in order, and
    are admitted as the first complete.  Short requests are not held back,
    and no step describes more pieces than the budget leaves."""
    import numpy as np
    lens = [5000] * 6 + [10] * 5
    free = small_cfg(max_slots=64)
    tight = small_cfg(max_slots=64, mem_budget=2 * 576 + 4 * 32)
    p_free = ex.exsum_server_plan(lens, free)
    p_tight = ex.exsum_server_plan(lens, tight)
    plan_invariants(lens, tight, p_tight)

    def concurrent(plan):
        spans = {}
        for r in np.unique(plan["req"][plan["slot"] >= 0]):
            st = plan["step"][plan["req"] == r]
            spans[int(r)] = (int(st.min()), int(st.max()))
        return max(sum(1 for a, b in spans.values() if a <= s <= b) for s in range(int(plan["step"].max()) + 1)), spans

    n_free, _ = concurrent(p_free)
    n_tight, spans = concurrent(p_tight)
    assert n_free == 6 and n_tight == 2
    # the waiting requests start in submission order, each after one has finished
    starts = [spans[r][0] for r in range(6)]
    assert starts == sorted(starts) and starts[2] > min(spans[0][1], spans[1][1])
    # the short requests do not wait behind the long ones that wait for room:
    # all are served before the third long request is admitted
    assert np.all(p_tight["step"][np.isin(p_tight["req"], range(6, 11))] < starts[2])
    assert np.all(p_free["step"][np.isin(p_free["req"], range(6, 11))] == 0)
    # pieces per step within what the budget leaves after the held slots
    for s in np.unique(p_tight["step"]):
        held = sum(1 for a, b in spans.values() if a <= s <= b)
        assert (p_tight["step"] == s).sum() * 32 + held * 576 <= tight.mem_budget
    # a budget below one slot and one piece is rejected
    import ctypes
    P = ctypes.c_void_p
    h = P(0)
    bad = small_cfg(mem_budget=600)
    assert lib.exsum_server_create(ctypes.byref(bad), None, ctypes.byref(h)) == 1
    with pytest.raises(ex.ExsumError):
        ex.exsum_server_plan(lens, bad)


def test_server_host_side_checks(lib):
    import ctypes
    P = ctypes.c_void_p
    bad = small_cfg(piece_terms=0)
    h = P(0)
    assert lib.exsum_server_create(ctypes.byref(bad), None, ctypes.byref(h)) == 1
    for field, value in (("step_terms", 1), ("max_slots", 0), ("max_inflight", 65), ("max_pieces", 0),
                         ("short_max", -1), ("precombine", 65)):
        c = small_cfg(**{field: value})
        assert lib.exsum_server_create(ctypes.byref(c), None, ctypes.byref(h)) == 1, field
    assert lib.exsum_server_create(None, None, None) == 1
    n = ctypes.c_int64(0)
    assert lib.exsum_server_submit(None, P(8), 1, P(8), ctypes.byref(n)) == 1
    assert lib.exsum_server_step(None, ctypes.byref(n)) == 1
    assert lib.exsum_server_poll(None, None, 0, ctypes.byref(n)) == 1
    assert lib.exsum_server_drain(None) == 1
    assert lib.exsum_server_destroy(None) == 0
    d = ctypes.c_double(0)
    assert lib.exsum_server_replay(None, None, None, None, None, 0, None, None, ctypes.byref(d)) == 1
    # a trace whose arrivals go backwards, or a negative length, is refused before any device work
    import numpy as np
    st = np.zeros(2, dtype=np.int64)
    ln = np.array([1, -1], dtype=np.int64)
    ar = np.array([0.0, 1.0])
    lat = np.zeros(2)
    args = [P(8), P(st.ctypes.data), P(ln.ctypes.data), P(ar.ctypes.data), 2, P(8), None, P(lat.ctypes.data),
            ctypes.byref(d)]
    assert lib.exsum_serial_replay(*args) == 1
    ln[1] = 1
    ar[1] = -1.0
    assert lib.exsum_serial_replay(*args) == 1
    lens = np.array([-1], dtype=np.int64)
    cnt = ctypes.c_int64(0)
    assert lib.exsum_server_plan(None, P(lens.ctypes.data), 1, 0, None, None, None, None, None, None,
                                 ctypes.byref(cnt)) == 1


def test_further_reductions_host_checks(lib):
    import ctypes
    P = ctypes.c_void_p
    assert lib.exsum_sqnorm_f64(None, 4, P(8), None) == 1
    assert lib.exsum_sqnorm_f64(P(8), -1, P(8), None) == 1
    assert lib.exsum_dot_f64(P(8), None, 4, P(8), None) == 1
    assert lib.exsum_dot_f64(P(8), P(8), 4, None, None) == 1
    assert lib.exsum_mean_f64(P(8), 1 << 40, P(8), None) == 1
    assert lib.exsum_f32(None, 3, P(8), None) == 1
    assert lib.exsum_dot_f32(P(8), None, 3, P(8), None) == 1
    assert lib.exsum_dot_f32(P(8), P(8), -1, P(8), None) == 1
    assert lib.exsum_check_offsets(P(8), -1, -1, P(8), None) == 1
    assert lib.exsum_check_offsets(None, 3, -1, P(8), None) == 1
    assert lib.exsum_check_offsets(P(8), 3, -1, None, None) == 1
    assert lib.exsum_check_offsets(P(8), 1 << 31, -1, P(8), None) == 1
    # the accumulator state must be 64-byte aligned device memory
    assert lib.exsum_acc_zero(None, None) == 1
    assert lib.exsum_acc_zero(P(64 + 8), None) == 1
    assert lib.exsum_acc_add_f64(P(64), None, 5, None) == 1
    assert lib.exsum_acc_add_f64(P(64), P(8), -2, None) == 1
    assert lib.exsum_acc_add_f64(P(64), None, 0, None) == 0          # nothing to add
    assert lib.exsum_acc_merge(P(64), P(64), None) == 1              # a state into itself
    assert lib.exsum_acc_merge(P(64), P(96), None) == 1
    assert lib.exsum_acc_round_f64(P(64), None, None) == 1
    assert ex.EXSUM_ACC_BYTES == 576


def test_tuning_file_checks(lib, tmp_path):
    # checked on the host before any device query
    assert lib.exsum_load_tuning(None) == 1
    assert lib.exsum_load_tuning(str(tmp_path / "missing.json").encode()) == 1
    bad = tmp_path / "bad.json"
    bad.write_text('{"exsum_tuning": 1, "device": "x"}')
    assert lib.exsum_load_tuning(str(bad).encode()) == 1
    other = tmp_path / "v2.json"
    other.write_text('{"exsum_tuning": 2, "device": "x", "arch": "y", "cus": 1, "config": {}}')
    assert lib.exsum_load_tuning(str(other).encode()) == 1
    assert lib.exsum_autotune(None, None, -1, None) == 1
