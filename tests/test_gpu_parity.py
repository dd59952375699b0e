"""Parity of the HIP checker (through the C ABI) with the CPU oracle, element by element."""
import os
import sys

import numpy as np
import pytest

import oracle
import tracegen
from golden_io import all_cases
from tracegen.format import KIND, make_meta

pytestmark = pytest.mark.gpu

CASES = all_cases()


@pytest.fixture(scope="module")
def rc():
    from paper_2111_12478_amd import RaceChecker
    c = RaceChecker(0)
    yield c
    c.close()


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("case", CASES, ids=[c.name for c in CASES])
def test_golden(rc, case):
    _say(f"golden {case.name}")
    got = rc.check(case.grid, case.events)
    assert got.status == 0, got
    np.testing.assert_array_equal(got.pairs, case.expected)


@pytest.mark.parametrize("seed", list(range(0, 400)))
def test_random_traces(rc, seed):
    grid, ev = tracegen.random_trace(seed)
    want = oracle.check(grid, ev)
    got = rc.check(grid, ev)
    assert got.status == want.status == 0, (seed, got, want)
    np.testing.assert_array_equal(got.pairs, want.pairs, err_msg=f"seed {seed}")


@pytest.mark.parametrize("seed", list(range(1000, 1040)))
def test_random_traces_larger(rc, seed):
    grid, ev = tracegen.random_trace(seed, max_blocks=6, max_tpb=40, max_events=6000)
    want = oracle.check(grid, ev)
    got = rc.check(grid, ev)
    assert got.status == want.status == 0, (seed, got, want)
    np.testing.assert_array_equal(got.pairs, want.pairs, err_msg=f"seed {seed}")


def test_tiny_workload_matches_oracle_and_bruteforce(rc):
    grid, ev, st, plants = tracegen.generate(tracegen.tiny())
    bf = oracle.bruteforce(grid, ev)
    want = oracle.check(grid, ev)
    np.testing.assert_array_equal(bf.pairs, want.pairs)
    got = rc.check(grid, ev)
    assert got.status == 0
    np.testing.assert_array_equal(got.pairs, want.pairs)
    assert len(plants) == 3 and set(plants.tolist()) <= set(got.pairs.ravel().tolist())


@pytest.mark.parametrize("scale", [64, 16])
def test_large_workload_scaled(rc, scale):
    cfg = tracegen.large(seed=2, scale=scale)
    grid, ev, st, plants = tracegen.generate(cfg)
    _say(f"large/{scale}: {len(ev)} events")
    want = oracle.check(grid, ev)
    got = rc.check(grid, ev)
    assert got.status == want.status == 0
    np.testing.assert_array_equal(got.pairs, want.pairs)
    assert set(plants.tolist()) <= set(got.pairs.ravel().tolist())


def test_repeat_check_same_trace(rc):
    grid, ev = tracegen.random_trace(77, max_events=2000)
    tr, ws, keep = rc.prepare(grid, ev)
    try:
        a = rc.run(tr)
        b = rc.run(tr)
    finally:
        from paper_2111_12478_amd import rd_trace_free
        rd_trace_free(rc.ctx, tr)
    np.testing.assert_array_equal(a.pairs, b.pairs)
    np.testing.assert_array_equal(a.pairs, oracle.check(grid, ev).pairs)


def test_graph_replays_follow_the_events(rc):
    # from its second check on, a trace's check is one graph launch: replays with other sort
    # variants, with and without profiled kernels, and over device events rewritten in place (the
    # graph reads them again) all match the oracle
    import ctypes
    import torch
    from paper_2111_12478_amd import load_library, rd_get_tuning, rd_set_tuning, rd_trace_free
    grid, ev_a, _, _ = tracegen.generate(tracegen.tiny(seed=11))
    grid_b, ev_b, _, _ = tracegen.generate(tracegen.tiny(seed=12))
    assert tuple(grid_b) == tuple(grid) and ev_a.shape == ev_b.shape
    want = {}
    for name, e in (("a", ev_a), ("b", ev_b)):
        want[name] = oracle.check(grid, e)
    dev = torch.from_numpy(ev_a.view(np.int32).copy()).cuda()
    tr, ws, keep = rc.prepare(grid, dev)
    lib = load_library()
    lib.rd_profile_enable.argtypes = [ctypes.c_void_p, ctypes.c_char_p]
    saved = rd_get_tuning(rc.ctx)
    try:
        for step, (name, variant, prof) in enumerate([("a", 0, False), ("a", 0, False), ("b", 0, False),
                                                      ("b", 3, False), ("a", 3, True), ("a", 3, True),
                                                      ("b", 5, False), ("a", 0, False)]):
            src = ev_a if name == "a" else ev_b
            dev.copy_(torch.from_numpy(src.view(np.int32)))
            rd_set_tuning(rc.ctx, variant)
            lib.rd_profile_enable(rc.ctx, b"*" if prof else None)
            got = rc.run(tr)
            torch.cuda.synchronize()
            w = want[name]
            assert got.status == w.status, (step, got, w)
            if w.status == 0:
                np.testing.assert_array_equal(got.pairs, w.pairs, err_msg=f"step {step}")
    finally:
        lib.rd_profile_enable(rc.ctx, None)
        rd_set_tuning(rc.ctx, saved)
        rd_trace_free(rc.ctx, tr)


def test_graph_built_without_knowledge_stages_checks_again_when_needed(rc):
    # a trace without releases, acquires or warp barriers is replayed from a graph built without the
    # knowledge stages; rewritten in place into one that has fence-adjacent atomics (releases and
    # acquires), the replay finds that and the report comes from a whole check again, then back
    import torch
    from paper_2111_12478_amd import rd_trace_free
    from tracegen.format import KIND, make_meta
    grid, ev_a, _, _ = tracegen.generate(tracegen.tiny(seed=31))
    kinds = ev_a[:, 2] & 15
    assert not np.isin(kinds, (KIND["F"], KIND["WBAR"], KIND["ACQ"], KIND["REL"])).any()
    # the same records with some reads turned into device fences (a fence right before or after an
    # atomic of its thread makes it a release or an acquire); still a valid trace
    ev_b = ev_a.copy()
    reads = np.nonzero(kinds == KIND["R"])[0]
    for i in reads[::7]:
        ev_b[i] = (0, ev_b[i, 1], make_meta(KIND["F"], 1, 0), 0)
    want = {"a": oracle.check(grid, ev_a), "b": oracle.check(grid, ev_b)}
    assert want["a"].status == want["b"].status == 0
    assert not np.array_equal(want["a"].pairs, want["b"].pairs)
    dev = torch.from_numpy(ev_a.view(np.int32).copy()).cuda()
    tr, ws, keep = rc.prepare(grid, dev)
    try:
        for step, name in enumerate(["a", "a", "a", "b", "b", "b", "a", "a", "b"]):
            dev.copy_(torch.from_numpy((ev_a if name == "a" else ev_b).view(np.int32)))
            got = rc.run(tr)
            torch.cuda.synchronize()
            assert got.status == 0, (step, got)
            np.testing.assert_array_equal(got.pairs, want[name].pairs, err_msg=f"step {step}")
    finally:
        rd_trace_free(rc.ctx, tr)


def test_report_length_changes_between_checks(rc):
    # the report copy is sized by the trace's previous report: reports that grow, shrink, are cut
    # by a small capacity or only counted all come out whole and in order
    import torch
    from paper_2111_12478_amd import rd_trace_free
    cases = [tracegen.generate(tracegen.tiny(seed=s)) for s in (21, 22, 23, 24)]
    grid = cases[0][0]
    cases = [c for c in cases if tuple(c[0]) == tuple(grid) and c[1].shape == cases[0][1].shape]
    want = [oracle.check(grid, c[1]) for c in cases]
    counts = sorted({len(w.pairs) for w in want if w.status == 0})
    assert len(counts) >= 2, counts
    dev = torch.from_numpy(cases[0][1].view(np.int32).copy()).cuda()
    tr, ws, keep = rc.prepare(grid, dev)
    try:
        order = [0, 1, 2, 3, 3, 2, 1, 0, 0]
        for step, j in enumerate(order):
            dev.copy_(torch.from_numpy(cases[j % len(cases)][1].view(np.int32)))
            w = want[j % len(cases)]
            cap = 2 if step in (4, 6) else None
            got = rc.run(tr, cap) if cap else rc.run(tr)
            torch.cuda.synchronize()
            assert got.status == (w.status if w.status != 0 or not cap or len(w.pairs) <= cap else -4), (step, got)
            if w.status == 0:
                ref = w.pairs if not cap else w.pairs[:cap]
                np.testing.assert_array_equal(got.pairs, ref, err_msg=f"step {step}")
    finally:
        rd_trace_free(rc.ctx, tr)


def _check_with_stats(rc, grid, ev):
    from paper_2111_12478_amd import rd_trace_free, rd_trace_stats
    tr, ws, keep = rc.prepare(grid, ev)
    try:
        res = rc.run(tr)
        return res, (rd_trace_stats(rc.ctx, tr) if res.status == 0 else None)
    finally:
        rd_trace_free(rc.ctx, tr)


@pytest.mark.parametrize("seed", list(range(7000, 7030)))
def test_random_traces_wide_addresses(rc, seed):
    # global words spread over about 2^31 addresses: 32-bit location keys leave no room for the
    # category and phase, which ride in the thread word instead (three arrays through the sort)
    grid, ev = tracegen.random_trace(seed, max_blocks=4, max_tpb=16, max_events=3000)
    ev = ev.copy()
    glob = ((ev[:, 2] >> 6) & 1) == 0
    ev[glob, 0] = ev[glob, 0] * np.uint32(1 << 29)
    want = oracle.check(grid, ev)
    got, stats = _check_with_stats(rc, grid, ev)
    assert got.status == want.status, (seed, got, want)
    if want.status == 0:
        np.testing.assert_array_equal(got.pairs, want.pairs, err_msg=f"seed {seed}")
        if stats["key_bits"] + 2 + int(stats["max_phase"]).bit_length() > 32:
            assert stats["packed"] == 2, stats


def test_elements_in_four_arrays(rc):
    # 32-bit location keys, 65,536 threads and 16,384 barriers: neither the key word nor the thread
    # word has room for the category and the phase, so the info array moves through the sort too
    m = make_meta
    ev = [(0, 0, m(KIND["W"]), 0)] + [(0, 0, m(KIND["BAR"]), 0)] * 16384
    ev += [((1 << 31) + 5, 0, m(KIND["W"]), 0), (0, 0, m(KIND["R"]), 0)]
    ev += [(0, 1, m(KIND["W"]), 0), ((1 << 31) + 5, 1, m(KIND["R"]), 0)]
    ev = np.array(ev, dtype=np.uint32)
    want = oracle.check((65536, 1), ev)
    got, stats = _check_with_stats(rc, (65536, 1), ev)
    assert got.status == 0 and stats["packed"] == 0, (got, stats)
    np.testing.assert_array_equal(got.pairs, want.pairs)


def test_device_resident_events(rc):
    import torch
    grid, ev, _, _ = tracegen.generate(tracegen.tiny(seed=9))
    dev = torch.from_numpy(ev.view(np.int32)).cuda()
    got = rc.check(grid, dev)
    np.testing.assert_array_equal(got.pairs, oracle.check(grid, ev).pairs)


def test_empty_and_single(rc):
    got = rc.check((1, 4), np.zeros((0, 4), np.uint32))
    assert got.status == 0 and len(got.pairs) == 0
    got = rc.check((1, 4), np.array([[5, 0, make_meta(KIND["W"]), 0]], np.uint32))
    assert got.status == 0 and len(got.pairs) == 0


def test_one_hot_location_ragged(rc):
    # every event on one word, sizes that leave ragged tiles
    for n in (4095, 4097, 12289):
        rng = np.random.default_rng(n)
        ev = np.zeros((n, 4), np.uint32)
        ev[:, 0] = 9
        ev[:, 1] = rng.integers(0, 64, n)
        ev[:, 2] = np.where(rng.random(n) < 0.01, make_meta(KIND["W"]), make_meta(KIND["R"]))
        want = oracle.check((2, 32), ev)
        got = rc.check((2, 32), ev, limits={"max_pairs": 1 << 25})
        assert got.status == 0, got
        np.testing.assert_array_equal(got.pairs, want.pairs)


def test_one_hot_location_many_blocks(rc):
    # one word touched by four blocks: every access is checked against its whole prefix, and the
    # n^2/128 chunks of that check overflow the chunk queue (capacity n)
    for n in (4097, 9001):
        rng = np.random.default_rng(n + 1)
        ev = np.zeros((n, 4), np.uint32)
        ev[:, 0] = 9
        ev[:, 1] = rng.integers(0, 64, n)
        ev[:, 2] = np.where(rng.random(n) < 0.01, make_meta(KIND["W"]), make_meta(KIND["R"]))
        want = oracle.check((4, 16), ev)
        got = rc.check((4, 16), ev, limits={"max_pairs": 1 << 25})
        assert got.status == 0, got
        np.testing.assert_array_equal(got.pairs, want.pairs)


def test_one_hot_location_one_block(rc):
    # one block in one phase: only the access's own run can race, and the chunks over the run
    # overflow the queue, so the accesses are queued whole (with the run flag) instead
    for n in (4097, 9001):
        rng = np.random.default_rng(n + 2)
        ev = np.zeros((n, 4), np.uint32)
        ev[:, 0] = 5
        ev[:, 1] = rng.integers(0, 64, n)
        ev[:, 2] = np.where(rng.random(n) < 0.01, make_meta(KIND["W"]), make_meta(KIND["R"]))
        want = oracle.check((1, 64), ev)
        got = rc.check((1, 64), ev, limits={"max_pairs": 1 << 25})
        assert got.status == 0, got
        np.testing.assert_array_equal(got.pairs, want.pairs)


def test_hot_location_among_others(rc):
    # a hot word shared by eight blocks inside an ordinary trace: the queue overflows part way, so
    # some tiles queue chunks and later ones whole accesses
    rng = np.random.default_rng(31)
    n = 40000
    ev = np.zeros((n, 4), np.uint32)
    hot = rng.random(n) < 0.15
    ev[:, 0] = np.where(hot, 7, 100 + rng.integers(0, 5000, n))
    ev[:, 1] = rng.integers(0, 8 * 32, n)
    ev[:, 2] = np.where(rng.random(n) < 0.05, make_meta(KIND["W"]), make_meta(KIND["R"]))
    want = oracle.check((8, 32), ev)
    got = rc.check((8, 32), ev, limits={"max_pairs": 1 << 25})
    assert got.status == 0, got
    np.testing.assert_array_equal(got.pairs, want.pairs)


def test_pair_buffer_overflow_is_reported(rc):
    # 64 threads of one block each write one word: C(64, 2) = 2016 pairs, buffer of 1000
    ev = np.array([(3, t, make_meta(KIND["W"]), 0) for t in range(64)], np.uint32)
    got = rc.check((1, 64), ev, limits={"max_pairs": 1000})
    assert got.status == -2, got
    from paper_2111_12478_amd import rd_races
    got = rc.check((1, 64), ev, limits={"max_pairs": 2016})
    assert got.status == 0 and len(got.pairs) == 2016


def test_truncated_report(rc):
    grid, ev, _, _ = tracegen.generate(tracegen.tiny())
    want = oracle.check(grid, ev).pairs
    got = rc.check(grid, ev, capacity=5)
    assert got.status == -4
    np.testing.assert_array_equal(got.pairs, want[:5])


from test_oracle_validation import CASES as VCASES  # noqa: E402


@pytest.mark.parametrize("name,grid,events,status,bad", VCASES, ids=[c[0] for c in VCASES])
def test_validation_matches_oracle(rc, name, grid, events, status, bad):
    got = rc.check(grid, events)
    assert got.status == status, (name, got)
    assert got.bad_index == bad, (name, got)


# ---------------------------------------------------------------- halo-exchange stencil traces

@pytest.mark.parametrize("seed,shape", [(s, sh) for s in range(4) for sh in
                                        [(2, 2, 8, 2, 3), (4, 4, 32, 3, 4), (3, 5, 16, 4, 5), (8, 8, 64, 5, 3)]])
def test_stencil_traces(rc, seed, shape):
    rb, cb, tpb, rows, sweeps = shape
    cfg = tracegen.stencil_small(seed=seed, rb=rb, cb=cb, tpb=tpb, rows=rows, sweeps=sweeps, plant_rate=0.08)
    grid, ev, st, plants = tracegen.generate_stencil(cfg)
    _say(f"stencil seed {seed} shape {shape}: {len(ev)} events, {len(plants)} plants")
    want = oracle.check(grid, ev)
    got = rc.check(grid, ev)
    assert got.status == want.status == 0, (got, want)
    np.testing.assert_array_equal(got.pairs, want.pairs)


def test_stencil_unplanted_is_race_free(rc):
    cfg = tracegen.stencil_small(seed=9, rb=16, cb=16, tpb=64, rows=4, sweeps=4, plant_rate=0.0)
    grid, ev, st, plants = tracegen.generate_stencil(cfg)
    _say(f"unplanted stencil: {len(ev)} events")
    want = oracle.check(grid, ev)
    assert want.status == 0 and len(want.pairs) == 0, want
    got = rc.check(grid, ev)
    assert got.status == 0 and len(got.pairs) == 0, got


@pytest.mark.parametrize("seed,plant_rate", [(5, 2e-3), (6, 0.0), (7, 5e-3)])
def test_stencil_full_grid_lock_chain(rc, seed, plant_rate):
    # the full 64 x 64 grid of blocks (one sweep, one row per block): the reduction's lock is
    # handed through 4,096 critical sections, so the knowledge engine replays that chain over
    # several windows of operations; planted block-scope downgrades break it at some sections
    cfg = tracegen.stencil_small(seed=seed, rb=64, cb=64, tpb=32, rows=1, sweeps=1, plant_rate=plant_rate)
    grid, ev, st, plants = tracegen.generate_stencil(cfg)
    n_ops = int(np.isin(ev[:, 2] & 15, (6, 7)).sum())
    _say(f"full-grid stencil seed {seed}: {len(ev)} events, {n_ops} lock operations, {len(plants)} plants")
    assert n_ops == 2 * 4096
    want = oracle.check(grid, ev)
    # knowledge vectors are 8,192 words wide here (4,096 blocks + 4,096 releasing threads)
    got = rc.check(grid, ev, limits={"clock_bytes": 4 << 30})
    assert got.status == want.status == 0, (got, want)
    np.testing.assert_array_equal(got.pairs, want.pairs)
    if plant_rate == 0.0:
        assert len(want.pairs) == 0


def test_stencil_full_grid_pool_too_small_is_reported(rc):
    # the same trace with the default 256 MiB knowledge-vector pool: more vectors than fit, so the
    # engine numbers no operation and every later stage that reads knowledge skips; the check
    # reports RD_ENOMEM (this once read tables the engine had not written)
    cfg = tracegen.stencil_small(seed=5, rb=64, cb=64, tpb=32, rows=1, sweeps=1, plant_rate=2e-3)
    grid, ev, st, plants = tracegen.generate_stencil(cfg)
    got = rc.check(grid, ev)
    assert got.status == -2, got


# ---------------------------------------------------------------- traces without warp barriers
# (their knowledge vectors come from the parallel engine; warp barriers use the interpreter)

@pytest.mark.parametrize("seed", list(range(5000, 5300)))
def test_random_traces_no_warp_barriers(rc, seed):
    grid, ev = tracegen.random_trace(seed, wbar=False)
    want = oracle.check(grid, ev)
    got = rc.check(grid, ev)
    assert got.status == want.status, (seed, got, want)
    if want.status == 0:
        np.testing.assert_array_equal(got.pairs, want.pairs, err_msg=f"seed {seed}")
    else:
        assert got.bad_index == want.bad_index


@pytest.mark.parametrize("seed", list(range(6000, 6040)))
def test_random_traces_no_warp_barriers_larger(rc, seed):
    grid, ev = tracegen.random_trace(seed, max_blocks=8, max_tpb=48, max_events=8000, wbar=False)
    want = oracle.check(grid, ev)
    got = rc.check(grid, ev)
    assert got.status == want.status, (seed, got, want)
    if want.status == 0:
        np.testing.assert_array_equal(got.pairs, want.pairs, err_msg=f"seed {seed}")


# ---------------------------------------------------------------- location-sort variants

def _n_variants():
    from paper_2111_12478_amd import rd_tuning_count
    return rd_tuning_count()


@pytest.mark.parametrize("variant", list(range(_n_variants())))
def test_sort_variants_match_oracle(rc, variant):
    import paper_2111_12478_amd as rd
    assert rd.rd_tuning_count() == _n_variants()
    rb, waves, items = rd.rd_tuning_get(variant)
    _say(f"variant {variant}: {rb}-bit digits, {waves} waves x {items} items")
    assert rd.rd_set_tuning(rc.ctx, variant) == 0
    try:
        cases = [tracegen.random_trace(s, max_blocks=6, max_tpb=40, max_events=6000) for s in range(7000, 7012)]
        g, ev, _, _ = tracegen.generate(tracegen.large(seed=2, scale=32))
        cases.append((g, ev))
        cfg = tracegen.stencil_small(seed=variant, rb=8, cb=8, tpb=64, rows=4, sweeps=3, plant_rate=0.05)
        g, ev, _, _ = tracegen.generate_stencil(cfg)
        cases.append((g, ev))
        for j, (g, ev) in enumerate(cases):
            want = oracle.check(g, ev)
            got = rc.check(g, ev)
            assert got.status == want.status == 0, (variant, j, got, want)
            np.testing.assert_array_equal(got.pairs, want.pairs, err_msg=f"variant {variant} case {j}")
    finally:
        rd.rd_set_tuning(rc.ctx, 0)


def test_autotune_picks_a_variant_and_keeps_results(rc):
    import torch
    import paper_2111_12478_amd as rd
    g, ev, _, _ = tracegen.generate(tracegen.large(seed=2, scale=16))
    want = oracle.check(g, ev)
    tr, ws, keep = rc.prepare(g, ev)
    try:
        st, best, ms = rd.rd_autotune(rc.ctx, [tr], None, 0, torch.cuda.current_stream().cuda_stream)
        assert st == 0 and 0 <= best < rd.rd_tuning_count() and all(m > 0 for m in ms), (st, best, ms)
        assert rd.rd_get_tuning(rc.ctx) == best
        got = rc.report(tr)
        np.testing.assert_array_equal(got.pairs, want.pairs)
    finally:
        rd.rd_trace_free(rc.ctx, tr)
        rd.rd_set_tuning(rc.ctx, 0)
