"""Unique race kinds (rd_race_kinds) against the oracle's definition, through the C ABI.

A kind is the unordered pair of the two racing accesses' site ids (aux words), counted over the
race pairs (Table 2, Section 6).  The traces' aux words are rewritten with seeded site ids of
several spreads; expected kinds come from the oracle's pairs, never from the GPU's."""
import numpy as np
import pytest

import oracle
import tracegen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rc():
    from paper_2111_12478_amd import RaceChecker
    r = RaceChecker(0)
    yield r
    r.close()


def _with_sites(ev, seed, spread):
    # site ids on the accesses only (a warp barrier's aux word is its lane mask)
    ev = np.array(ev, dtype=np.uint32)
    rng = np.random.default_rng(seed)
    if spread == "distinct":
        site = np.arange(ev.shape[0], dtype=np.uint32) * 7 + 3
    elif spread == "one":
        site = np.full(ev.shape[0], 0xdeadbeef, dtype=np.uint32)
    elif spread == "wide":
        site = rng.integers(0, 1 << 32, ev.shape[0], dtype=np.uint64).astype(np.uint32)
    else:
        site = rng.integers(0, int(spread), ev.shape[0]).astype(np.uint32)
    access = np.isin(ev[:, 2] & 15, [0, 1, 2, 6, 7])
    ev[access, 3] = site[access]
    return ev


def _gpu_kinds(rc, grid, ev, capacity=None, report_first=True):
    from paper_2111_12478_amd import rd_check, rd_trace_free
    tr, ws, keep = rc.prepare(grid, ev)
    try:
        if report_first:
            got_pairs = rc.run(tr)
        else:
            import torch
            assert rd_check(rc.ctx, tr, torch.cuda.current_stream().cuda_stream) == 0
            got_pairs = None
        st, kinds = rc.kinds(tr, capacity)
        return st, kinds, got_pairs
    finally:
        rd_trace_free(rc.ctx, tr)


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("spread", ["distinct", "one", "wide", 5, 40])
def test_kinds_tiny_traces(rc, seed, spread):
    grid, ev, _, _ = tracegen.generate(tracegen.tiny(seed=100 + seed))
    ev = _with_sites(ev, seed, spread)
    want_pairs = oracle.check(grid, ev)
    assert want_pairs.status == 0
    want = oracle.race_kinds(ev, want_pairs.pairs)
    st, got, res = _gpu_kinds(rc, grid, ev)
    assert st == 0, (seed, spread)
    np.testing.assert_array_equal(res.pairs, want_pairs.pairs)
    np.testing.assert_array_equal(got, want, err_msg=f"seed {seed} spread {spread}")


@pytest.mark.parametrize("seed", range(6))
def test_kinds_random_traces(rc, seed):
    from tracegen.randtrace import random_trace
    grid, ev = random_trace(seed=4000 + seed, max_blocks=6, max_tpb=40, max_events=3000)
    ev = _with_sites(ev, seed, 9)
    want_pairs = oracle.check(grid, ev)
    assert want_pairs.status == 0
    want = oracle.race_kinds(ev, want_pairs.pairs)
    st, got, _ = _gpu_kinds(rc, grid, ev)
    assert st == 0
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("spread", [64, "wide"])
def test_kinds_scaled_large_trace(rc, spread):
    # 2M events, tens of thousands of pairs: the kind sort runs over many tiles
    grid, ev, _, _ = tracegen.generate(tracegen.large(scale=8))
    ev = _with_sites(ev, 77, spread)
    want_pairs = oracle.check(grid, ev)
    assert want_pairs.status == 0 and want_pairs.pairs.shape[0] > 4096
    want = oracle.race_kinds(ev, want_pairs.pairs)
    st, got, _ = _gpu_kinds(rc, grid, ev)
    assert st == 0
    np.testing.assert_array_equal(got, want)


def test_kinds_capacity_and_count_only(rc):
    grid, ev, _, _ = tracegen.generate(tracegen.tiny(seed=131))
    ev = _with_sites(ev, 3, 40)
    want = oracle.race_kinds(ev, oracle.check(grid, ev).pairs)
    assert want.shape[0] > 3
    st, got, _ = _gpu_kinds(rc, grid, ev, capacity=3)
    assert st == -4  # RD_ETRUNC
    np.testing.assert_array_equal(got, want[:3])
    st, got, _ = _gpu_kinds(rc, grid, ev, capacity=0)
    assert st == -4 and got.shape[0] == 0


def test_kinds_without_the_report_first(rc):
    grid, ev, _, _ = tracegen.generate(tracegen.tiny(seed=132))
    ev = _with_sites(ev, 4, 6)
    want = oracle.race_kinds(ev, oracle.check(grid, ev).pairs)
    st, got, _ = _gpu_kinds(rc, grid, ev, report_first=False)
    assert st == 0
    np.testing.assert_array_equal(got, want)


def test_kinds_of_a_race_free_trace(rc):
    grid, ev, _, _ = tracegen.generate(tracegen.tiny(seed=133))
    # keep only the first thread's events: nothing can race
    ev = ev[ev[:, 1] == ev[0, 1]]
    assert oracle.check(grid, ev).pairs.shape[0] == 0
    st, got, _ = _gpu_kinds(rc, grid, ev)
    assert st == 0 and got.shape == (0, 3)


def test_kinds_of_batch_members(rc):
    # members of a batched check are checked alone for their kinds; results equal the oracle's
    from paper_2111_12478_amd import (rd_batch_workspace_bytes, rd_check_many, rd_trace_free)
    import torch
    items = [tracegen.generate(tracegen.tiny(seed=140 + j))[:2] for j in range(3)]
    items = [(g, _with_sites(e, j, 7)) for j, (g, e) in enumerate(items)]
    bound = [rc.prepare(g, e) for g, e in items]
    traces = [b[0] for b in bound]
    try:
        nbytes = rd_batch_workspace_bytes(rc.ctx, traces, None)
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda:0")
        assert rd_check_many(rc.ctx, traces, ws.data_ptr(), ws.numel(), None,
                             torch.cuda.current_stream().cuda_stream) == 0
        for (g, e), t in zip(items, traces):
            want = oracle.race_kinds(e, oracle.check(g, e).pairs)
            st, got = rc.kinds(t)
            assert st == 0
            np.testing.assert_array_equal(got, want)
        torch.cuda.synchronize()
    finally:
        for t in traces:
            rd_trace_free(rc.ctx, t)
