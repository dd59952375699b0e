"""Served form (rd_server_*): continuous batching under an HBM budget.  Every request's answer --
pairs, status, first offending index -- equals the oracle's for the same trace checked alone,
whatever else was in flight with it."""
import threading

import numpy as np
import pytest

import oracle
import tracegen
from test_oracle_validation import CASES as INVALID_CASES

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rc():
    from paper_2111_12478_amd import RaceChecker
    c = RaceChecker(0)
    yield c
    c.close()


def _say(msg):
    print(msg, flush=True)


def _requests(seed, n_mix, scale):
    items = []
    for c in tracegen.batch(seed=seed, n_traces=n_mix, scale=scale):
        g, ev, _, _ = tracegen.generate(c)
        items.append((g, ev))
    for s in range(seed * 100, seed * 100 + 30):
        g, ev = tracegen.random_trace(s, max_blocks=4, max_tpb=12, max_events=600)
        items.append((g, ev))  # random warp sizes: these cannot all share a pass
    for name, grid, ev, status, bad in INVALID_CASES:
        items.append((tuple(grid) if len(grid) == 3 else tuple(grid) + (32,), ev))
    rng = np.random.default_rng(seed)
    return [items[j] for j in rng.permutation(len(items))]


def _check_all(items, got):
    for j, ((g, ev), (r, info)) in enumerate(zip(items, got)):
        want = oracle.check(g, ev)
        assert r.status == want.status, (j, r, want)
        if want.status == 0:
            np.testing.assert_array_equal(r.pairs, want.pairs, err_msg=f"request {j}")
            assert info.n_races == len(want.pairs)
        elif want.status == -3:
            assert r.bad_index == want.bad_index, (j, r.bad_index, want.bad_index)
        assert info.submit_s <= info.start_s <= info.done_s


@pytest.mark.parametrize("inflight", [1, 2, 3])
def test_served_alone_equals_mix(rc, inflight):
    from paper_2111_12478_amd import Server
    items = _requests(5, 12, 16)
    _say(f"served: {len(items)} requests, {inflight} in flight")
    srv = Server(rc, 2 << 30, max_batch=16, max_inflight=inflight)
    try:
        tickets = [srv.submit(g, ev) for g, ev in items]
        got = [srv.wait(t) for t in tickets]
        passes, done = srv.stats()
        assert done == len(items)
        assert passes < len(items)  # requests shared passes
    finally:
        srv.close()
    _check_all(items, got)


def test_served_small_budget_admits_as_memory_returns(rc):
    from paper_2111_12478_amd import Server, RaceChecker
    items = _requests(6, 16, 8)
    # room for roughly one of the larger requests at a time
    biggest = max(len(ev) for _, ev in items)
    budget = rc.workspace_bytes((2048, 256, 32), biggest) + 64 * biggest + (64 << 20)
    _say(f"served: budget {budget >> 20} MiB for {len(items)} requests")
    srv = Server(rc, budget, max_batch=64, max_inflight=2)
    try:
        tickets = [srv.submit(g, ev) for g, ev in items]
        got = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    _check_all(items, got)


def test_served_request_larger_than_budget(rc):
    from paper_2111_12478_amd import Server, RD_ENOMEM
    g, ev, _, _ = tracegen.generate(tracegen.batch(seed=7, n_traces=1, scale=1)[0])
    srv = Server(rc, 1 << 20, max_inflight=1)
    try:
        t_big = srv.submit(g, ev)
        r, info = srv.wait(t_big)
        assert r.status == RD_ENOMEM
    finally:
        srv.close()


def test_served_concurrent_submitters(rc):
    from paper_2111_12478_amd import Server
    items = _requests(9, 12, 16)
    srv = Server(rc, 2 << 30, max_batch=8, max_inflight=2)
    got = [None] * len(items)

    def run(part):
        for j in part:
            t = srv.submit(*items[j])
            got[j] = srv.wait(t)

    try:
        threads = [threading.Thread(target=run, args=(list(range(k, len(items), 4)),)) for k in range(4)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
    finally:
        srv.close()
    _check_all(items, got)
