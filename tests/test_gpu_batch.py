"""Batched form (rd_check_many): every member's report equals the oracle's, and the plain
checker's, for the same trace -- pairs, status and first offending index."""
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


def _assert_same(got, want, what):
    assert got.status == want.status, (what, got, want)
    if want.status == 0:
        np.testing.assert_array_equal(got.pairs, want.pairs, err_msg=what)
    elif want.status == -3:
        assert got.bad_index == want.bad_index, (what, got.bad_index, want.bad_index)


def _mix_items(seed, n_traces, scale):
    items = []
    for c in tracegen.batch(seed=seed, n_traces=n_traces, scale=scale):
        g, ev, _, _ = tracegen.generate(c)
        items.append((g, ev))
    return items


@pytest.mark.parametrize("seed", [4, 40, 41])
def test_batch_of_mixed_traces(rc, seed):
    items = _mix_items(seed, 14, 16)
    _say(f"batch seed {seed}: {len(items)} traces, {sum(len(e) for _, e in items)} events")
    got = rc.check_many(items)
    assert len(got) == len(items)
    for j, ((g, ev), r) in enumerate(zip(items, got)):
        want = oracle.check(g, ev)
        _assert_same(r, want, f"seed {seed} member {j}")


def test_batch_equals_plain(rc):
    items = _mix_items(7, 10, 8)
    _say("batch vs plain")
    got = rc.check_many(items)
    for j, ((g, ev), r) in enumerate(zip(items, got)):
        plain = rc.check(g, ev)
        _assert_same(r, plain, f"member {j}")


def test_batch_of_random_traces_one_warp_size(rc):
    # random traces with every kind of event, grouped by warp size so that they merge
    by_ws = {}
    for seed in range(3000, 3400):
        g, ev = tracegen.random_trace(seed, max_blocks=4, max_tpb=12, max_events=800)
        by_ws.setdefault(g[2], []).append((g, ev))
    for ws, items in sorted(by_ws.items()):
        _say(f"random batch warp size {ws}: {len(items)} traces")
        got = rc.check_many(items)
        for j, ((g, ev), r) in enumerate(zip(items, got)):
            want = oracle.check(g, ev)
            _assert_same(r, want, f"ws {ws} member {j}")


def test_batch_with_invalid_members(rc):
    # malformed members fall back to their own check: same status and first offending index
    groups = {}
    for name, grid, ev, status, bad in INVALID_CASES:
        g = tuple(grid) if len(grid) == 3 else tuple(grid) + (32,)
        groups.setdefault(g[2], []).append((g, ev))
    for ws, bad_items in sorted(groups.items()):
        items = (_mix_items(9, 3, 32) if ws == 32 else []) + bad_items + (_mix_items(10, 2, 32) if ws == 32 else [])
        _say(f"batch with {len(bad_items)} malformed members, warp size {ws}")
        got = rc.check_many(items)
        for j, ((g, ev), r) in enumerate(zip(items, got)):
            want = oracle.check(g, ev)
            _assert_same(r, want, f"ws {ws} member {j}")


def test_batch_mixed_warp_sizes_checked_one_by_one(rc):
    items = []
    for seed in range(3500, 3530):
        items.append(tracegen.random_trace(seed, max_blocks=3, max_tpb=8, max_events=300))
    assert len({g[2] for g, _ in items}) > 1
    got = rc.check_many(items)
    for j, ((g, ev), r) in enumerate(zip(items, got)):
        _assert_same(r, oracle.check(g, ev), f"member {j}")


def test_batch_empty_and_single_members(rc):
    items = [((2, 64, 32), np.zeros((0, 4), np.uint32))] + _mix_items(11, 2, 32) + \
            [((1, 32, 32), np.zeros((0, 4), np.uint32))]
    got = rc.check_many(items)
    for j, ((g, ev), r) in enumerate(zip(items, got)):
        _assert_same(r, oracle.check(g, ev), f"member {j}")
    one = _mix_items(12, 1, 16)
    got = rc.check_many(one)
    _assert_same(got[0], oracle.check(*one[0]), "single")


def test_batch_member_over_its_pair_limit(rc):
    # a member whose pairs exceed its own max_pairs reports what the plain check reports
    from paper_2111_12478_amd import RD_ENOMEM
    items = _mix_items(13, 4, 8)
    want = [oracle.check(g, ev) for g, ev in items]
    k = int(np.argmax([len(w.pairs) for w in want]))
    assert len(want[k].pairs) > 2
    plain = rc.check(*items[k], limits={"max_pairs": 2})
    assert plain.status == RD_ENOMEM
    got = rc.check_many(items, limits={"max_pairs": 2})
    for j, r in enumerate(got):
        if len(want[j].pairs) > 2:
            assert r.status == RD_ENOMEM, (j, r)
        else:
            _assert_same(r, want[j], f"member {j}")


def test_batch_repeated(rc):
    items = _mix_items(14, 6, 16)
    a = rc.check_many(items)
    b = rc.check_many(items)
    for j, (x, y) in enumerate(zip(a, b)):
        _assert_same(x, y, f"member {j}")


def test_batch_graph_replays(rc):
    # one captured batched pass, replayed: first on traces A, then with B's events written in place
    # (same sizes), with eager checks and synchronisation between the replays
    import dataclasses
    import torch
    import paper_2111_12478_amd as rd
    cfgs = tracegen.batch(seed=15, n_traces=6, scale=16)
    a_items, b_items = [], []
    for c in cfgs:
        g, ev, _, _ = tracegen.generate(c)
        a_items.append((g, ev))
        g2, ev2, _, _ = tracegen.generate(dataclasses.replace(c, seed=c.seed + 1000))
        assert ev2.shape == ev.shape
        b_items.append((g2, ev2))
    dev = [torch.from_numpy(ev.view(np.int32)).cuda() for _, ev in a_items]
    bound = [rc.prepare(g, d) for (g, _), d in zip(a_items, dev)]
    traces = [b[0] for b in bound]
    stream = torch.cuda.Stream()
    try:
        nbytes = rd.rd_batch_workspace_bytes(rc.ctx, traces, None)
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        with torch.cuda.stream(stream):
            st, graph = rd.rd_batch_capture(rc.ctx, traces, ws.data_ptr(), nbytes, None, stream.cuda_stream)
            assert st == 0, rd.rd_last_error(rc.ctx)
            try:
                for rep, items in enumerate([a_items, a_items, b_items, b_items, a_items]):
                    for d, (_, ev) in zip(dev, items):
                        d.copy_(torch.from_numpy(ev.view(np.int32)))
                    stream.synchronize()
                    assert rd.rd_graph_launch(rc.ctx, graph, stream.cuda_stream) == 0
                    got = rc.report_many(traces)
                    for j, ((g, ev), r) in enumerate(zip(items, got)):
                        _assert_same(r, oracle.check(g, ev), f"replay {rep} member {j}")
                    # eager work between replays
                    other = rc.check(*b_items[0])
                    _assert_same(other, oracle.check(*b_items[0]), "eager")
                    torch.cuda.synchronize()
            finally:
                rd.rd_graph_free(rc.ctx, graph)
    finally:
        for t in traces:
            rd.rd_trace_free(rc.ctx, t)
