"""The lockset pass on the GPU (rd_lockset, through the C ABI) against the lockset oracle, pair by
pair: the golden traces, random lock traces (explicit and fence-inferred locks, nested sections,
block and device scopes, flag publications, barriers), random traces with every event kind,
stencil traces with their device lock, traces without locks; the limits and the report left
behind."""
import numpy as np
import pytest

import oracle
import tracegen
from golden_io import all_cases
from tracegen.format import KIND, make_meta
from tracegen.locktrace import lock_trace

pytestmark = pytest.mark.gpu

CASES = all_cases()


@pytest.fixture(scope="module")
def rc():
    from paper_2111_12478_amd import RaceChecker
    c = RaceChecker(0)
    yield c
    c.close()


def _lockset(rc, grid, ev, limits=None):
    from paper_2111_12478_amd import rd_trace_free
    tr, ws, keep = rc.prepare(grid, ev, limits)
    try:
        return rc.lockset(tr), rc.report(tr)
    finally:
        rd_trace_free(rc.ctx, tr)


def _same(rc, grid, ev, what):
    want = oracle.lockset(grid, ev)
    got, _ = _lockset(rc, grid, ev)
    assert got.status == want.status, (what, got, want)
    if want.status == 0:
        np.testing.assert_array_equal(got.pairs, want.pairs, err_msg=what)
    else:
        assert got.bad_index == want.bad_index, what
    return got


@pytest.mark.parametrize("case", CASES, ids=[c.name for c in CASES])
def test_golden(rc, case):
    got, _ = _lockset(rc, case.grid, case.events)
    assert got.status == 0, got
    np.testing.assert_array_equal(got.pairs, case.by_reading["lockset"])


@pytest.mark.parametrize("seed", range(150))
def test_lock_traces(rc, seed):
    opts = dict(barriers=bool(seed % 3 == 1), flags=bool(seed % 2), inferred=bool(seed % 5 != 0))
    grid, ev = lock_trace(seed, max_blocks=4, max_tpb=6, max_events=400, **opts)
    _same(rc, grid, ev, f"lock trace {seed} {opts}")


@pytest.mark.parametrize("seed", range(20))
def test_lock_traces_larger(rc, seed):
    grid, ev = lock_trace(10_000 + seed, max_blocks=8, max_tpb=32, max_events=20_000, flags=True,
                          barriers=bool(seed % 2))
    got = _same(rc, grid, ev, f"larger lock trace {seed}")
    print(f"larger lock trace {seed}: {len(ev)} events, {len(got.pairs)} pairs", flush=True)


@pytest.mark.parametrize("seed", range(60))
def test_random_traces_every_kind(rc, seed):
    grid, ev = tracegen.random_trace(seed)
    _same(rc, grid, ev, f"random trace {seed}")


@pytest.mark.parametrize("seed", [1, 2])
def test_stencil_traces(rc, seed):
    cfg = tracegen.stencil_small(seed=seed, rb=4, cb=4, tpb=32, rows=3, sweeps=3, plant_rate=0.05)
    grid, ev, _, _ = tracegen.generate_stencil(cfg)
    got = _same(rc, grid, ev, f"stencil {seed}")
    print(f"stencil {seed}: {len(ev)} events, {len(got.pairs)} lockset pairs", flush=True)


def test_no_locks_no_pairs_and_the_report_stays(rc):
    grid, ev, _, _ = tracegen.generate(tracegen.large(seed=2, scale=64))
    got, rep = _lockset(rc, grid, ev)
    assert got.status == 0 and len(got.pairs) == 0
    # the trace's report afterwards is its happens-before report
    want = oracle.check(grid, ev)
    assert rep.status == 0
    np.testing.assert_array_equal(rep.pairs, want.pairs)


def test_invalid_trace(rc):
    grid, ev = lock_trace(3, max_events=100)
    bad = ev.copy()
    bad[len(bad) // 2, 2] = 0x80
    _same(rc, grid, bad, "invalid")


@pytest.mark.parametrize("depth", [8, 64, 65])
def test_nested_locks(rc, depth):
    # one thread holds `depth` locks at once; both sides keep 64 and refuse more with RD_ENOMEM
    m = make_meta
    ev = [(300 + k, 0, m(KIND["ACQ"], 1), 0) for k in range(depth)]
    ev += [(100, 0, m(KIND["W"]), 0), (100, 1, m(KIND["W"]), 0)]
    ev += [(300 + k, 0, m(KIND["REL"], 1), 0) for k in reversed(range(depth))]
    ev = np.array(ev, dtype=np.uint32)
    got = _same(rc, (1, 2), ev, f"{depth} locks")
    assert got.status == (0 if depth <= 64 else -2)


def test_pool_too_small(rc):
    grid, ev = lock_trace(5, max_events=200)
    got, _ = _lockset(rc, grid, ev, limits={"clock_bytes": 1 << 20})
    assert got.status == -2, got


def test_small_capacity_runs_again(rc):
    # the binding's buffer holds fewer pairs than the pass finds: RD_ETRUNC, then one more pass with
    # room for all of them; and the C call itself with a short buffer writes the first pairs
    from paper_2111_12478_amd import rd_lockset, rd_trace_free, RD_ETRUNC
    for seed in range(40):
        grid, ev = lock_trace(seed, max_blocks=4, max_tpb=6, max_events=400, flags=True)
        want = oracle.lockset(grid, ev)
        if want.status == 0 and len(want.pairs) >= 3:
            break
    else:
        pytest.skip("no seed with three lockset pairs")
    tr, ws, keep = rc.prepare(grid, ev)
    try:
        got = rc.lockset(tr, capacity=1)
        assert got.status == 0, got
        np.testing.assert_array_equal(got.pairs, want.pairs)
        out = np.zeros((2, 2), np.uint32)
        st, n = rd_lockset(rc.ctx, tr, out.ctypes.data, 2)
        assert st == RD_ETRUNC and n == len(want.pairs)
        np.testing.assert_array_equal(out, want.pairs[:2])
    finally:
        rd_trace_free(rc.ctx, tr)
