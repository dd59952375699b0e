"""The GWCP pass on the GPU (rd_gwcp, through the C ABI) against the GWCP oracle (Algorithms 1 and 2
of Section 4.1), pair by pair: the golden traces with a GWCP expectation, random lock traces
(explicit and fence-inferred locks, nested sections, block and device scopes, flag publications,
barriers), random traces with every event kind (warp barriers included), stencil traces with their
device lock, traces without locks; every happens-before race is a GWCP race where critical sections
exclude each other; the limits and the report left behind."""
import numpy as np
import pytest

import oracle
import tracegen
from golden_io import all_cases
from tracegen.format import KIND, make_meta
from tracegen.locktrace import lock_trace

pytestmark = pytest.mark.gpu

GW = [c for c in all_cases() if "gwcp" in c.by_reading]
ALL = all_cases()


@pytest.fixture(scope="module")
def rc():
    from paper_2111_12478_amd import RaceChecker
    c = RaceChecker(0)
    yield c
    c.close()


def _gwcp(rc, grid, ev, limits=None):
    from paper_2111_12478_amd import rd_trace_free
    tr, ws, keep = rc.prepare(grid, ev, limits)
    try:
        return rc.gwcp(tr), rc.report(tr)
    finally:
        rd_trace_free(rc.ctx, tr)


def _same(rc, grid, ev, what):
    want = oracle.gwcp(grid, ev)
    got, _ = _gwcp(rc, grid, ev)
    assert got.status == want.status, (what, got, want)
    if want.status == 0:
        np.testing.assert_array_equal(got.pairs, want.pairs, err_msg=what)
    else:
        assert got.bad_index == want.bad_index, what
    return got


@pytest.mark.parametrize("case", GW, ids=[c.name for c in GW])
def test_golden(rc, case):
    got, _ = _gwcp(rc, case.grid, case.events)
    assert got.status == 0, got
    np.testing.assert_array_equal(got.pairs, case.by_reading["gwcp"])


@pytest.mark.parametrize("case", ALL, ids=[c.name for c in ALL])
def test_golden_traces_against_the_oracle(rc, case):
    _same(rc, case.grid, case.events, case.name)


@pytest.mark.parametrize("seed", range(120))
def test_lock_traces(rc, seed):
    opts = dict(barriers=bool(seed % 3 == 1), flags=bool(seed % 2), inferred=bool(seed % 5 != 0))
    grid, ev = lock_trace(seed, max_blocks=4, max_tpb=6, max_events=400, **opts)
    got = _same(rc, grid, ev, f"lock trace {seed} {opts}")
    if not opts["flags"]:
        # critical sections exclude each other (a flag acquire is never released, so with flags it
        # opens a section that others enter): every happens-before race is a GWCP race
        hb = oracle.check(grid, ev)
        assert {tuple(p) for p in hb.pairs.tolist()} <= {tuple(p) for p in got.pairs.tolist()}


@pytest.mark.parametrize("seed", range(8))
def test_lock_traces_larger(rc, seed):
    grid, ev = lock_trace(10_000 + seed, max_blocks=8, max_tpb=32, max_events=8_000, flags=True,
                          barriers=bool(seed % 2))
    got = _same(rc, grid, ev, f"larger lock trace {seed}")
    print(f"larger lock trace {seed}: {len(ev)} events, {len(got.pairs)} GWCP pairs", flush=True)


@pytest.mark.parametrize("seed", range(60))
def test_random_traces_every_kind(rc, seed):
    grid, ev = tracegen.random_trace(seed)
    _same(rc, grid, ev, f"random trace {seed}")


@pytest.mark.parametrize("seed", [1, 2])
def test_stencil_traces(rc, seed):
    cfg = tracegen.stencil_small(seed=seed, rb=4, cb=4, tpb=32, rows=3, sweeps=3, plant_rate=0.05)
    grid, ev, _, _ = tracegen.generate_stencil(cfg)
    got = _same(rc, grid, ev, f"stencil {seed}")
    print(f"stencil {seed}: {len(ev)} events, {len(got.pairs)} GWCP pairs", flush=True)


def test_no_locks_equals_happens_before_and_the_report_stays(rc):
    grid, ev, _, _ = tracegen.generate(tracegen.large(seed=2, scale=256))
    assert grid[0] * grid[1] <= 4096
    got, rep = _gwcp(rc, grid, ev)
    want = oracle.check(grid, ev)
    assert got.status == 0, got
    np.testing.assert_array_equal(got.pairs, oracle.gwcp(grid, ev).pairs)
    # the trace's report afterwards is its happens-before report
    assert rep.status == 0
    np.testing.assert_array_equal(rep.pairs, want.pairs)


def test_invalid_trace(rc):
    grid, ev = lock_trace(3, max_events=100)
    bad = ev.copy()
    bad[len(bad) // 2, 2] = 0x80
    _same(rc, grid, bad, "invalid")


@pytest.mark.parametrize("depth", [8, 64, 65])
def test_nested_locks(rc, depth):
    # one thread holds `depth` locks at once; the pass keeps 64 and refuses more with RD_ENOMEM
    m = make_meta
    ev = [(300 + k, 0, m(KIND["ACQ"], 1), 0) for k in range(depth)]
    ev += [(100, 0, m(KIND["W"]), 0), (100, 1, m(KIND["W"]), 0)]
    ev += [(300 + k, 0, m(KIND["REL"], 1), 0) for k in reversed(range(depth))]
    ev = np.array(ev, dtype=np.uint32)
    got, _ = _gwcp(rc, (1, 2), ev)
    if depth <= 64:
        want = oracle.gwcp((1, 2), ev)
        assert got.status == 0
        np.testing.assert_array_equal(got.pairs, want.pairs)
    else:
        assert got.status == -2, got


def test_too_many_threads(rc):
    # dense clocks: at most 4096 threads
    ev = np.array([(100, 0, make_meta(KIND["W"]), 0), (100, 4100, make_meta(KIND["W"]), 0)], dtype=np.uint32)
    got, _ = _gwcp(rc, (8, 1024), ev)
    assert got.status == -1, got


def test_pool_too_small(rc):
    grid, ev = lock_trace(5, max_events=200)
    got, _ = _gwcp(rc, grid, ev, limits={"clock_bytes": 1 << 16})
    assert got.status == -2, got


@pytest.mark.parametrize("seed", range(3))
def test_wide_lock_traces(rc, seed):
    # 2,048 threads, 32 lock words, 4,096 data words: long lock queues, many pairs
    grid, ev = lock_trace(500 + seed, max_events=30_000, flags=bool(seed % 2), barriers=True, grid=(8, 256),
                          locks=32, data_words=4096)
    got = _same(rc, grid, ev, f"wide lock trace {seed}")
    print(f"wide lock trace {seed}: {len(ev)} events, {len(got.pairs)} GWCP pairs", flush=True)
