"""Pins of the GWCP oracle (Section 4): Algorithms 1-2 (oracle.gwcp) against the paper's worked
examples and hand-derived traces, against the definition's fixpoint (oracle.gwcp_bruteforce) on
random lock traces, and against invariants that follow from the definition."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from golden_io import all_cases
from tracegen.format import KIND
from tracegen.locktrace import lock_trace
from tracegen.randtrace import random_trace

GW = [c for c in all_cases() if "gwcp" in c.by_reading]


def _set(p):
    return {(int(a), int(b)) for a, b in p}


def _has_barrier(ev):
    k = ev[:, 2] & 15
    return bool(np.isin(k, (KIND["BAR"], KIND["WBAR"])).any())


@pytest.mark.parametrize("case", GW, ids=[c.name for c in GW])
def test_golden(case):
    want = case.by_reading["gwcp"]
    r = oracle.gwcp(case.grid, case.events)
    assert r.status == 0, r
    np.testing.assert_array_equal(r.pairs, want)
    b = oracle.gwcp_bruteforce(case.grid, case.events)
    assert b.status == 0
    if _has_barrier(case.events):
        assert _set(b.pairs) <= _set(want)  # the definition orders at least what the algorithm does
    else:
        np.testing.assert_array_equal(b.pairs, want)


def test_every_golden_case_states_gwcp():
    assert len(GW) == len(all_cases())


def test_paper_figures():
    by = {c.name: c for c in all_cases()}
    # Figure 3: HB orders e1 before e6, GWCP predicts the race
    f3 = by["f03_hb_hides_wcp"]
    assert len(oracle.check(f3.grid, f3.events).pairs) == 0
    assert _set(oracle.gwcp(f3.grid, f3.events).pairs) == {(0, 5)}
    # Figure 5: (e1, e14) is reported
    f5 = by["f05_scoped_locks"]
    assert (0, 13) in _set(oracle.gwcp(f5.grid, f5.events).pairs)


@settings(max_examples=250, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.integers(min_value=0, max_value=2**31 - 1), st.booleans())
def test_algorithm_equals_definition_on_lock_traces(seed, flags):
    # synchronisation by critical sections (and flag publications): the setting in which WCP's
    # vector-clock algorithm computes its relation exactly
    grid, ev = lock_trace(seed, flags=flags)
    a = oracle.gwcp(grid, ev)
    b = oracle.gwcp_bruteforce(grid, ev)
    assert a.status == b.status == 0
    np.testing.assert_array_equal(a.pairs, b.pairs, err_msg=f"seed={seed} flags={flags}")


@settings(max_examples=200, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.integers(min_value=0, max_value=2**31 - 1), st.booleans())
def test_algorithm_orders_no_more_than_definition_with_barriers(seed, flags):
    grid, ev = lock_trace(seed, barriers=True, flags=flags)
    a = oracle.gwcp(grid, ev)
    b = oracle.gwcp_bruteforce(grid, ev)
    assert a.status == b.status == 0
    assert _set(b.pairs) <= _set(a.pairs), (seed, sorted(_set(b.pairs) - _set(a.pairs))[:5])


@settings(max_examples=200, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.integers(min_value=0, max_value=2**31 - 1), st.booleans())
def test_gwcp_reports_every_hb_race(seed, barriers):
    # GWCP is weaker than happens-before on traces whose critical sections exclude each other:
    # every happens-before race is a GWCP race
    grid, ev = lock_trace(seed, barriers=barriers)
    h = oracle.check(grid, ev)
    g = oracle.gwcp(grid, ev)
    assert h.status == g.status == 0
    assert _set(h.pairs) <= _set(g.pairs)


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.integers(min_value=0, max_value=2**31 - 1))
def test_without_locks_gwcp_is_happens_before(seed):
    # with barriers as the only synchronisation, rule (iii) is happens-before's barrier rule
    grid, ev = random_trace(seed, wbar=True)
    k = ev[:, 2] & 15
    keep = ~np.isin(k, (KIND["ACQ"], KIND["REL"], KIND["F"]))
    ev = ev[keep]  # no lock event, and no fence, so no atomic is a lock operation
    h = oracle.check(grid, ev)
    if h.status != 0:
        return  # dropping events can break a warp barrier's discipline
    g = oracle.gwcp(grid, ev)
    b = oracle.gwcp_bruteforce(grid, ev)
    np.testing.assert_array_equal(g.pairs, h.pairs)
    np.testing.assert_array_equal(b.pairs, h.pairs)


def test_larger_lock_traces_are_consistent():
    # a few hundred threads: GWCP contains HB and the algorithm finishes
    for seed in range(5):
        grid, ev = lock_trace(seed + 900, max_blocks=8, max_tpb=32, max_events=20000)
        h = oracle.check(grid, ev)
        g = oracle.gwcp(grid, ev)
        assert h.status == g.status == 0
        assert _set(h.pairs) <= _set(g.pairs)


def test_rejects_malformed_traces_like_the_detector():
    grid, ev = lock_trace(3)
    bad = ev.copy()
    bad[min(5, len(bad) - 1), 2] |= 0x100
    assert oracle.gwcp(grid, bad).status == -3
    assert oracle.gwcp(grid, bad).bad_index == oracle.check(grid, bad).bad_index
