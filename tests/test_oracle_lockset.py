"""Pins of the lockset oracle (oracle.lockset): the pass the paper describes for ScoRD (Section 2.2,
Section 3; after Eraser) against the paper's statements about it, hand-derived golden traces, a
closed form, and invariants that follow from the analysis (traces without locks report nothing; one
lock around every thread's whole program protects every pair)."""
import numpy as np
import pytest

import oracle
import tracegen
from golden_io import all_cases
from tracegen.format import KIND, make_meta
from tracegen.locktrace import lock_trace

LS = [c for c in all_cases() if "lockset" in c.by_reading]


def _set(p):
    return {(int(a), int(b)) for a, b in p}


def test_every_golden_case_states_the_lockset_report():
    assert len(LS) == len(all_cases())


@pytest.mark.parametrize("case", LS, ids=[c.name for c in LS])
def test_golden(case):
    r = oracle.lockset(case.grid, case.events)
    assert r.status == 0, r
    np.testing.assert_array_equal(r.pairs, case.by_reading["lockset"])


def test_paper_statements():
    by = {c.name: c for c in all_cases()}
    # Figure 3: the lockset at e6 holds l, the one at e1 is empty: reported
    assert _set(oracle.lockset(by["f03_hb_hides_wcp"].grid, by["f03_hb_hides_wcp"].events).pairs) == {(0, 5)}
    # Figure 4: both accesses unprotected: ScoRD skips the lockset analysis
    assert len(oracle.lockset(by["f04_fence_alone"].grid, by["f04_fence_alone"].events).pairs) == 0
    # Figure 5: e1 and e14 hold no lock, so ScoRD misses their race
    assert (0, 13) not in _set(oracle.lockset(by["f05_scoped_locks"].grid, by["f05_scoped_locks"].events).pairs)
    # one access protected, the other not: detected
    c = by["lockset_one_protected"]
    assert _set(oracle.lockset(c.grid, c.events).pairs) == {(0, 2)}


@pytest.mark.parametrize("T", [2, 3, 8, 33])
def test_closed_form_one_unprotected_writer(T):
    # thread 0 writes x with no lock, then threads 1..T-1 each write x inside a section on one
    # device lock: only the first protected write follows the unprotected one (one lockset pair);
    # happens-before orders none of thread 0's write with the others (T - 1 pairs)
    m = make_meta
    ev = [(100, 0, m(KIND["W"]), 0)]
    for t in range(1, T):
        ev += [(200, t, m(KIND["ACQ"], 1), 0), (100, t, m(KIND["W"]), 0), (200, t, m(KIND["REL"], 1), 0)]
    ev = np.array(ev, dtype=np.uint32)
    grid = (1, T)
    assert _set(oracle.lockset(grid, ev).pairs) == {(0, 2)}
    assert len(oracle.check(grid, ev).pairs) == T - 1


@pytest.mark.parametrize("seed", range(6))
def test_no_locks_no_report(seed):
    cfg = tracegen.large(seed=seed, scale=256)
    grid, ev, _, _ = tracegen.generate(cfg)
    kinds = ev[:, 2] & 15
    assert not np.isin(kinds, (KIND["ACQ"], KIND["REL"], KIND["F"])).any()
    r = oracle.lockset(grid, ev)
    assert r.status == 0 and len(r.pairs) == 0
    assert len(oracle.check(grid, ev).pairs) > 0  # racy by happens-before all the same


@pytest.mark.parametrize("seed", range(40))
def test_one_lock_around_every_program_protects_everything(seed):
    # a fresh device lock acquired as every thread's first event and released as its last: every
    # access then holds it, so every pair shares a lock (barrier-free traces, so the added events
    # keep the trace valid)
    grid, ev = lock_trace(seed, max_blocks=3, max_tpb=4, max_events=200)
    tids = np.unique(ev[:, 1])
    first = {int(t): int(np.nonzero(ev[:, 1] == t)[0][0]) for t in tids}
    last = {int(t): int(np.nonzero(ev[:, 1] == t)[0][-1]) for t in tids}
    out = []
    for i, e in enumerate(ev.tolist()):
        if first[e[1]] == i:
            out.append((999, e[1], make_meta(KIND["ACQ"], 1), 0))
        out.append(tuple(e))
        if last[e[1]] == i:
            out.append((999, e[1], make_meta(KIND["REL"], 1), 0))
    big = np.array(out, dtype=np.uint32)
    assert oracle.validate(grid, big).status == 0
    r = oracle.lockset(grid, big)
    assert r.status == 0 and len(r.pairs) == 0, r.pairs
    # and without that lock the same traces do report lockset pairs somewhere
    assert oracle.lockset(grid, ev).status == 0


def test_lockset_pairs_are_consecutive_conflicting_accesses():
    # every reported pair is two accesses of one location, different threads, one of them writing
    seen = 0
    for seed in range(60):
        grid, ev = lock_trace(seed, max_events=300, flags=True)
        r = oracle.lockset(grid, ev)
        assert r.status == 0
        for a, b in r.pairs.tolist():
            assert a < b and ev[a, 0] == ev[b, 0] and ev[a, 1] != ev[b, 1]
            assert (ev[a, 2] & 15) != KIND["R"] or (ev[b, 2] & 15) != KIND["R"]
            seen += 1
    assert seen > 0


def test_invalid_trace_same_index_as_the_checker():
    grid, ev = lock_trace(3, max_events=100)
    bad = ev.copy()
    bad[len(bad) // 2, 2] = 0x80
    assert oracle.lockset(grid, bad).status == -3
    assert oracle.lockset(grid, bad).bad_index == oracle.check(grid, bad).bad_index
