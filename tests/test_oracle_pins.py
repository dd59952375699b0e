"""Pins of the oracle against things other than itself: brute-force closure on random valid
traces with every event kind, closed-form pair counts, invariants of the race definition, and
the two clock stores against each other."""
from itertools import combinations

import numpy as np
import pytest
from hypothesis import given, settings, HealthCheck
from hypothesis import strategies as st

import oracle
from tracegen.format import KIND, make_meta
from tracegen.randtrace import random_trace

W, R, A, F, BAR, ACQ, REL = (KIND[k] for k in ("W", "R", "A", "F", "BAR", "ACQ", "REL"))


def _pairs_set(p):
    return {(int(a), int(b)) for a, b in p}


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.integers(min_value=0, max_value=2**31 - 1))
def test_vector_clocks_equal_bruteforce_on_random_traces(seed):
    grid, ev = random_trace(seed)
    bf = oracle.bruteforce(grid, ev)
    assert bf.status == 0, (seed, bf)
    for dense in (False, True):
        vc = oracle.check(grid, ev, dense=dense)
        assert vc.status == 0, (seed, dense, vc)
        np.testing.assert_array_equal(vc.pairs, bf.pairs, err_msg=f"seed={seed} dense={dense}")


@settings(max_examples=60, deadline=None)
@given(st.integers(min_value=0, max_value=2**31 - 1))
def test_inclusive_reading_agrees_between_bruteforce_and_clocks(seed):
    grid, ev = random_trace(seed)
    bf = oracle.bruteforce(grid, ev, inclusive=True)
    vc = oracle.check(grid, ev, dense=False, inclusive=True)
    assert bf.status == 0 and vc.status == 0
    np.testing.assert_array_equal(vc.pairs, bf.pairs)


@settings(max_examples=40, deadline=None)
@given(st.integers(min_value=0, max_value=2**31 - 1))
def test_larger_random_traces_clock_stores_agree(seed):
    grid, ev = random_trace(seed, max_blocks=6, max_tpb=16, max_events=3000)
    a = oracle.check(grid, ev, dense=False)
    b = oracle.check(grid, ev, dense=True)
    assert a.status == 0 and b.status == 0
    np.testing.assert_array_equal(a.pairs, b.pairs)


@pytest.mark.parametrize("T", [1, 2, 5, 32, 64])
def test_intrawarp_closed_form(T):
    # Figure 2 "intrawarp": T threads of one block each write data[0]: C(T,2) racing pairs
    ev = np.array([(7, t, make_meta(W), 0) for t in range(T)], dtype=np.uint32)
    r = oracle.check((1, T), ev)
    assert r.status == 0 and len(r.pairs) == T * (T - 1) // 2
    assert _pairs_set(r.pairs) == set(combinations(range(T), 2))


@pytest.mark.parametrize("B,T", [(1, 4), (2, 3), (3, 2), (4, 8)])
def test_interblock_scope_closed_form(B, T):
    # Figure 2 "interblk_scope": block-scoped atomics race across blocks: T^2 * B(B-1)/2 pairs;
    # device-scoped ones never race (Section 5.1)
    for scope, expect in ((0, T * T * B * (B - 1) // 2), (1, 0), (2, 0)):
        ev = np.array([(7, t, make_meta(A, scope), 0) for t in range(B * T)], dtype=np.uint32)
        r = oracle.check((B, T), ev)
        bf = oracle.bruteforce((B, T), ev)
        assert r.status == 0 and len(r.pairs) == expect
        np.testing.assert_array_equal(r.pairs, bf.pairs)


def _conflict(e1, e2, tpb):
    k1, k2 = e1[2] & 15, e2[2] & 15
    acc = (0, 1, 2, 6, 7)
    if k1 not in acc or k2 not in acc or e1[1] == e2[1]:
        return False
    sp1, sp2 = (e1[2] >> 6) & 1, (e2[2] >> 6) & 1
    if sp1 != sp2 or e1[0] != e2[0]:
        return False
    if sp1 == 1 and e1[1] // tpb != e2[1] // tpb:
        return False
    wr = lambda k: k in (1, 2, 6, 7)
    at = lambda k: k in (2, 6, 7)
    if not (wr(k1) or wr(k2)):
        return False
    if at(k1) and at(k2):
        s1, s2 = (e1[2] >> 4) & 3, (e2[2] >> 4) & 3
        if s1 != 0 or s2 != 0 or e1[1] // tpb == e2[1] // tpb:
            return False
    return True


@settings(max_examples=80, deadline=None)
@given(st.integers(min_value=0, max_value=2**31 - 1))
def test_no_sync_reports_every_conflicting_pair(seed):
    # Invariant I1: with no synchronisation at all, every conflicting cross-thread pair races
    rng = np.random.default_rng(seed)
    nb, tpb = int(rng.integers(1, 4)), int(rng.integers(1, 5))
    n = int(rng.integers(0, 60))
    ev = np.zeros((n, 4), dtype=np.uint32)
    for i in range(n):
        k = int(rng.choice([0, 1, 2]))
        ev[i] = (int(rng.integers(0, 4)), int(rng.integers(0, nb * tpb)),
                 make_meta(k, int(rng.integers(0, 3)), int(rng.integers(0, 2))), 0)
    r = oracle.check((nb, tpb), ev)
    assert r.status == 0
    want = {(i, j) for i in range(n) for j in range(i + 1, n) if _conflict(ev[i], ev[j], tpb)}
    assert _pairs_set(r.pairs) == want


@settings(max_examples=80, deadline=None)
@given(st.integers(min_value=0, max_value=2**31 - 1))
def test_barrier_only_traces_follow_the_phase_rule(seed):
    # Invariant I3: with block barriers as the only synchronisation, a conflicting pair races iff
    # the threads are in different blocks or passed the same number of barriers
    rng = np.random.default_rng(seed)
    nb, tpb = int(rng.integers(1, 4)), int(rng.integers(1, 5))
    n_ph = int(rng.integers(1, 4))
    progs = []
    for t in range(nb * tpb):
        p = []
        for ph in range(n_ph):
            for _ in range(int(rng.integers(0, 4))):
                p.append((int(rng.integers(0, 4)), t, make_meta(int(rng.choice([0, 1, 2])),
                          int(rng.integers(0, 3)), int(rng.integers(0, 2))), 0))
            if ph + 1 < n_ph:
                p.append((0, t, make_meta(BAR), 0))
        progs.append(p or [(0, t, make_meta(R), 0)])
    # phase-synchronous random interleave (valid by construction)
    ev, phase = [], []
    for ph in range(n_ph):
        chunks = []
        for t in range(nb * tpb):
            bars = [i for i, e in enumerate(progs[t]) if (e[2] & 15) == BAR]
            lo = 0 if ph == 0 else bars[ph - 1] + 1
            hi = bars[ph] + 1 if ph < len(bars) else len(progs[t])
            chunks.append(list(progs[t][lo:hi]))
        while any(chunks):
            t = int(rng.choice([i for i, c in enumerate(chunks) if c]))
            e = chunks[t].pop(0)
            ev.append(e)
            phase.append(ph if (e[2] & 15) != BAR else -1)
    ev = np.array(ev, dtype=np.uint32).reshape(-1, 4)
    r = oracle.check((nb, tpb), ev)
    assert r.status == 0, r
    n = len(ev)
    want = {(i, j) for i in range(n) for j in range(i + 1, n)
            if _conflict(ev[i], ev[j], tpb)
            and (ev[i][1] // tpb != ev[j][1] // tpb or phase[i] == phase[j])}
    assert _pairs_set(r.pairs) == want


@settings(max_examples=80, deadline=None)
@given(st.integers(min_value=0, max_value=2**31 - 1))
def test_removing_synchronisation_never_removes_races(seed):
    # Invariant I2: replacing every fence by an unrelated private read (so no atomic is inferred as
    # a release or acquire) only drops happens-before edges, so the race set can only grow
    grid, ev = random_trace(seed)
    ev2 = ev.copy()
    for i in range(len(ev2)):
        if (ev2[i][2] & 15) == F:
            ev2[i] = (1_000_000 + ev2[i][1], ev2[i][1], make_meta(R), 0)
    a = oracle.check(grid, ev)
    b = oracle.check(grid, ev2)
    assert a.status == 0 and b.status == 0
    assert _pairs_set(a.pairs) <= _pairs_set(b.pairs)


def test_canonical_order():
    grid, ev = random_trace(12345, max_events=800)
    r = oracle.check(grid, ev)
    p = r.pairs.astype(np.int64)
    assert np.all(p[:, 0] < p[:, 1])
    keys = p[:, 0] * (1 << 32) + p[:, 1]
    assert np.all(np.diff(keys) > 0)
