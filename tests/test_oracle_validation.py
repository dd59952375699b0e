"""Trace validation of the oracle on hand-made malformed traces (first offending index)."""
import numpy as np
import pytest

import oracle
from tracegen.format import KIND, make_meta

R, W, F, BAR, WBAR = (KIND[k] for k in ("R", "W", "F", "BAR", "WBAR"))


def ev(*rows):
    return np.array(rows, dtype=np.uint32).reshape(-1, 4)


CASES = [
    # (name, grid, events, status, first bad index)
    ("ok_empty", (1, 2), ev(), 0, -1),
    ("reserved_meta_bit", (1, 2), ev((1, 0, make_meta(R), 0), (1, 1, make_meta(R) | 0x80, 0)), -3, 1),
    ("kind_out_of_range", (1, 2), ev((1, 0, 9, 0)), -3, 0),
    ("scope_out_of_range", (1, 2), ev((1, 0, make_meta(R), 0), (1, 0, make_meta(R, 3), 0)), -3, 1),
    ("tid_out_of_range", (2, 2), ev((1, 3, make_meta(W), 0), (1, 4, make_meta(W), 0)), -3, 1),
    ("fence_in_shared", (1, 2), ev((0, 0, make_meta(F, 1, 1), 0)), -3, 0),
    ("bar_in_shared", (1, 2), ev((0, 0, make_meta(BAR, 0, 1), 0)), -3, 0),
    # thread 0 continues past its barrier before thread 1 has arrived
    ("runs_ahead_of_barrier", (1, 2), ev((0, 0, make_meta(BAR), 0), (5, 0, make_meta(R), 0),
                                          (0, 1, make_meta(BAR), 0)), -3, 1),
    # thread 1 is active but never reaches the barrier: the instance never completes
    ("barrier_never_completes", (1, 2), ev((0, 0, make_meta(BAR), 0), (5, 1, make_meta(R), 0),
                                            (5, 0, make_meta(R), 0)), -3, 2),
    # an inactive thread (no events) is not a participant: the barrier completes
    ("inactive_thread_not_waited_for", (1, 3), ev((0, 0, make_meta(BAR), 0), (0, 1, make_meta(BAR), 0),
                                                   (5, 0, make_meta(R), 0)), 0, -1),
    ("trailing_barrier_ok", (1, 2), ev((5, 0, make_meta(W), 0), (0, 0, make_meta(BAR), 0)), 0, -1),
    # warp barrier whose mask lacks the emitting lane
    ("wbar_lane_not_in_mask", (1, 4, 2), ev((1, 1, make_meta(WBAR), 1)), -3, 0),
    # lane 0 continues before lane 1 arrives
    ("wbar_runs_ahead", (1, 4, 2), ev((1, 0, make_meta(WBAR), 3), (5, 0, make_meta(R), 0),
                                       (1, 1, make_meta(WBAR), 3)), -3, 1),
    # masks of one instance disagree
    ("wbar_mask_mismatch", (1, 4, 2), ev((1, 0, make_meta(WBAR), 3), (1, 1, make_meta(WBAR), 2)), -3, 1),
    ("wbar_ok", (1, 4, 2), ev((1, 0, make_meta(WBAR), 3), (1, 1, make_meta(WBAR), 3),
                               (5, 0, make_meta(R), 0)), 0, -1),
    # record errors are reported even when a barrier error comes earlier
    ("record_error_precedence", (1, 2), ev((0, 0, make_meta(BAR), 0), (5, 0, make_meta(R), 0),
                                            (0, 1, make_meta(BAR), 0), (1, 0, 8, 0)), -3, 3),
]


@pytest.mark.parametrize("name,grid,events,status,bad", CASES, ids=[c[0] for c in CASES])
def test_validation(name, grid, events, status, bad):
    for fn in (oracle.validate, oracle.check, oracle.bruteforce):
        r = fn(grid, events)
        assert r.status == status, (fn.__name__, r)
        assert r.bad_index == bad, (fn.__name__, r)


@pytest.mark.parametrize("grid", [(0, 4), (1, 0), (1, 1025), (1, 4, 33), (65536, 65536)])
def test_bad_grid(grid):
    r = oracle.check(grid, ev((0, 0, make_meta(R), 0)))
    assert r.status == -1


# ---------------------------------------------------------------- seeded malformed traces

from tracegen import random_trace  # noqa: E402
from tracegen.mutate import RECORD_KINDS, mutate  # noqa: E402


@pytest.mark.parametrize("kind", RECORD_KINDS)
@pytest.mark.parametrize("seed", range(40))
def test_record_rule_mutations_first_index(kind, seed):
    # a valid trace with one broken record: record rules are checked before barrier rules, so the
    # first offending index is the changed record's, whatever the rest of the trace does
    grid, ev0 = random_trace(seed)
    assert oracle.validate(grid, ev0).status == 0
    ev1, changed = mutate(grid, ev0, kind, seed + 1000)
    r = oracle.validate(grid, ev1)
    if not changed:
        assert r.status == 0
        return
    assert r.status == -3 and r.bad_index == min(changed), (kind, seed, r, changed)
    # the detector rejects it the same way
    c = oracle.check(grid, ev1)
    assert c.status == -3 and c.bad_index == min(changed)
