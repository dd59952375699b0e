"""The oracle against the paper's worked examples (tests/golden): brute-force closure and both
clock stores of the vector-clock detector must produce exactly the stated pairs."""
import numpy as np
import pytest

import oracle
from golden_io import all_cases

CASES = all_cases()


@pytest.mark.parametrize("case", CASES, ids=[c.name for c in CASES])
def test_bruteforce_matches_golden(case):
    r = oracle.bruteforce(case.grid, case.events)
    assert r.status == 0, r
    np.testing.assert_array_equal(r.pairs, case.expected)


@pytest.mark.parametrize("dense", [False, True], ids=["floor_clocks", "dense_clocks"])
@pytest.mark.parametrize("case", CASES, ids=[c.name for c in CASES])
def test_vector_clock_detector_matches_golden(case, dense):
    r = oracle.check(case.grid, case.events, dense=dense)
    assert r.status == 0, r
    np.testing.assert_array_equal(r.pairs, case.expected)


INCLUSIVE = [c for c in CASES if "inclusive" in c.by_reading]


@pytest.mark.parametrize("case", INCLUSIVE, ids=[c.name for c in INCLUSIVE])
def test_inclusive_reading_matches_golden(case):
    # the oracle's switch for the other reading of the scope rule, pinned by hand-derived pairs
    # (brute-force closure and both clock stores)
    want = case.by_reading["inclusive"]
    r = oracle.bruteforce(case.grid, case.events, inclusive=True)
    assert r.status == 0, r
    np.testing.assert_array_equal(r.pairs, want)
    for dense in (False, True):
        r = oracle.check(case.grid, case.events, dense=dense, inclusive=True)
        assert r.status == 0, r
        np.testing.assert_array_equal(r.pairs, want)


def test_inclusive_cases_present():
    assert len(INCLUSIVE) >= 5
