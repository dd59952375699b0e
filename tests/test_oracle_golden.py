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
