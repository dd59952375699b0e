"""Pins of oracle.race_kinds (unique race kinds, the paper's Table 2 column "unique kinds" of
Section 6, with a kind read as the unordered pair of the two accesses' site ids)."""
import numpy as np

import oracle


def _events(n, aux):
    ev = np.zeros((n, 4), dtype=np.uint32)
    ev[:, 3] = aux
    return ev


def test_no_pairs_no_kinds():
    assert oracle.race_kinds(_events(4, 7), np.zeros((0, 2), np.uint32)).shape == (0, 3)


def test_distinct_sites_one_kind_per_pair():
    # every event its own site: each pair is its own kind, the sites being the events' own
    rng = np.random.default_rng(5)
    n = 200
    perm = rng.permutation(1000)[:n].astype(np.uint32)
    ev = _events(n, perm)
    a = rng.integers(0, n - 1, 300)
    b = a + 1 + rng.integers(0, 5, 300)
    keep = b < n
    pairs = np.unique(np.stack([a[keep], b[keep]], 1), axis=0).astype(np.uint32)
    got = oracle.race_kinds(ev, pairs)
    assert got.shape[0] == pairs.shape[0]
    assert (got[:, 2] == 1).all()
    want = sorted((min(perm[x], perm[y]), max(perm[x], perm[y])) for x, y in pairs)
    assert [tuple(r[:2]) for r in got] == want


def test_one_site_one_kind():
    ev = _events(50, 9)
    pairs = np.array([[i, j] for i in range(10) for j in range(i + 1, 12)], dtype=np.uint32)
    got = oracle.race_kinds(ev, pairs)
    assert got.tolist() == [[9, 9, pairs.shape[0]]]


def test_order_of_the_two_sites_does_not_matter():
    # events 0..3 with sites 5, 3, 3, 5: (0,1) is (5,3), (2,3) is (3,5): one kind, two pairs
    ev = _events(4, np.array([5, 3, 3, 5], np.uint32))
    got = oracle.race_kinds(ev, np.array([[0, 1], [2, 3]], np.uint32))
    assert got.tolist() == [[3, 5, 2]]


def test_counts_add_up_and_rows_increase():
    rng = np.random.default_rng(11)
    ev = _events(500, rng.integers(0, 12, 500).astype(np.uint32))
    a = rng.integers(0, 499, 2000)
    b = np.minimum(a + 1 + rng.integers(0, 40, 2000), 499)
    pairs = np.unique(np.stack([a, b], 1), axis=0).astype(np.uint32)
    got = oracle.race_kinds(ev, pairs).astype(np.int64)
    assert got[:, 2].sum() == pairs.shape[0]
    assert (got[:, 0] <= got[:, 1]).all()
    keys = got[:, 0] * (1 << 32) + got[:, 1]
    assert (np.diff(keys) > 0).all()
