"""Error and fallback paths of the HIP checker through the C ABI: bad grids and workspaces, calls
out of order, the knowledge-vector pool running out, the parallel knowledge engine handing a trace
to the sequential interpreter, and seeded malformed traces against the oracle's first offending
index."""
import numpy as np
import pytest

import oracle
import tracegen
from tracegen.format import KIND, make_meta
from tracegen.mutate import BARRIER_KINDS, RECORD_KINDS, mutate

pytestmark = pytest.mark.gpu

R, W, ACQ, REL, WBAR = (KIND[k] for k in ("R", "W", "ACQ", "REL", "WBAR"))


@pytest.fixture(scope="module")
def rc():
    from paper_2111_12478_amd import RaceChecker
    c = RaceChecker(0)
    yield c
    c.close()


@pytest.mark.parametrize("grid", [(0, 4), (1, 0), (1, 1025), (1, 4, 33), (1 << 22, 1024)])
def test_bad_grid_rejected(rc, grid):
    import paper_2111_12478_amd as rd
    with pytest.raises(rd.RdError) as e:
        rd.rd_workspace_bytes(rc.ctx, grid, 16)
    assert e.value.status == rd.RD_EINVAL
    st, tr = rd.rd_trace_upload(rc.ctx, grid, None, 0, 1, None, 0, None, None)
    assert st == rd.RD_EINVAL and not tr


def test_bad_workspace_rejected(rc):
    import torch
    import paper_2111_12478_amd as rd
    ev = np.array([(5, 0, make_meta(W), 0), (5, 1, make_meta(W), 0)], np.uint32)
    need = rd.rd_workspace_bytes(rc.ctx, (1, 2), 2)
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    st, tr = rd.rd_trace_upload(rc.ctx, (1, 2), ev.ctypes.data, 2, 0, ws.data_ptr() + 16, need, None, stream)
    assert st == rd.RD_EINVAL and not tr  # not 256-byte aligned
    st, tr = rd.rd_trace_upload(rc.ctx, (1, 2), ev.ctypes.data, 2, 0, ws.data_ptr(), need - 256, None, stream)
    assert st == rd.RD_ENOMEM and not tr  # too small
    st, tr = rd.rd_trace_upload(rc.ctx, (1, 2), ev.ctypes.data, 2, 0, ws.data_ptr(), need, None, stream)
    assert st == rd.RD_OK
    try:
        st, n = rd.rd_races(rc.ctx, tr, None, 0)
        assert st == rd.RD_ESTATE  # rd_races before rd_check
        assert rd.rd_check(rc.ctx, tr, stream) == rd.RD_OK
        st, n = rd.rd_races(rc.ctx, tr, None, 0)
        assert st == rd.RD_ETRUNC and n == 1
    finally:
        rd.rd_trace_free(rc.ctx, tr)
    torch.cuda.synchronize()


def test_member_without_workspace_needs_a_batch(rc):
    import torch
    import paper_2111_12478_amd as rd
    dev = torch.zeros((4, 4), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    st, tr = rd.rd_trace_upload(rc.ctx, (1, 4), dev.data_ptr(), 4, 1, None, 0, None, stream)
    assert st == rd.RD_OK
    try:
        assert rd.rd_check(rc.ctx, tr, stream) == rd.RD_ESTATE
    finally:
        rd.rd_trace_free(rc.ctx, tr)


def _lock_trace(n_sections, n_threads, n_locks, seed, per_section=1, p_plain=0.0, words_per_lock=1):
    """Critical sections one after another in trace order: ACQ(l, DEV); per_section reads or
    writes of words that l protects (words_per_lock of them); REL(l, DEV); with probability
    p_plain an unprotected write of a random protected word comes between two sections."""
    rng = np.random.default_rng(seed)
    t = rng.integers(0, n_threads, n_sections)
    lk = rng.integers(0, n_locks, n_sections)
    base = 1 << 20
    rows = []
    acc = rng.random((n_sections, per_section)) < 0.5
    word = rng.integers(0, words_per_lock, (n_sections, per_section))
    for s in range(n_sections):
        if p_plain and rng.random() < p_plain:
            w = base + int(rng.integers(0, n_locks)) * words_per_lock + int(rng.integers(0, words_per_lock))
            rows.append((w, int(rng.integers(0, n_threads)), make_meta(W), 0))
        rows.append((int(lk[s]), int(t[s]), make_meta(ACQ, 1), 0))
        for a, wd in zip(acc[s], word[s]):
            rows.append((base + int(lk[s]) * words_per_lock + int(wd), int(t[s]), make_meta(W if a else R), 0))
        rows.append((int(lk[s]), int(t[s]), make_meta(REL, 1), 0))
    return np.array(rows, np.uint32)


def test_knowledge_pool_exhausted_is_reported(rc):
    ev = _lock_trace(40, 8, 3, seed=1, p_plain=0.2)
    grid = (2, 4)
    want = oracle.check(grid, ev)
    assert want.status == 0
    got = rc.check(grid, ev, limits={"clock_bytes": 64})
    assert got.status == -2, got  # RD_ENOMEM
    got = rc.check(grid, ev)
    assert got.status == 0
    np.testing.assert_array_equal(got.pairs, want.pairs)


def test_interpreter_pool_exhausted_is_reported(rc):
    # a warp barrier sends the trace to the sequential interpreter
    ev = _lock_trace(40, 8, 3, seed=2, p_plain=0.2)
    wb = np.array([(7, 0, make_meta(WBAR), 1)], np.uint32)
    ev = np.concatenate([wb, ev])
    grid = (2, 4, 4)
    want = oracle.check(grid, ev)
    assert want.status == 0
    got = rc.check(grid, ev, limits={"clock_bytes": 64})
    assert got.status == -2, got
    got = rc.check(grid, ev)
    assert got.status == 0
    np.testing.assert_array_equal(got.pairs, want.pairs)


def test_engine_hands_acquire_heavy_trace_to_interpreter(rc):
    # more than a quarter of 4.3M events are releases and acquires: past the parallel engine's
    # capacity, so the sequential interpreter builds the knowledge vectors
    n_sections = 4_300_000 // 6
    ev = _lock_trace(n_sections, 64, 4096, seed=3, per_section=4, p_plain=2e-3, words_per_lock=16)
    grid = (2, 32)
    n = len(ev)
    ral = int(np.isin(ev[:, 2] & 15, (ACQ, REL)).sum())
    assert n > (1 << 22) + 4 and ral > n // 4, (n, ral)
    print(f"acquire-heavy trace: {n} events, {ral} releases and acquires", flush=True)
    want = oracle.check(grid, ev)
    assert want.status == 0 and len(want.pairs) > 0
    got = rc.check(grid, ev, limits={"clock_bytes": 1 << 30})
    assert got.status == 0, got
    np.testing.assert_array_equal(got.pairs, want.pairs)


@pytest.mark.parametrize("kind", RECORD_KINDS + BARRIER_KINDS)
@pytest.mark.parametrize("seed", range(25))
def test_malformed_traces_match_oracle(rc, kind, seed):
    grid, ev0 = tracegen.random_trace(seed + 300)
    ev1, _ = mutate(grid, ev0, kind, seed)
    want = oracle.check(grid, ev1)
    got = rc.check(grid, ev1)
    assert got.status == want.status, (kind, seed, got, want)
    if want.status == -3:
        assert got.bad_index == want.bad_index, (kind, seed, got, want)
    elif want.status == 0:
        np.testing.assert_array_equal(got.pairs, want.pairs)
