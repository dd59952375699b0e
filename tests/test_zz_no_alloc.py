"""rd_check_static (the check in the library's fixed scratch array, allocating nothing) against the
ordinary entry points (rd_trace_upload + rd_check + rd_races in a caller workspace), through the C
ABI: equal reports, statuses and first offending indices, two calls in a row, the second smaller."""
import ctypes

import numpy as np
import pytest

import tracegen
from tracegen.format import KIND, make_meta

pytestmark = pytest.mark.gpu

SCRATCH = 128 << 20
CLOCK = 8 << 20


@pytest.fixture(scope="module")
def rc():
    from paper_2111_12478_amd import RaceChecker
    c = RaceChecker(0)
    yield c
    c.close()


def _static(rc, grid, ev, limits=None, capacity=None):
    import torch
    import paper_2111_12478_amd as rd
    n = int(ev.shape[0])
    dev = torch.from_numpy(np.ascontiguousarray(ev, dtype=np.uint32).view(np.int32)).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    st, total = rd.rd_check_static(rc.ctx, grid, dev.data_ptr() if n else None, n, limits, None, 0, stream)
    if st not in (rd.RD_OK, rd.RD_ETRUNC):
        return st, np.zeros((0, 2), np.uint32), rd.rd_last_error(rc.ctx)[0]
    cap = total if capacity is None else capacity
    out = np.zeros((max(cap, 1), 2), dtype=np.uint32)
    st, total2 = rd.rd_check_static(rc.ctx, grid, dev.data_ptr() if n else None, n, limits, out.ctypes.data, cap,
                                    stream)
    assert total2 == total
    bad = rd.rd_last_error(rc.ctx)[0] if st == rd.RD_ETRACE else -1
    return st, out[: min(cap, total)], bad


def _plain(rc, grid, ev, limits):
    r = rc.check(grid, ev, limits)
    return r.status, r.pairs, (r.bad_index if r.status == -3 else -1)


def _same(rc, grid, ev):
    lim = {"clock_bytes": CLOCK}
    a = _static(rc, grid, ev)
    b = _plain(rc, grid, ev, lim)
    assert a[0] == b[0], (a[0], b[0])
    assert a[2] == b[2]
    np.testing.assert_array_equal(a[1], b[1])
    return a


def test_static_then_smaller(rc):
    print("static: large/64 then tiny", flush=True)
    # 262,144 events, 16 blocks x 256 threads: a workspace of about 105 MiB
    grid, ev, _, _ = tracegen.generate(tracegen.large(seed=2, scale=64))
    st, pairs, _ = _same(rc, grid, ev)
    assert st == 0 and len(pairs) > 0
    grid2, ev2, _, _ = tracegen.generate(tracegen.tiny())
    st2, pairs2, _ = _same(rc, grid2, ev2)
    assert st2 == 0 and len(pairs2) > 0


@pytest.mark.parametrize("seed", [3, 11, 5003, 5010])
def test_static_random_traces_twice(rc, seed):
    print(f"static: random seed {seed}", flush=True)
    g1, e1 = tracegen.random_trace(seed, max_blocks=6, max_tpb=40, max_events=6000)
    _same(rc, g1, e1)
    # the second call smaller: a prefix of the same valid trace (a prefix of a valid trace is valid)
    _same(rc, g1, e1[: len(e1) // 2])


def test_static_stencil_lock_chain(rc):
    print("static: stencil 4 x 4 blocks", flush=True)
    cfg = tracegen.stencil_small(seed=9, rb=4, cb=4, tpb=32, rows=3, sweeps=4, plant_rate=0.08)
    grid, ev, _, _ = tracegen.generate_stencil(cfg)
    _same(rc, grid, ev)


def test_static_invalid_trace_and_truncation(rc):
    print("static: invalid trace, truncation", flush=True)
    grid = (1, 2)
    m = make_meta
    ev = np.array([[0, 0, m(KIND["W"]), 0], [0, 1, m(KIND["W"]), 0], [0, 0, 99, 0]], dtype=np.uint32)
    _same(rc, grid, ev)
    ev = ev[:2]
    st, pairs, _ = _static(rc, grid, ev, capacity=0)
    assert st == -4 and len(pairs) == 0
    st, pairs, _ = _same(rc, grid, ev)
    assert st == 0 and pairs.tolist() == [[0, 1]]


def test_static_empty(rc):
    st, pairs, _ = _static(rc, (1, 1), np.zeros((0, 4), np.uint32))
    assert st == 0 and len(pairs) == 0


def test_static_too_large_is_refused(rc):
    import paper_2111_12478_amd as rd
    grid = (1024, 256)
    n = 8 << 20
    need = rd.rd_workspace_bytes(rc.ctx, grid, n, {"clock_bytes": CLOCK})
    assert need > SCRATCH
    import torch
    out = np.zeros((4, 2), np.uint32)
    dummy = torch.zeros(64, dtype=torch.int32, device="cuda")
    # refused on the host before anything is launched (the events are never read)
    st, total = rd.rd_check_static(rc.ctx, grid, dummy.data_ptr(), n, None, out.ctypes.data, 4,
                                   torch.cuda.current_stream().cuda_stream)
    assert st == rd.RD_ENOMEM and total == 0



def test_static_largest_stated_size(rc):
    # the size the header states fits: about 400,000 events (399,457 here, 24 blocks x 256 threads)
    print("static: large/42", flush=True)
    grid, ev, _, _ = tracegen.generate(tracegen.large(seed=2, scale=42))
    assert len(ev) > 399_000
    st, pairs, _ = _same(rc, grid, ev)
    assert st == 0 and len(pairs) > 0
