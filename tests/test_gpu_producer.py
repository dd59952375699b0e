"""The device-side producer (include/rd_device.h): example kernels record their own events on the
GPU, straight into device memory; the trace they leave is valid, and the checker reading it in
place (rd_trace_upload with events_on_device = 1) reports exactly what the oracle reports for it:
no race for the correct kernels, the planted ones otherwise."""
import ctypes
import os

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
DEMO = os.path.join(os.path.dirname(HERE), "paper_2111_12478_amd", "librd_demo.so")


@pytest.fixture(scope="module")
def rc():
    from paper_2111_12478_amd import RaceChecker
    c = RaceChecker(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def demo(rc):
    lib = ctypes.CDLL(DEMO)
    lib.rd_demo_mem_words.restype = ctypes.c_uint64
    lib.rd_demo_mem_words.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    lib.rd_demo_run.restype = ctypes.c_int
    lib.rd_demo_run.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
    return lib


def _record(demo, which, nb, nt, plant, cap=1 << 22):
    """Runs a demo kernel; returns (grid, device events (M, 4) int32, host copy, error word)."""
    import torch
    words = demo.rd_demo_mem_words(nb, nt)
    mem = torch.zeros(words, dtype=torch.int32, device="cuda")
    mem[: nb * nt] = torch.arange(nb * nt, dtype=torch.int32, device="cuda") % 7
    ev = torch.zeros((cap, 4), dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    print(f"demo {which} {nb}x{nt} plant {plant}", flush=True)
    assert demo.rd_demo_run(which, nb, nt, plant, mem.data_ptr(), ev.data_ptr(), cap, count.data_ptr(), stream) == 0
    torch.cuda.synchronize()
    n = int(count.item())
    assert n <= cap
    err = int(mem[-1].item())
    return (nb, nt), ev[:n], ev[:n].cpu().numpy().view(np.uint32), err


def _check_both(rc, grid, dev_ev, host_ev):
    want = oracle.check(grid, host_ev)
    assert want.status == 0, want
    got = rc.check(grid, dev_ev)
    assert got.status == 0, got
    np.testing.assert_array_equal(got.pairs, want.pairs)
    return want.pairs


@pytest.mark.parametrize("nb,nt", [(4, 64), (16, 128), (64, 256)])
def test_reduce_is_race_free(rc, demo, nb, nt):
    grid, dev, host, err = _record(demo, 0, nb, nt, 0)
    assert err == 0
    pairs = _check_both(rc, grid, dev, host)
    assert len(pairs) == 0
    # every event of every thread is there: its reads, writes, barriers; thread 0 of each block
    # takes the lock once
    kinds = host[:, 2] & 15
    assert int((kinds == 4).sum()) == nb * nt * (1 + int(np.log2(nt)))
    assert int((kinds == 6).sum()) == nb and int((kinds == 7).sum()) == nb


@pytest.mark.parametrize("plant", [1, 2, 3])
def test_reduce_planted_races(rc, demo, plant):
    nb, nt = 8, 64
    grid, dev, host, err = _record(demo, 0, nb, nt, plant)
    assert err == 0
    pairs = _check_both(rc, grid, dev, host)
    assert len(pairs) > 0
    space = (host[pairs[:, 0], 2] >> 6) & 1
    if plant & 1:  # blocks race on the accumulator (a global word)
        assert (space == 0).any()
    if plant & 2:  # every block races in its shared memory
        blocks = set((host[pairs[space == 1, 1], 1] // nt).tolist())
        assert blocks == set(range(nb))


@pytest.mark.parametrize("nb,nt", [(2, 64), (16, 64), (64, 128)])
def test_chain_is_race_free(rc, demo, nb, nt):
    grid, dev, host, err = _record(demo, 1, nb, nt, 0)
    assert err == 0
    pairs = _check_both(rc, grid, dev, host)
    assert len(pairs) == 0


@pytest.mark.parametrize("plant", [1, 2])
def test_chain_planted_races(rc, demo, plant):
    nb, nt = 8, 64
    grid, dev, host, err = _record(demo, 1, nb, nt, plant)
    assert err == 0
    pairs = _check_both(rc, grid, dev, host)
    # block 1's readers race with block 0's write of its value
    firsts = host[pairs[:, 0]]
    seconds = host[pairs[:, 1]]
    assert ((firsts[:, 1] == 0) & ((seconds[:, 1] // nt) == 1)).sum() == nt


def test_lockset_of_a_recorded_trace(rc, demo):
    # the lock-protected accumulator: no lockset pair; without the lock: no lock held at all, so
    # the lockset pass skips the unprotected pairs (as the paper says of ScoRD)
    for plant in (0, 1):
        grid, dev, host, err = _record(demo, 0, 8, 64, plant)
        want = oracle.lockset(grid, host)
        from paper_2111_12478_amd import rd_trace_free
        tr, ws, keep = rc.prepare(grid, dev)
        try:
            got = rc.lockset(tr)
        finally:
            rd_trace_free(rc.ctx, tr)
        assert got.status == want.status == 0
        np.testing.assert_array_equal(got.pairs, want.pairs)
        assert len(want.pairs) == 0
