"""CPU oracle for scoped happens-before race checking (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  The product path (the HIP checker in ``paper_2111_12478_amd``) never does,
and the two share no code.

The C library ``liborc.so`` (built from ``rd_oracle.c`` by :func:`build`) holds two independent
computations of the race report:

* :func:`bruteforce` -- the declarative definition: the scoped happens-before graph of the trace
  (program order, block/warp barriers, release -> acquire with the scope rule; paper Section 2.2
  rules (i), (iii), (iv)) closed transitively with bitsets, and every conflicting pair it leaves
  unordered (race definition of Section 1 / Section 2.2).  Tiny traces only.
* :func:`check` -- the paper's per-event vector-clock detector (Algorithm 1 clock updates, epoch
  check against the per-location history of Section 4.1), with either dense vector clocks or
  block-floor + exception clocks with the forced barrier compression of Section 5.2.
* :func:`gwcp` -- the predictive relation GWCP of Section 4 tracked by Algorithms 1 and 2 (P, N, C
  and H clocks, Acq/Rel queues, locksets and lock-location clocks), dense clocks.
* :func:`gwcp_bruteforce` -- GWCP's definition (rules (i)-(iv)) as a fixpoint over event pairs;
  tiny traces only.
* :func:`lockset` -- the lockset pass the paper describes for ScoRD (Section 2.2, Section 3).

Traces are ``(N, 4)`` uint32 arrays of records ``(addr, tid, meta, aux)``; pairs come back as an
``(M, 2)`` uint32 array of trace indices ``(first, second)``, first < second, sorted.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_SRC = os.path.join(_HERE, "rd_oracle.c")

OK, EINVAL, ENOMEM, ETRACE = 0, -1, -2, -3


class OraclePairs(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("cap", ctypes.c_uint64), ("data", ctypes.POINTER(ctypes.c_uint32))]


def build(force: bool = True) -> str:
    """Compile rd_oracle.c into liborc.so with gcc (plain C, no HIP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        vp = ctypes.c_void_p
        lib.orc_check.argtypes = [u32, u32, u32, vp, u64, i32, i32, ctypes.POINTER(u64), ctypes.POINTER(OraclePairs)]
        lib.orc_check.restype = i32
        lib.orc_bruteforce.argtypes = [u32, u32, u32, vp, u64, i32, ctypes.POINTER(u64), ctypes.POINTER(OraclePairs)]
        lib.orc_bruteforce.restype = i32
        lib.orc_gwcp.argtypes = [u32, u32, u32, vp, u64, ctypes.POINTER(u64), ctypes.POINTER(OraclePairs)]
        lib.orc_gwcp.restype = i32
        lib.orc_gwcp_bruteforce.argtypes = [u32, u32, u32, vp, u64, ctypes.POINTER(u64), ctypes.POINTER(OraclePairs)]
        lib.orc_gwcp_bruteforce.restype = i32
        lib.orc_lockset.argtypes = [u32, u32, u32, vp, u64, ctypes.POINTER(u64), ctypes.POINTER(OraclePairs)]
        lib.orc_lockset.restype = i32
        lib.orc_validate.argtypes = [u32, u32, u32, vp, u64, ctypes.POINTER(u64)]
        lib.orc_validate.restype = i32
        lib.orc_pairs_free.argtypes = [ctypes.POINTER(OraclePairs)]
        lib.orc_pairs_free.restype = None
        _lib = lib
    return _lib


class OracleResult:
    """status (0 ok, -1 bad grid, -2 out of memory, -3 bad trace), bad_index, pairs."""

    def __init__(self, status: int, bad_index: int, pairs: np.ndarray):
        self.status = status
        self.bad_index = bad_index
        self.pairs = pairs

    def __repr__(self):
        return f"OracleResult(status={self.status}, bad_index={self.bad_index}, n_pairs={len(self.pairs)})"


def _events(events) -> np.ndarray:
    ev = np.ascontiguousarray(np.asarray(events, dtype=np.uint32))
    if ev.ndim != 2 or ev.shape[1] != 4:
        raise ValueError("events must be an (N, 4) uint32 array of (addr, tid, meta, aux)")
    return ev


def _take_pairs(lib, out: OraclePairs) -> np.ndarray:
    n = int(out.n)
    if n == 0:
        res = np.zeros((0, 2), dtype=np.uint32)
    else:
        buf = np.ctypeslib.as_array(out.data, shape=(2 * n,))
        res = buf.reshape(n, 2).copy()
    lib.orc_pairs_free(ctypes.byref(out))
    return res


def _bad(v: int) -> int:
    return -1 if v == (1 << 64) - 1 else int(v)


def check(grid, events, dense: bool = False, inclusive: bool = False) -> OracleResult:
    """Per-event vector-clock detector.  grid = (n_blocks, threads_per_block[, warp_size])."""
    lib = _load()
    ev = _events(events)
    nb, tpb, ws = (list(grid) + [32])[:3]
    bad = ctypes.c_uint64(0)
    out = OraclePairs()
    rc = lib.orc_check(nb, tpb, ws, ev.ctypes.data, ev.shape[0], int(dense), int(inclusive),
                       ctypes.byref(bad), ctypes.byref(out))
    return OracleResult(rc, _bad(bad.value), _take_pairs(lib, out))


def bruteforce(grid, events, inclusive: bool = False) -> OracleResult:
    """Transitive closure of the happens-before graph (<= 16384 events)."""
    lib = _load()
    ev = _events(events)
    nb, tpb, ws = (list(grid) + [32])[:3]
    bad = ctypes.c_uint64(0)
    out = OraclePairs()
    rc = lib.orc_bruteforce(nb, tpb, ws, ev.ctypes.data, ev.shape[0], int(inclusive),
                            ctypes.byref(bad), ctypes.byref(out))
    return OracleResult(rc, _bad(bad.value), _take_pairs(lib, out))


def gwcp(grid, events) -> OracleResult:
    """GWCP-predictable races by Algorithms 1 and 2 of Section 4.1 (<= 8192 threads)."""
    lib = _load()
    ev = _events(events)
    nb, tpb, ws = (list(grid) + [32])[:3]
    bad = ctypes.c_uint64(0)
    out = OraclePairs()
    rc = lib.orc_gwcp(nb, tpb, ws, ev.ctypes.data, ev.shape[0], ctypes.byref(bad), ctypes.byref(out))
    return OracleResult(rc, _bad(bad.value), _take_pairs(lib, out))


def gwcp_bruteforce(grid, events) -> OracleResult:
    """GWCP-unordered conflicting pairs from the definition, rules (i)-(iv) (<= 4096 events)."""
    lib = _load()
    ev = _events(events)
    nb, tpb, ws = (list(grid) + [32])[:3]
    bad = ctypes.c_uint64(0)
    out = OraclePairs()
    rc = lib.orc_gwcp_bruteforce(nb, tpb, ws, ev.ctypes.data, ev.shape[0], ctypes.byref(bad), ctypes.byref(out))
    return OracleResult(rc, _bad(bad.value), _take_pairs(lib, out))


def lockset(grid, events) -> OracleResult:
    """The lockset pass of Section 2.2 / Section 3 (ScoRD after Eraser): each access against its
    location's previous access, reported when they conflict, one of them holds a lock and no lock
    is common to both."""
    lib = _load()
    ev = _events(events)
    nb, tpb, ws = (list(grid) + [32])[:3]
    bad = ctypes.c_uint64(0)
    out = OraclePairs()
    rc = lib.orc_lockset(nb, tpb, ws, ev.ctypes.data, ev.shape[0], ctypes.byref(bad), ctypes.byref(out))
    return OracleResult(rc, _bad(bad.value), _take_pairs(lib, out))


def validate(grid, events) -> OracleResult:
    """Trace validation only: status and the first offending event index."""
    lib = _load()
    ev = _events(events)
    nb, tpb, ws = (list(grid) + [32])[:3]
    bad = ctypes.c_uint64(0)
    rc = lib.orc_validate(nb, tpb, ws, ev.ctypes.data, ev.shape[0], ctypes.byref(bad))
    return OracleResult(rc, _bad(bad.value), np.zeros((0, 2), dtype=np.uint32))


def race_kinds(events, pairs) -> np.ndarray:
    """Unique race kinds of a report (the "unique kinds" counted in the paper's Table 2, Section 6).

    The paper does not define a kind; the reading taken here: a kind is the unordered pair of the
    two accesses' site ids (the records' ``aux`` words), so the same two program sites racing in
    either order are one kind.  Returns a ``(K, 3)`` uint32 array of ``(site_lo, site_hi, count)``,
    rows in ascending ``(site_lo, site_hi)`` order, ``count`` the number of racing pairs of the kind.
    Parity pins: special cases only (every site distinct, every site equal, swapped order).
    """
    ev = _events(events)
    pr = np.asarray(pairs, dtype=np.uint32).reshape(-1, 2)
    if pr.shape[0] == 0:
        return np.zeros((0, 3), dtype=np.uint32)
    sa = ev[pr[:, 0], 3]
    sb = ev[pr[:, 1], 3]
    sites = np.stack([np.minimum(sa, sb), np.maximum(sa, sb)], axis=1)
    kinds, counts = np.unique(sites, axis=0, return_counts=True)
    return np.concatenate([kinds, counts.astype(np.uint32)[:, None]], axis=1).astype(np.uint32)
