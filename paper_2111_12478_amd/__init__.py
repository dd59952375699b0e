"""Scoped happens-before race checking of GPU event traces on MI355X (gfx950).

A thin ctypes binding of ``librd.so`` (``include/rd.h``).  The functions named ``rd_*`` mirror the
C interface one to one (argument marshalling only); :class:`RaceChecker` wraps them for the common
case: a torch-owned workspace on the current HIP device, the current torch stream, and a numpy
report.  Every step of the check runs in the library's HIP kernels; there is no other code path:
if the library is not built, or there is no GPU, the calls raise.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librd.so")

RD_OK, RD_EINVAL, RD_ENOMEM, RD_ETRACE, RD_ETRUNC, RD_EHIP, RD_ESTATE = 0, -1, -2, -3, -4, -5, -6
READ, WRITE, ATOMIC, FENCE, BAR, WBAR, ACQ, REL = range(8)
BLOCK, DEVICE, SYSTEM = 0, 1, 2
GLOBAL, SHARED = 0, 1


class rd_grid(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_uint32), ("threads_per_block", ctypes.c_uint32),
                ("warp_size", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class rd_limits(ctypes.Structure):
    _fields_ = [("max_pairs", ctypes.c_uint64), ("clock_bytes", ctypes.c_uint64)]


class rd_pair(ctypes.Structure):
    _fields_ = [("first", ctypes.c_uint32), ("second", ctypes.c_uint32)]


class rd_server_config(ctypes.Structure):
    _fields_ = [("device_bytes", ctypes.c_uint64), ("max_batch", ctypes.c_uint32), ("max_inflight", ctypes.c_uint32)]


class rd_request_info(ctypes.Structure):
    _fields_ = [("n_races", ctypes.c_uint64), ("bad_index", ctypes.c_uint64), ("submit_s", ctypes.c_double),
                ("start_s", ctypes.c_double), ("done_s", ctypes.c_double)]


class rd_tuning(ctypes.Structure):
    _fields_ = [("radix_bits", ctypes.c_uint32), ("waves_per_block", ctypes.c_uint32),
                ("items_per_lane", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class rd_stats(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_uint64), ("n_accesses", ctypes.c_uint64), ("kind_count", ctypes.c_uint64 * 8),
                ("key_bits", ctypes.c_uint32), ("max_phase", ctypes.c_uint32), ("engine", ctypes.c_uint32),
                ("packed", ctypes.c_uint32), ("clock_vectors", ctypes.c_uint64), ("clock_words", ctypes.c_uint64),
                ("clock_bytes", ctypes.c_uint64), ("dense_clock_bytes", ctypes.c_uint64),
                ("engine_ops", ctypes.c_uint64), ("engine_groups", ctypes.c_uint64), ("slow_chunks", ctypes.c_uint64),
                ("race_pairs", ctypes.c_uint64), ("workspace_bytes", ctypes.c_uint64)]


class RdError(RuntimeError):
    def __init__(self, status, msg, event_index=None):
        super().__init__(f"{msg} (status {status})")
        self.status = status
        self.event_index = event_index


_lib = None

# Contexts and servers still open when the interpreter exits are closed by an exit handler, while
# the HIP runtime (and any profiler attached to it) is still alive; a finaliser that runs during
# interpreter shutdown makes no HIP call.
_open = weakref.WeakSet()


@atexit.register
def _close_all():
    # servers first: each holds its checker's context
    for obj in sorted(list(_open), key=lambda o: 0 if isinstance(o, Server) else 1):
        try:
            obj.close()
        except Exception:
            pass


def load_library():
    """Loads librd.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2111_12478_amd/build.py")
        # torch first: the library then binds to the HIP runtime torch has loaded, so the process
        # holds one runtime whichever of the two is used first
        import torch  # noqa: F401
        lib = ctypes.CDLL(LIB_PATH)
        vp, u64, i32, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint32
        P = ctypes.POINTER
        sig = {
            "rd_init": ([ctypes.c_int, P(vp)], i32),
            "rd_shutdown": ([vp], i32),
            "rd_workspace_bytes": ([vp, P(rd_grid), u64, P(rd_limits), P(u64)], i32),
            "rd_trace_upload": ([vp, P(rd_grid), vp, u64, ctypes.c_int, vp, u64, P(rd_limits), vp, P(vp)], i32),
            "rd_check": ([vp, vp, vp], i32),
            "rd_races": ([vp, vp, vp, u64, P(u64)], i32),
            "rd_check_static": ([vp, P(rd_grid), vp, u64, P(rd_limits), vp, u64, P(u64), vp], i32),
            "rd_race_kinds": ([vp, vp, vp, u64, P(u64)], i32),
            "rd_lockset": ([vp, vp, vp, u64, P(u64)], i32),
            "rd_gwcp": ([vp, vp, vp, u64, P(u64)], i32),
            "rd_trace_free": ([vp, vp], i32),
            "rd_trace_stats": ([vp, vp, P(rd_stats)], i32),
            "rd_batch_workspace_bytes": ([vp, P(vp), u32, P(rd_limits), P(u64)], i32),
            "rd_check_many": ([vp, P(vp), u32, vp, u64, P(rd_limits), vp], i32),
            "rd_races_many": ([vp, P(vp), u32, vp, u64, P(u64), P(i32)], i32),
            "rd_batch_capture": ([vp, P(vp), u32, vp, u64, P(rd_limits), vp, P(vp)], i32),
            "rd_graph_launch": ([vp, vp, vp], i32),
            "rd_graph_free": ([vp, vp], i32),
            "rd_tuning_count": ([P(u32)], i32),
            "rd_tuning_get": ([u32, P(rd_tuning)], i32),
            "rd_set_tuning": ([vp, u32], i32),
            "rd_get_tuning": ([vp, P(u32)], i32),
            "rd_autotune": ([vp, P(vp), u32, vp, u64, vp, P(u32), P(ctypes.c_double)], i32),
            "rd_server_open": ([vp, vp, P(rd_server_config), P(vp)], i32),
            "rd_server_submit": ([vp, P(rd_grid), vp, u64, P(u64)], i32),
            "rd_server_wait": ([vp, u64, vp, u64, P(rd_request_info)], i32),
            "rd_server_stats": ([vp, P(u64), P(u64)], i32),
            "rd_server_close": ([vp], i32),
            "rd_strerror": ([i32], ctypes.c_char_p),
            "rd_last_error": ([vp, P(u64), ctypes.c_char_p, u64], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
    return _lib


# ---------------------------------------------------------------- the C interface, by name

def rd_init(device: int = 0) -> int:
    ctx = ctypes.c_void_p()
    st = load_library().rd_init(device, ctypes.byref(ctx))
    if st != RD_OK:
        raise RdError(st, f"rd_init({device}) failed")
    return ctx.value


def rd_shutdown(ctx: int) -> int:
    return load_library().rd_shutdown(ctx)


def _grid(grid) -> rd_grid:
    g = list(grid) + [0] * (3 - len(grid))
    return rd_grid(int(g[0]), int(g[1]), int(g[2]), 0)


def _limits(limits):
    if limits is None:
        return None
    if isinstance(limits, rd_limits):
        return ctypes.byref(limits)
    return ctypes.byref(rd_limits(int(limits.get("max_pairs", 0)), int(limits.get("clock_bytes", 0))))


def rd_workspace_bytes(ctx: int, grid, n_events: int, limits=None) -> int:
    out = ctypes.c_uint64()
    g = _grid(grid)
    st = load_library().rd_workspace_bytes(ctx, ctypes.byref(g), n_events, _limits(limits), ctypes.byref(out))
    if st != RD_OK:
        raise RdError(st, "rd_workspace_bytes failed")
    return out.value


def rd_trace_upload(ctx, grid, events_ptr, n_events, events_on_device, workspace_ptr, workspace_bytes,
                    limits, stream) -> tuple[int, int]:
    """Returns (status, trace handle)."""
    tr = ctypes.c_void_p()
    g = _grid(grid)
    st = load_library().rd_trace_upload(ctx, ctypes.byref(g), events_ptr, n_events, int(events_on_device),
                                        workspace_ptr, workspace_bytes, _limits(limits), stream, ctypes.byref(tr))
    return st, tr.value


def rd_check(ctx, trace, stream) -> int:
    return load_library().rd_check(ctx, trace, stream)


def rd_race_kinds(ctx, trace, out_ptr, capacity) -> tuple[int, int]:
    """Unique race kinds of a checked trace into (capacity, 3) uint32 records (site_lo, site_hi,
    count) at out_ptr.  Returns (status, total kinds)."""
    n = ctypes.c_uint64()
    st = load_library().rd_race_kinds(ctx, trace, out_ptr, capacity, ctypes.byref(n))
    return st, n.value


def rd_lockset(ctx, trace, out_ptr, capacity) -> tuple[int, int]:
    """The lockset pass over a bound trace: pairs into (capacity, 2) uint32 host memory at out_ptr.
    Returns (status, total pairs)."""
    n = ctypes.c_uint64()
    st = load_library().rd_lockset(ctx, trace, out_ptr, capacity, ctypes.byref(n))
    return st, n.value


def rd_gwcp(ctx, trace, out_ptr, capacity) -> tuple[int, int]:
    """The GWCP pass (Section 4) over a bound trace: pairs into (capacity, 2) uint32 host memory at
    out_ptr.  Returns (status, total pairs)."""
    n = ctypes.c_uint64()
    st = load_library().rd_gwcp(ctx, trace, out_ptr, capacity, ctypes.byref(n))
    return st, n.value


def rd_races(ctx, trace, out_ptr, capacity) -> tuple[int, int]:
    n = ctypes.c_uint64()
    st = load_library().rd_races(ctx, trace, out_ptr, capacity, ctypes.byref(n))
    return st, n.value


def rd_check_static(ctx, grid, events_ptr, n_events, limits, out_ptr, capacity, stream) -> tuple[int, int]:
    """Check of device-resident events in the library's static scratch array (allocates nothing);
    pairs into (capacity, 2) uint32 host memory at out_ptr.  Returns (status, total pairs)."""
    n = ctypes.c_uint64()
    g = _grid(grid)
    st = load_library().rd_check_static(ctx, ctypes.byref(g), events_ptr, n_events, _limits(limits), out_ptr,
                                        capacity, ctypes.byref(n), stream)
    return st, n.value


def _trace_array(traces):
    arr = (ctypes.c_void_p * max(1, len(traces)))()
    for j, t in enumerate(traces):
        arr[j] = t
    return arr


def rd_batch_workspace_bytes(ctx, traces, limits=None) -> int:
    out = ctypes.c_uint64()
    st = load_library().rd_batch_workspace_bytes(ctx, _trace_array(traces), len(traces), _limits(limits),
                                                 ctypes.byref(out))
    if st != RD_OK:
        raise RdError(st, "rd_batch_workspace_bytes failed")
    return out.value


def rd_check_many(ctx, traces, workspace_ptr, workspace_bytes, limits, stream) -> int:
    return load_library().rd_check_many(ctx, _trace_array(traces), len(traces), workspace_ptr, workspace_bytes,
                                        _limits(limits), stream)


def rd_races_many(ctx, traces, out_ptr, capacity):
    """Returns (status, counts (n,) uint64, statuses (n,) int32)."""
    n = len(traces)
    counts = np.zeros(max(n, 1), dtype=np.uint64)
    sts = np.zeros(max(n, 1), dtype=np.int32)
    st = load_library().rd_races_many(ctx, _trace_array(traces), n, out_ptr, capacity,
                                      counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                      sts.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return st, counts[:n], sts[:n]


def rd_batch_capture(ctx, traces, workspace_ptr, workspace_bytes, limits, stream) -> tuple[int, int]:
    g = ctypes.c_void_p()
    st = load_library().rd_batch_capture(ctx, _trace_array(traces), len(traces), workspace_ptr, workspace_bytes,
                                         _limits(limits), stream, ctypes.byref(g))
    return st, g.value


def rd_graph_launch(ctx, graph, stream) -> int:
    return load_library().rd_graph_launch(ctx, graph, stream)


def rd_graph_free(ctx, graph) -> int:
    return load_library().rd_graph_free(ctx, graph)


def rd_tuning_count() -> int:
    n = ctypes.c_uint32()
    load_library().rd_tuning_count(ctypes.byref(n))
    return n.value


def rd_tuning_get(index) -> tuple[int, int, int]:
    t = rd_tuning()
    st = load_library().rd_tuning_get(index, ctypes.byref(t))
    if st != RD_OK:
        raise RdError(st, "rd_tuning_get failed")
    return t.radix_bits, t.waves_per_block, t.items_per_lane


def rd_set_tuning(ctx, index) -> int:
    return load_library().rd_set_tuning(ctx, index)


def rd_get_tuning(ctx) -> int:
    v = ctypes.c_uint32()
    load_library().rd_get_tuning(ctx, ctypes.byref(v))
    return v.value


def rd_autotune(ctx, traces, workspace_ptr, workspace_bytes, stream):
    """Returns (status, best index, ms per variant)."""
    k = rd_tuning_count()
    best = ctypes.c_uint32()
    ms = (ctypes.c_double * k)()
    st = load_library().rd_autotune(ctx, _trace_array(traces), len(traces), workspace_ptr, workspace_bytes or 0,
                                    stream, ctypes.byref(best), ms)
    return st, best.value, list(ms)


def rd_server_open(ctx, arena_ptr, device_bytes, max_batch=0, max_inflight=0) -> int:
    srv = ctypes.c_void_p()
    cfg = rd_server_config(int(device_bytes), int(max_batch), int(max_inflight))
    st = load_library().rd_server_open(ctx, arena_ptr, ctypes.byref(cfg), ctypes.byref(srv))
    if st != RD_OK:
        raise RdError(st, "rd_server_open failed")
    return srv.value


def rd_server_submit(srv, grid, events_ptr, n_events) -> int:
    t = ctypes.c_uint64()
    g = _grid(grid)
    st = load_library().rd_server_submit(srv, ctypes.byref(g), events_ptr, n_events, ctypes.byref(t))
    if st != RD_OK:
        raise RdError(st, "rd_server_submit failed")
    return t.value


def rd_server_wait(srv, ticket, out_ptr, capacity) -> tuple[int, rd_request_info]:
    info = rd_request_info()
    st = load_library().rd_server_wait(srv, ticket, out_ptr, capacity, ctypes.byref(info))
    return st, info


def rd_server_stats(srv) -> tuple[int, int]:
    p, r = ctypes.c_uint64(), ctypes.c_uint64()
    load_library().rd_server_stats(srv, ctypes.byref(p), ctypes.byref(r))
    return p.value, r.value


def rd_server_close(srv) -> int:
    return load_library().rd_server_close(srv)


def rd_trace_free(ctx, trace) -> int:
    return load_library().rd_trace_free(ctx, trace)


def rd_trace_stats(ctx, trace) -> dict:
    """Figures of the trace's last check (see rd_stats in include/rd.h) as a dict."""
    out = rd_stats()
    st = load_library().rd_trace_stats(ctx, trace, ctypes.byref(out))
    if st != RD_OK:
        raise RdError(st, "rd_trace_stats failed")
    d = {name: getattr(out, name) for name, _ in rd_stats._fields_}
    d["kind_count"] = list(out.kind_count)
    return d


def rd_strerror(status: int) -> str:
    return load_library().rd_strerror(status).decode()


def rd_last_error(ctx) -> tuple[int, str]:
    idx = ctypes.c_uint64()
    buf = ctypes.create_string_buffer(256)
    load_library().rd_last_error(ctx, ctypes.byref(idx), buf, 256)
    v = idx.value
    return (-1 if v == (1 << 64) - 1 else v), buf.value.decode()


# ---------------------------------------------------------------- convenience wrapper

class CheckResult:
    def __init__(self, status, pairs, bad_index=-1, message=""):
        self.status = status
        self.pairs = pairs
        self.bad_index = bad_index
        self.message = message

    def __repr__(self):
        return f"CheckResult(status={self.status}, bad_index={self.bad_index}, n_pairs={len(self.pairs)})"


class RaceChecker:
    """One context on a HIP device; check() runs the whole pipeline on the current torch stream."""

    def __init__(self, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the race checker needs a HIP device")
        self.torch = torch
        self.device = device
        self.ctx = rd_init(device)
        self._report_len = {}  # trace handle -> length of its last report
        _open.add(self)

    def close(self):
        if self.ctx:
            rd_shutdown(self.ctx)
            self.ctx = None

    def __del__(self):
        # during interpreter shutdown (module globals may already be gone) no HIP call is made: the
        # exit handler has closed the context while the runtime was alive
        try:
            if sys.is_finalizing():
                return
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, grid, n_events, limits=None):
        return rd_workspace_bytes(self.ctx, grid, n_events, limits)

    def prepare(self, grid, events, limits=None, workspace=None):
        """Binds events (numpy (N,4) uint32 on the host, or a torch tensor (N,4) int32/uint32 on the
        device) to a workspace.  Returns (trace handle, workspace tensor, events tensor or None)."""
        torch = self.torch
        n = int(events.shape[0])
        nbytes = self.workspace_bytes(grid, n, limits)
        if workspace is None or workspace.numel() < nbytes:
            workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
        stream = torch.cuda.current_stream(self.device).cuda_stream
        keep = None
        if isinstance(events, np.ndarray):
            ev = np.ascontiguousarray(events, dtype=np.uint32)
            keep = ev
            st, tr = rd_trace_upload(self.ctx, grid, ev.ctypes.data if n else None, n, 0, workspace.data_ptr(),
                                     workspace.numel(), limits, stream)
        else:
            ev = events.contiguous()
            keep = ev
            st, tr = rd_trace_upload(self.ctx, grid, ev.data_ptr() if n else None, n, 1, workspace.data_ptr(),
                                     workspace.numel(), limits, stream)
        if st != RD_OK:
            raise RdError(st, f"rd_trace_upload: {rd_last_error(self.ctx)[1]}")
        return tr, workspace, keep

    def run(self, trace, capacity=None):
        stream = self.torch.cuda.current_stream(self.device).cuda_stream
        st = rd_check(self.ctx, trace, stream)
        if st != RD_OK:
            raise RdError(st, f"rd_check: {rd_last_error(self.ctx)[1]}")
        return self.report(trace, capacity)

    def report(self, trace, capacity=None):
        if capacity is None:
            # one call into a new array sized by the trace's previous report (the pairs are written
            # straight into the array that is returned); a second one only when they do not fit
            buf = np.empty((max(self._report_len.get(trace, 0), 1 << 12), 2), dtype=np.uint32)
            st, n = rd_races(self.ctx, trace, buf.ctypes.data, len(buf))
            if st == RD_ETRUNC and n > len(buf):
                buf = np.empty((n, 2), dtype=np.uint32)
                st, n = rd_races(self.ctx, trace, buf.ctypes.data, len(buf))
            if st != RD_OK:
                idx, msg = rd_last_error(self.ctx)
                return CheckResult(st, np.zeros((0, 2), np.uint32), idx, msg)
            self._report_len[trace] = n
            return CheckResult(st, buf[:n])
        st, n = rd_races(self.ctx, trace, None, 0)
        if st not in (RD_OK, RD_ETRUNC):
            idx, msg = rd_last_error(self.ctx)
            return CheckResult(st, np.zeros((0, 2), np.uint32), idx, msg)
        out = np.zeros((max(capacity, 1), 2), dtype=np.uint32)
        st, n = rd_races(self.ctx, trace, out.ctypes.data, capacity)
        if st not in (RD_OK, RD_ETRUNC):
            idx, msg = rd_last_error(self.ctx)
            return CheckResult(st, np.zeros((0, 2), np.uint32), idx, msg)
        return CheckResult(st, out[: min(capacity, n)].copy())

    def check_many(self, items, limits=None, batch_limits=None, workspace=None):
        """Batched form: items = [(grid, events), ...]; one rd_check_many over all of them, then
        one report per item, in order.  Returns a list of CheckResult."""
        torch = self.torch
        bound = [self.prepare(g, ev, limits) for g, ev in items]
        traces = [b[0] for b in bound]
        try:
            nbytes = rd_batch_workspace_bytes(self.ctx, traces, batch_limits)
            if workspace is None or workspace.numel() < nbytes:
                workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
            stream = torch.cuda.current_stream(self.device).cuda_stream
            st = rd_check_many(self.ctx, traces, workspace.data_ptr(), workspace.numel(), batch_limits, stream)
            if st != RD_OK:
                raise RdError(st, f"rd_check_many: {rd_last_error(self.ctx)[1]}")
            return self.report_many(traces)
        finally:
            for t in traces:
                rd_trace_free(self.ctx, t)
                self._report_len.pop(t, None)
            del bound, workspace

    def kinds(self, trace, capacity=None):
        """Unique race kinds of a checked trace: (status, (K, 3) uint32 array of (site_lo, site_hi,
        count)), ascending; capacity None returns them all."""
        if capacity is None:
            # one call into a buffer of 4096 kinds; a second one only when they do not fit
            out = np.zeros((4096, 3), dtype=np.uint32)
            st, n = rd_race_kinds(self.ctx, trace, out.ctypes.data, len(out))
            if st == RD_ETRUNC and n > len(out):
                out = np.zeros((n, 3), dtype=np.uint32)
                st, n = rd_race_kinds(self.ctx, trace, out.ctypes.data, len(out))
            if st != RD_OK:
                return st, np.zeros((0, 3), dtype=np.uint32)
            return st, out[:n].copy()
        out = np.zeros((max(capacity, 1), 3), dtype=np.uint32)
        st, n = rd_race_kinds(self.ctx, trace, out.ctypes.data if capacity else None, capacity)
        return st, out[: min(capacity, n)].copy()

    def lockset(self, trace, capacity=1 << 16):
        """The lockset pass over a bound trace: CheckResult with the sorted pairs (the pass runs again
        with room for every pair when `capacity` is too small)."""
        out = np.zeros((max(capacity, 1), 2), dtype=np.uint32)
        st, n = rd_lockset(self.ctx, trace, out.ctypes.data, capacity)
        if st == RD_ETRUNC:
            out = np.zeros((max(n, 1), 2), dtype=np.uint32)
            st, n = rd_lockset(self.ctx, trace, out.ctypes.data, n)
        if st != RD_OK:
            idx, msg = rd_last_error(self.ctx)
            return CheckResult(st, np.zeros((0, 2), np.uint32), idx, msg)
        return CheckResult(st, out[:n].copy())

    def gwcp(self, trace, capacity=1 << 16):
        """The GWCP pass over a bound trace: CheckResult with the sorted pairs (the pass runs again
        with room for every pair when `capacity` is too small)."""
        out = np.zeros((max(capacity, 1), 2), dtype=np.uint32)
        st, n = rd_gwcp(self.ctx, trace, out.ctypes.data, capacity)
        if st == RD_ETRUNC:
            out = np.zeros((max(n, 1), 2), dtype=np.uint32)
            st, n = rd_gwcp(self.ctx, trace, out.ctypes.data, n)
        if st != RD_OK:
            idx, msg = rd_last_error(self.ctx)
            return CheckResult(st, np.zeros((0, 2), np.uint32), idx, msg)
        return CheckResult(st, out[:n].copy())

    def report_many(self, traces):
        """Reports of several checked traces through rd_races_many (one transfer per batch); a member
        whose status is an error is reported again through rd_races for its error details."""
        st, counts, sts = rd_races_many(self.ctx, traces, None, 0)
        total = int(counts[(sts == RD_OK) | (sts == RD_ETRUNC)].sum()) if len(traces) else 0
        out = np.zeros((max(total, 1), 2), dtype=np.uint32)
        st, counts, sts = rd_races_many(self.ctx, traces, out.ctypes.data, total)
        res, used = [], 0
        for t, c, s in zip(traces, counts, sts):
            c, s = int(c), int(s)
            if s == RD_OK:
                res.append(CheckResult(s, out[used: used + c].copy()))
                used += c
            else:
                res.append(self.report(t))
        return res

    def check(self, grid, events, limits=None, capacity=None):
        tr, ws, keep = self.prepare(grid, events, limits)
        try:
            return self.run(tr, capacity)
        finally:
            rd_trace_free(self.ctx, tr)
            self._report_len.pop(tr, None)
            del ws, keep


class Server:
    """Served form on a RaceChecker's device: ``submit`` (host events, kept alive here until answered)
    returns a ticket; ``wait`` returns (CheckResult, rd_request_info).  The arena is a torch
    allocation of ``budget_bytes`` made once at open."""

    def __init__(self, checker: RaceChecker, budget_bytes: int, max_batch: int = 0, max_inflight: int = 0):
        torch = checker.torch
        self.checker = checker
        self.arena = torch.empty(budget_bytes, dtype=torch.uint8, device=f"cuda:{checker.device}")
        self.srv = rd_server_open(checker.ctx, self.arena.data_ptr(), budget_bytes, max_batch, max_inflight)
        self._keep = {}
        _open.add(self)

    def submit(self, grid, events) -> int:
        ev = np.ascontiguousarray(events, dtype=np.uint32)
        n = int(ev.shape[0])
        t = rd_server_submit(self.srv, grid, ev.ctypes.data if n else None, n)
        self._keep[t] = ev
        return t

    def wait(self, ticket, capacity=1 << 20):
        out = np.zeros((max(capacity, 1), 2), dtype=np.uint32)
        st, info = rd_server_wait(self.srv, ticket, out.ctypes.data, capacity)
        self._keep.pop(ticket, None)
        n = int(info.n_races)
        bad = -1 if info.bad_index == (1 << 64) - 1 else int(info.bad_index)
        return CheckResult(st, out[: min(n, capacity)].copy() if st in (RD_OK, RD_ETRUNC) else
                           np.zeros((0, 2), np.uint32), bad), info

    def stats(self):
        return rd_server_stats(self.srv)

    def close(self):
        if self.srv:
            rd_server_close(self.srv)
            self.srv = None
            self._keep.clear()
            del self.arena
