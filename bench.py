"""Throughput of the scoped happens-before race check on one MI355X.

A step is one whole check of one trace: rd_check (every stage of the pipeline, on the device) and
rd_races (the report: pair sort on the device and the copy of the canonical pairs to the host).
Events are resident in HBM when the timed region starts.

With no --workload, every workload runs in one process and one JSON line reports them all:
  * the headline (`value`) is the largest single-GPU workload, the stencil-and-reduction trace
    (4096 blocks x 256 threads, 268,508,160 events, halo flags and a 4,096-section device lock),
    checked against the CPU oracle over the whole trace;
  * beside it (`configs`): the single large trace (1024 x 256 threads, 16,777,216 events, Zipf 1.1),
    the batched form (512 traces of uneven length, one captured graph launch vs one check per
    trace) and the served form (Poisson arrivals through the request loop under a 64 GiB budget,
    plus a saturating run of the same requests).
Per plain workload: K timed steps in 5 trials (median reported too), the dominant kernel's launch
time measured live with HIP events on its stream, the method's own bytes per check (16 B per
record, 32 B per distinct location, 8 B per race pair) over the dominant kernel's and the whole
check's time against the 8 TB/s HBM peak, HBM bytes per check from rocprofv3 counters where the
stored figures were taken on the current sources, end-to-end time with the upload from host
memory, and the oracle timed on this host over a bounded sample.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "memory events checked/sec (bit-exact race set) and % of HBM peak; batched vs plain"
ACCESS_KINDS = (0, 1, 2, 6, 7)
COUNTERS_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def say(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def source_digest() -> str:
    """Digest of every kernel source: stored counter figures are used only for the kernels they
    measured."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2111_12478_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            h.update(open(os.path.join(csrc, f), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "rd.h"), "rb").read())
    return h.hexdigest()[:16]


def distinct_locations(ev: np.ndarray, tpb: int) -> int:
    """Distinct locations the trace accesses: global words, and shared words of each block."""
    kind = ev[:, 2] & 15
    acc = np.isin(kind, ACCESS_KINDS)
    sh = ((ev[:, 2] >> 6) & 1) == 1
    g = ev[acc & ~sh, 0]
    n = 0
    if len(g):
        lo, hi = int(g.min()), int(g.max())
        if hi - lo < (1 << 30):
            seen = np.zeros(hi - lo + 1, dtype=np.bool_)
            seen[g - lo] = True
            n += int(np.count_nonzero(seen))
        else:
            n += int(len(np.unique(g)))
    m = acc & sh
    if m.any():
        key = (ev[m, 1].astype(np.uint64) // tpb) << np.uint64(32) | ev[m, 0].astype(np.uint64)
        n += int(len(np.unique(key)))
    return n


def method_bytes(n_events: int, locations: int, pairs: int) -> int:
    """What the method itself must move per check, independent of how it is computed: each record
    read once (16 B), one shadow summary per distinct location read and written (32 B), each race
    pair written (8 B)."""
    return 16 * n_events + 32 * locations + 8 * pairs


def sort_own_bytes(n_acc: int, packed: bool) -> int:
    """One pass of the location sort over its own arrays: each element read and written once
    (12 B per element when category and phase ride in the key or the thread word, else 16 B)."""
    return 2 * (12 if packed else 16) * n_acc


class KT(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_uint32), ("total_ms", ctypes.c_double)]


def _lib():
    import paper_2111_12478_amd as rd
    lib = rd.load_library()
    lib.rd_profile_enable.argtypes = [ctypes.c_void_p, ctypes.c_char_p]
    lib.rd_profile_read.argtypes = [ctypes.c_void_p, ctypes.POINTER(KT), ctypes.c_uint32,
                                    ctypes.POINTER(ctypes.c_uint32)]
    return lib


def read_profile(lib, ctx) -> dict:
    buf = (KT * 128)()
    cnt = ctypes.c_uint32()
    lib.rd_profile_read(ctx, buf, 128, ctypes.byref(cnt))
    return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms) for i in range(cnt.value)}


def merge_sort_passes(prof: dict, passes: int) -> dict:
    """The location sort runs one sweep per key digit: its passes count as one kernel; a pass past
    the key width (it exits at once) is left out."""
    names = {f"k_sort_sweep_p{p}" for p in range(passes)}
    out = {}
    for k, (c, ms) in prof.items():
        if k.startswith("k_sort_sweep_p"):
            if k not in names:
                continue
            k = "k_sort_sweep"
        c0, m0 = out.get(k, (0, 0.0))
        out[k] = (c0 + c, m0 + ms)
    return out


def stored_counters(workload: str, n_events: int, variant: int):
    """HBM bytes per check and per launch of each kernel from the rocprofv3 counter runs stored
    under profiles/, if they were taken on the current sources, this workload and sort variant."""
    try:
        t = json.load(open(COUNTERS_FILE))
    except (OSError, ValueError):
        return None
    if t.get("source_digest") != source_digest():
        return None
    w = t.get("workloads", {}).get(workload)
    if not w or w.get("events") != n_events or w.get("sort_variant") != variant:
        return None
    return w


def trials_of(steps: int) -> list[int]:
    """Steps per trial: five trials (as the paper averages five runs), fewer when K < 5."""
    k = min(5, steps)
    return [steps // k + (1 if i < steps % k else 0) for i in range(k)]


def plain_workload(args, rc, label: str, title: str, grid, ev: np.ndarray, limits: dict, oracle_fn=None,
                   cpu_sample=None, extra=None) -> dict:
    """Times K checks of one resident trace; returns the workload's JSON object.  oracle_fn() gives
    the oracle's report for parity (None: skipped); cpu_sample = (events, seconds, what) of the
    oracle on a bounded sample."""
    import torch
    import paper_2111_12478_amd as rd
    lib = _lib()
    n = int(ev.shape[0])
    dev_ev = torch.from_numpy(ev.view(np.int32)).cuda()
    tr, ws, keep = rc.prepare(grid, dev_ev, limits)
    res = rc.run(tr)
    if res.status != 0:
        raise RuntimeError(f"{label}: check failed: {res} {res.message}")
    tune_ms = None
    if args.sort_variant is not None:
        rd.rd_set_tuning(rc.ctx, args.sort_variant)
    elif not args.no_tune:
        st, best, tune_ms = rd.rd_autotune(rc.ctx, [tr], None, 0, torch.cuda.current_stream().cuda_stream)
        if st != rd.RD_OK:
            raise RuntimeError(f"rd_autotune failed: {st}")
    variant = rd.rd_get_tuning(rc.ctx)
    rb, waves, items = rd.rd_tuning_get(variant)
    say(f"{label}: {n:,} events resident, sort variant {variant} ({rb}-bit digits, {waves} waves x {items})")

    def step():
        r = rc.run(tr)
        if r.status != 0:
            raise RuntimeError(f"{label}: check failed: {r}")
        return r

    for _ in range(args.warmup):
        res = step()
    stats = rd.rd_trace_stats(rc.ctx, tr)
    passes = -(-stats["key_bits"] // rb) if stats["key_bits"] else 0
    # one profiled step finds the dominant kernel
    lib.rd_profile_enable(rc.ctx, b"*")
    step()
    prof = merge_sort_passes(read_profile(lib, rc.ctx), passes)
    lib.rd_profile_enable(rc.ctx, None)
    dom = max(prof.items(), key=lambda kv: kv[1][1])[0]
    if args.profile_all:
        for k, (c, ms) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
            say(f"  {k:28s} launches={c:3d} total={ms:8.3f} ms")

    # timed region: K steps in trials, the dominant kernel bracketed by HIP events on its stream
    # (recorded around its piece of the check's graph, which one untimed step captures)
    filt = b"k_sort_sweep_p*" if dom == "k_sort_sweep" else dom.encode()
    lib.rd_profile_enable(rc.ctx, filt)
    step()
    lib.rd_profile_enable(rc.ctx, filt)
    trial_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in trials_of(args.steps):
        a = time.perf_counter()
        for _ in range(k):
            res = step()
        torch.cuda.synchronize()
        trial_ms.append((time.perf_counter() - a) * 1e3 / k)
    t1 = time.perf_counter()
    kp = merge_sort_passes(read_profile(lib, rc.ctx), passes)
    lib.rd_profile_enable(rc.ctx, None)
    launches, total_ms = kp.get(dom, (0, 0.0))
    if dom == "k_sort_sweep":
        # one pair of events brackets the sweeps of a check (the empty passes past the key width
        # included): only the real passes count as launches
        launches = passes * args.steps
    avg_s = total_ms / max(1, launches) / 1e3
    elapsed = t1 - t0
    per = elapsed / args.steps
    pairs = res.pairs
    locations = distinct_locations(ev, grid[1])
    alg = method_bytes(n, locations, len(pairs))
    n_acc = int(stats["n_accesses"])
    counters = stored_counters(label, n, variant)
    traffic = counters["per_launch"].get(dom) if counters else None
    roof = {
        "bound": "hbm",
        "kernel": dom,
        "achieved": alg / avg_s / 1e9 if avg_s > 0 else 0.0,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": (alg / avg_s / 1e9) / HBM_PEAK_GBS if avg_s > 0 else 0.0,
        "traffic": traffic,
        "algorithmic_bytes_per_launch": alg,
        "algorithmic_bytes_per_event": alg / n,
        "avg_launch_ms": avg_s * 1e3,
        "launches": launches,
    }
    if dom == "k_sort_sweep":
        own = sort_own_bytes(n_acc, bool(stats["packed"]))
        roof["kernel_own_bytes_per_launch"] = own
        roof["kernel_own_frac"] = own / avg_s / 1e9 / HBM_PEAK_GBS
    pipe = {
        "algorithmic_bytes": alg,
        "algorithmic_bytes_per_event": alg / n,
        "algorithmic_gbs": alg / per / 1e9,
        "frac": alg / per / 1e9 / HBM_PEAK_GBS,
        "distinct_locations": locations,
    }
    if counters:
        cb = counters["per_check"]
        pipe.update({"counter_bytes": cb, "counter_bytes_per_event": cb / n, "counter_gbs": cb / per / 1e9,
                     "counter_frac": cb / per / 1e9 / HBM_PEAK_GBS})
    else:
        pipe.update({"counter_bytes": None, "counter_gbs": None, "counter_frac": None})
    kernels = sorted(((ms, k, c) for k, (c, ms) in prof.items()), reverse=True)[:8]

    # end to end: the events copied from page-locked host memory into the workspace, then the
    # check and the report (the first check of a bound trace runs kernel by kernel)
    e2e = []
    rd.rd_trace_free(rc.ctx, tr)
    rc._report_len.pop(tr, None)
    host = torch.from_numpy(ev.view(np.int32)).pin_memory()
    stream = torch.cuda.current_stream().cuda_stream
    for _ in range(3):
        torch.cuda.synchronize()
        a = time.perf_counter()
        st, tr2 = rd.rd_trace_upload(rc.ctx, grid, host.data_ptr(), n, 0, ws.data_ptr(), ws.numel(), limits, stream)
        if st != rd.RD_OK:
            raise RuntimeError(f"{label}: upload failed {st}")
        r2 = rc.run(tr2)
        e2e.append(time.perf_counter() - a)
        rd.rd_trace_free(rc.ctx, tr2)
        rc._report_len.pop(tr2, None)
        if r2.status != 0 or not np.array_equal(r2.pairs, pairs):
            raise RuntimeError(f"{label}: end-to-end check differs")
    del host, dev_ev, ws, keep

    out = {
        "value": n / per,
        "unit": "events/s",
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": per * 1e3,
        "trial_ms_per_step": trial_ms,
        "median_ms_per_step": float(np.median(trial_ms)),
        "median_events_per_s": n / (float(np.median(trial_ms)) / 1e3),
        "access_events_per_s": n_acc / per,
        "end_to_end": {"ms": float(np.median(e2e)) * 1e3, "events_per_s": n / float(np.median(e2e)),
                       "what": "events copied from page-locked host memory, check, report (median of 3)"},
        "config": {"workload": title, "events": n, "accesses": n_acc, "race_pairs": int(len(pairs)),
                   "key_bits": stats["key_bits"], "sort_passes": passes, "packed_elements": ["no", "key word", "thread word"][int(stats["packed"])],
                   "sort_variant": {"index": variant, "digit_bits": rb, "waves": waves, "items": items,
                                    "autotune_ms": tune_ms}},
        "roofline": roof,
        "pipeline": pipe,
        "top_kernels_ms": [[k, round(ms, 4), c] for ms, k, c in kernels],
        "memory": {"workspace_bytes": stats["workspace_bytes"], "clock_vectors": stats["clock_vectors"],
                   "clock_words": stats["clock_words"], "clock_bytes": stats["clock_bytes"],
                   "dense_clock_bytes": stats["dense_clock_bytes"],
                   "engine": ["none", "parallel", "interpreter"][stats["engine"]],
                   "engine_ops": stats["engine_ops"], "engine_groups": stats["engine_groups"]},
    }
    if extra:
        out["config"].update(extra(pairs))
    if cpu_sample is not None:
        m, secs, what = cpu_sample
        out["cpu_baseline"] = {"value": m / secs, "unit": "events/s", "cores": 1, "kind": "oracle",
                               "sample": what, "cpu_model": cpu_model()}
    if oracle_fn is not None:
        out["parity"] = parity_of(pairs, oracle_fn())
    return out, pairs


def parity_of(pairs, want) -> str:
    return ("bit-exact, whole trace" if want is not None and np.array_equal(want, pairs) else
            f"MISMATCH gpu={len(pairs)} oracle={None if want is None else len(want)}")


def oracle_prefix(grid, ev, m: int):
    """The oracle on the first m events (a prefix of a valid trace is valid); (pairs, seconds)."""
    import oracle
    sub = np.ascontiguousarray(ev[:m])
    c0 = time.perf_counter()
    r = oracle.check(grid, sub)
    return r, time.perf_counter() - c0


def _oracle_child(conn, grid, ev):
    import oracle
    r = oracle.check(grid, ev)
    conn.send((r.status, r.pairs))
    conn.close()


def background_oracle(grid, ev):
    """Starts the oracle over the whole trace in a forked process (before this process touches the
    GPU); returns a function that waits for its report."""
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    a, b = ctx.Pipe(duplex=False)
    p = ctx.Process(target=_oracle_child, args=(b, grid, ev), daemon=True)
    p.start()
    b.close()

    def wait():
        try:
            st, pairs = a.recv()
        except EOFError:
            p.join()
            return None
        p.join()
        return pairs if st == 0 else None
    return wait


# ---------------------------------------------------------------- workloads

def stencil_inputs(args):
    import tracegen
    cfg = tracegen.stencil()
    if args.scale > 1:
        cfg = tracegen.StencilConfig(rb=max(1, cfg.rb // args.scale), cb=cfg.cb, tpb=cfg.tpb, rows=cfg.rows,
                                     sweeps=cfg.sweeps, pitch=cfg.pitch, group=cfg.group,
                                     plant_rate=cfg.plant_rate * args.scale, seed=cfg.seed)
    t0 = time.perf_counter()
    grid, ev, gst, plants = tracegen.generate_stencil(cfg)
    say(f"stencil: {len(ev):,} events generated in {time.perf_counter() - t0:.1f} s, {len(plants)} plants")
    return cfg, grid, ev, plants


def _plants_missing(cfg, grid, ev, pairs, plants):
    """Planted downgrades that do not show up: a fence pair as a race between the neighbour block
    (first) and the acquiring block (second), a lock pair as a race of the section's block on the
    accumulator or the lock word."""
    tpb = grid[1]
    if len(pairs) == 0:
        return len(plants)
    fb = ev[pairs[:, 0], 1] // tpb
    sb = ev[pairs[:, 1], 1] // tpb
    have = set(zip(fb.tolist(), sb.tolist()))
    lock_second = set(sb[np.isin(ev[pairs[:, 1], 0], ev[pairs[:, 0], 0])].tolist())
    missing = 0
    for kind, b, s, d in plants.tolist():
        if kind == 0:
            r, c = divmod(b, cfg.cb)
            nb = [(r - 1) * cfg.cb + c, (r + 1) * cfg.cb + c, r * cfg.cb + c - 1, r * cfg.cb + c + 1][d]
            missing += (nb, b) not in have
        else:
            missing += b not in lock_second
    return missing


def run_stencil(args, rc, inputs, cpu_sample):
    """The stencil trace; its oracle comparison is made by the caller (the oracle may still run)."""
    cfg, grid, ev, plants = inputs
    n = len(ev)
    title = (f"stencil and reduction, plain method: {grid[0]} blocks x {grid[1]} threads, {n:,} events, "
             f"{cfg.sweeps} sweeps of a 5-point stencil over two {cfg.rb * cfg.rows} x {cfg.cb * cfg.tpb} "
             f"buffers (row pitch {cfg.pitch} words), halo flags, device lock over {grid[0]:,} sections, "
             f"{len(plants)} planted scope downgrades, seed {cfg.seed}")
    limits = {"clock_bytes": int(os.environ.get("RD_CLOCK_BYTES", str(16 << 30)))}
    return plain_workload(args, rc, "stencil", title, grid, ev, limits, oracle_fn=None, cpu_sample=cpu_sample,
                          extra=lambda pairs: {"plants": int(len(plants)),
                                               "plants_missing": _plants_missing(cfg, grid, ev, pairs, plants)})


def run_large(args, rc, with_oracle: bool):
    import tracegen
    cfg = tracegen.large(seed=2, scale=args.scale)
    grid, ev, gstats, plants = tracegen.generate(cfg)
    n = len(ev)
    title = (f"single large trace, plain method: {grid[0]} blocks x {grid[1]} threads, {n:,} events, "
             f"{cfg.n_global + cfg.n_blocks * cfg.n_shared:,} words (Zipf {cfg.zipf_s}), seed {cfg.seed}")
    want = sample = None
    if with_oracle:
        import oracle
        c0 = time.perf_counter()
        r = oracle.check(grid, ev)
        secs = time.perf_counter() - c0
        want = r.pairs if r.status == 0 else None
        sample = (n, secs, f"the whole {n:,}-event trace, one core")
    out, _ = plain_workload(args, rc, "large", title, grid, ev, {"max_pairs": max(1 << 20, n // 4)},
                         oracle_fn=(lambda: want) if with_oracle else None, cpu_sample=sample,
                         extra=lambda pairs: {"plants": int(len(plants))})
    # unique race kinds of the report (site-id pairs: each event's position in its thread's program)
    return out, (grid, ev, want)


def race_kinds_figures(rc, grid, ev, want):
    """rd_race_kinds on the large trace: kinds, wall time per call, parity with the oracle's."""
    import torch
    import oracle
    tr, ws, keep = rc.prepare(grid, torch.from_numpy(ev.view(np.int32)).cuda(), {"max_pairs": max(1 << 20, len(ev) // 4)})
    try:
        res = rc.run(tr)
        st, kinds = rc.kinds(tr)
        torch.cuda.synchronize()
        k0 = time.perf_counter()
        for _ in range(5):
            st, kinds = rc.kinds(tr)
        k1 = time.perf_counter()
        out = {"kinds": int(kinds.shape[0]), "pairs": int(len(res.pairs)), "status": int(st),
               "ms_per_call": (k1 - k0) * 1e3 / 5}
        if want is not None:
            wk = oracle.race_kinds(ev, want)
            out["parity"] = "bit-exact" if np.array_equal(wk, kinds) else f"MISMATCH gpu={len(kinds)} oracle={len(wk)}"
        return out
    finally:
        import paper_2111_12478_amd as rd
        rd.rd_trace_free(rc.ctx, tr)
        rc._report_len.pop(tr, None)


def run_analyses(args, rc, with_oracle: bool) -> dict:
    """The two other analyses over one lock-heavy trace (8 blocks of 256 threads, 32 lock words,
    65,536 data words, nested and fence-inferred critical sections, flag publications, barriers):
    the lockset pass (rd_lockset) and the GWCP
    pass (rd_gwcp), each call a check of its own, the pass and the report copy, timed beside the
    happens-before check of the same trace; parity of both reports with the oracle's."""
    import torch
    import paper_2111_12478_amd as rd
    from tracegen.locktrace import lock_trace
    n_target = max(2_000, 200_000 // args.scale)
    seed = 77
    grid, ev = lock_trace(seed, max_events=n_target, flags=True, barriers=True, grid=(8, 256), locks=32,
                          data_words=max(64, 65536 // args.scale))
    n = int(len(ev))
    title = (f"lock trace: {grid[0]} blocks x {grid[1]} threads, {n:,} events, 32 lock words, "
             f"{max(64, 65536 // args.scale):,} data words, nested and fence-inferred critical sections, "
             f"flag publications, barriers, seed {seed}")
    say(f"analyses: {title}")
    dev_ev = torch.from_numpy(ev.view(np.int32)).cuda()
    # 2,048 threads release: knowledge vectors of 2,056 words, and the GWCP pass keeps a copy of P
    # (2,048 words) per event that changes it
    tr, ws, keep = rc.prepare(grid, dev_ev, {"max_pairs": max(1 << 20, n // 4), "clock_bytes": 8 << 30})
    out = {"workload": title, "events": n, "threads": int(grid[0] * grid[1])}
    try:
        def timed(fn, reps):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                r = fn()
            torch.cuda.synchronize()
            return r, (time.perf_counter() - t0) * 1e3 / reps

        reps = max(1, min(args.steps, 5))
        hb, hb_ms = timed(lambda: rc.run(tr), reps)
        ls, ls_ms = timed(lambda: rc.lockset(tr), reps)
        gw, gw_ms = timed(lambda: rc.gwcp(tr, capacity=1 << 22), min(reps, 2))
        out["happens_before"] = {"ms_per_call": hb_ms, "events_per_s": n / (hb_ms / 1e3), "pairs": int(len(hb.pairs)),
                                 "status": int(hb.status)}
        out["lockset"] = {"ms_per_call": ls_ms, "events_per_s": n / (ls_ms / 1e3), "pairs": int(len(ls.pairs)),
                          "status": int(ls.status), "what": "rd_lockset: a check, the lockset pass, the report copy"}
        out["gwcp"] = {"ms_per_call": gw_ms, "events_per_s": n / (gw_ms / 1e3), "pairs": int(len(gw.pairs)),
                       "status": int(gw.status), "what": "rd_gwcp: a check, the GWCP pass, the report copy"}
        if with_oracle:
            import oracle
            for name, fn, got in (("lockset", oracle.lockset, ls), ("gwcp", oracle.gwcp, gw)):
                c0 = time.perf_counter()
                want = fn(grid, ev)
                secs = time.perf_counter() - c0
                same = want.status == got.status and np.array_equal(want.pairs, got.pairs)
                out[name]["parity"] = "bit-exact" if same else f"MISMATCH gpu={len(got.pairs)} oracle={len(want.pairs)}"
                out[name]["cpu_baseline"] = {"value": n / secs, "unit": "events/s", "cores": 1, "kind": "oracle",
                                             "sample": f"the whole {n:,}-event trace, one core"}
        for name, r in (("happens-before", hb), ("lockset", ls), ("GWCP", gw)):
            if r.status != 0:
                raise RuntimeError(f"analyses: {name} failed: {r}")
        say(f"analyses: happens-before {hb_ms:.2f} ms, lockset {ls_ms:.2f} ms, GWCP {gw_ms:.2f} ms per call")
    finally:
        rd.rd_trace_free(rc.ctx, tr)
        rc._report_len.pop(tr, None)
    return out


def _gen_member(cfg):
    import tracegen
    g, ev, _, _ = tracegen.generate(cfg)
    return g, ev


def _oracle_member(item):
    import oracle
    g, ev = item
    t0 = time.perf_counter()
    r = oracle.check(g, ev)
    return r.status, r.pairs, time.perf_counter() - t0


def run_batched(args, rc, with_oracle: bool) -> dict:
    """512 independent traces (lengths lognormal around 200K events): one rd_check + rd_races per
    trace in turn (plain), one rd_check_many + rd_races_many (batched, eager), and the batched pass
    captured once into a HIP graph and replayed with one launch per step (graph, the headline of
    this workload)."""
    import concurrent.futures as cf
    import torch
    import tracegen
    import paper_2111_12478_amd as rd

    cfgs = tracegen.batch(seed=4, n_traces=args.batch_traces, scale=args.scale)
    workers = min(16, host_cores())
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        items = list(ex.map(_gen_member, cfgs, chunksize=4))
    n_total = sum(int(ev.shape[0]) for _, ev in items)
    say(f"batched: {len(items)} traces, {n_total:,} events generated")
    limits = {"clock_bytes": 16 << 20}
    # a stream of its own: the captured pass is launched on a non-default stream
    side = torch.cuda.Stream()
    ctx_stream = torch.cuda.stream(side)
    ctx_stream.__enter__()
    bound = [rc.prepare(g, torch.from_numpy(ev.view(np.int32)).cuda(), limits) for g, ev in items]
    traces = [b[0] for b in bound]
    bws_bytes = rd.rd_batch_workspace_bytes(rc.ctx, traces, None)
    bws = torch.empty(bws_bytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    say(f"batched: bound, member workspaces {sum(b[1].numel() for b in bound) / 2**30:.1f} GiB, "
        f"batch workspace {bws_bytes / 2**30:.1f} GiB")
    tune_ms = None
    if args.sort_variant is not None:
        rd.rd_set_tuning(rc.ctx, args.sort_variant)
    elif not args.no_tune:
        st, best, tune_ms = rd.rd_autotune(rc.ctx, traces, bws.data_ptr(), bws.numel(), stream)
        if st != rd.RD_OK:
            raise RuntimeError(f"rd_autotune failed: {st}")
    variant = rd.rd_get_tuning(rc.ctx)
    st, graph = rd.rd_batch_capture(rc.ctx, traces, bws.data_ptr(), bws.numel(), None, stream)
    if st != rd.RD_OK:
        raise RuntimeError(f"rd_batch_capture failed: {st}")

    def plain_step():
        return [rc.run(t) for t in traces]

    def eager_step():
        s = rd.rd_check_many(rc.ctx, traces, bws.data_ptr(), bws.numel(), None, stream)
        if s != rd.RD_OK:
            raise RuntimeError(f"rd_check_many failed: {s}")
        return rc.report_many(traces)

    def graph_step():
        s = rd.rd_graph_launch(rc.ctx, graph, stream)
        if s != rd.RD_OK:
            raise RuntimeError(f"rd_graph_launch failed: {s}")
        return rc.report_many(traces)

    def timed(fn, steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, res

    plain_steps = max(1, min(args.steps, 3))
    for _ in range(max(1, min(args.warmup, 2))):
        plain_res = plain_step()
        eager_res = eager_step()
        graph_res = graph_step()
    t_plain, plain_res = timed(plain_step, plain_steps)
    t_eager, eager_res = timed(eager_step, args.steps)
    t_graph, graph_res = timed(graph_step, args.steps)
    say(f"batched: plain {t_plain * 1e3:.2f}, eager {t_eager * 1e3:.2f}, graph {t_graph * 1e3:.2f} ms/step")
    same = all(a.status == b.status == c.status == 0 and np.array_equal(a.pairs, b.pairs) and
               np.array_equal(a.pairs, c.pairs) for a, b, c in zip(plain_res, eager_res, graph_res))
    n_pairs = sum(len(r.pairs) for r in graph_res)
    out = {
        "value": n_total / t_graph,
        "unit": "events/s",
        "steps": args.steps,
        "ms_per_step": t_graph * 1e3,
        "config": {
            "workload": f"batched form: {len(items)} traces, lengths lognormal(median 204,800, sigma 1) in "
                        f"[10,240, 4,194,304], 2^U{{6..11}} blocks x 128|256 threads, mix of the large trace, "
                        f"seed 4; one captured graph launch (rd_batch_capture / rd_graph_launch) + rd_races_many",
            "events": n_total, "race_pairs": int(n_pairs),
            "sort_variant": {"index": variant, "autotune_ms": tune_ms}},
        "plain": {"value": n_total / t_plain, "ms_per_step": t_plain * 1e3, "steps": plain_steps,
                  "form": "one rd_check + rd_races per trace, in turn, same resident events"},
        "eager_batched": {"value": n_total / t_eager, "ms_per_step": t_eager * 1e3,
                          "form": "one rd_check_many + rd_races_many (launched kernel by kernel)"},
        "batched_vs_plain": t_plain / t_graph,
        "batched_equals_plain": bool(same),
        "pipeline": {"algorithmic_bytes_per_event": None},
    }
    locs = sum(distinct_locations(ev, g[1]) for g, ev in items)
    alg = method_bytes(n_total, locs, n_pairs)
    out["pipeline"] = {"algorithmic_bytes": alg, "algorithmic_bytes_per_event": alg / n_total,
                       "algorithmic_gbs": alg / t_graph / 1e9, "frac": alg / t_graph / 1e9 / HBM_PEAK_GBS}
    if with_oracle:
        rng = np.random.default_rng(4)
        sample, budget = [], 0
        for j in rng.permutation(len(items)):
            if budget + int(items[j][1].shape[0]) > 40_000_000:
                continue
            sample.append(int(j))
            budget += int(items[j][1].shape[0])
        c0 = time.perf_counter()
        with cf.ProcessPoolExecutor(max_workers=workers) as ex:
            res = list(ex.map(_oracle_member, [items[j] for j in sample], chunksize=1))
        c1 = time.perf_counter()
        ok = all(st == 0 and np.array_equal(p, graph_res[j].pairs) for j, (st, p, _) in zip(sample, res))
        out["cpu_baseline"] = {"value": budget / (c1 - c0), "unit": "events/s", "cores": workers, "kind": "oracle",
                               "sample": f"{len(sample)} of the {len(items)} traces ({budget:,} events), one trace "
                                         f"per process", "cpu_model": cpu_model()}
        out["parity"] = ("bit-exact: every member equal to its plain check; the oracle on "
                         f"{len(sample)} members ({budget / n_total:.1%} of the events)") if ok and same else "MISMATCH"
    rd.rd_graph_free(rc.ctx, graph)
    for t in traces:
        rd.rd_trace_free(rc.ctx, t)
        rc._report_len.pop(t, None)
    torch.cuda.synchronize()
    ctx_stream.__exit__(None, None, None)
    del bound, bws
    return out


def _served_cfg(i, n):
    import tracegen
    return tracegen.MixConfig(n_blocks=max(1, -(-n // 16384)), tpb=256, n_events=n, n_global=max(16, (n // 16) * 4 // 5),
                              n_shared=max(1, (n // 16 - (n // 16) * 4 // 5) // max(1, -(-n // 16384))),
                              zipf_s=1.1, p_write=0.30, p_atomic_block=0.01, p_atomic_device=0.01, bar_period=64,
                              fence_period=512, plant_rate=1e-4, p_plant_same_block=0.5, plant_victim_cap=256,
                              frac_ro=0.3, frac_da=0.05, frac_priv=0.7, frac_pro=0.25, p_read_ro=0.3, seed=5,
                              trace_index=i)


def run_served(args, rc, with_oracle: bool) -> dict:
    """Poisson arrivals (rate, window) of check requests with sizes log-uniform on [102,400,
    8,388,608] events (256 threads per block, one block per 16,384 events, the mix of the large
    trace, seed 5; events in page-locked host memory), answered by the request loop under a 64 GiB
    arena: open loop for latency, then
    the same requests submitted at once (saturated) for capacity; both again with one request per
    pass and one pass in flight (plain).  Requests draw their traces from a pool of distinct
    generated traces."""
    import concurrent.futures as cf
    import threading
    import torch
    import paper_2111_12478_amd as rd

    rng = np.random.default_rng(5)
    n_req = int(rng.poisson(args.served_rate * args.served_seconds))
    arrivals = np.sort(rng.uniform(0.0, args.served_seconds, n_req))
    sizes = np.exp(rng.uniform(np.log(102_400), np.log(8_388_608), args.served_distinct)).astype(np.int64)
    pick = rng.integers(0, args.served_distinct, n_req)
    cfgs = [_served_cfg(i, int(sizes[i]) // args.scale) for i in range(args.served_distinct)]
    workers = min(16, host_cores())
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        pool = list(ex.map(_gen_member, cfgs, chunksize=1))
    # the requests' events in page-locked host memory (as a serving front end would receive them),
    # so the copies into the arena run at the link's rate
    pinned = [torch.from_numpy(ev.view(np.int32)).pin_memory() for _, ev in pool]
    pool = [(g, t.numpy().view(np.uint32)) for (g, _), t in zip(pool, pinned)]
    say(f"served: {n_req} requests over {args.served_seconds:.0f} s from {len(pool)} distinct traces")
    alone = [rc.check(g, ev) for g, ev in pool]  # each distinct trace checked alone (plain)
    budget = 64 << 30

    def run(max_batch, max_inflight, open_loop):
        srv = rd.Server(rc, budget, max_batch=max_batch, max_inflight=max_inflight)
        tickets = [None] * n_req
        results = [None] * n_req
        ready = [threading.Event() for _ in range(n_req)]

        def submitter():
            t0 = time.perf_counter()
            for i in range(n_req):
                if open_loop:
                    d = arrivals[i] - (time.perf_counter() - t0)
                    if d > 0:
                        time.sleep(d)
                tickets[i] = srv.submit(*pool[pick[i]])
                ready[i].set()

        def waiter():
            for i in range(n_req):
                ready[i].wait()
                results[i] = srv.wait(tickets[i])

        ts = threading.Thread(target=submitter)
        tw = threading.Thread(target=waiter)
        ts.start(); tw.start(); ts.join(); tw.join()
        passes, done = srv.stats()
        srv.close()
        lat = np.array([r[1].done_s - r[1].submit_s for r in results])
        t_first = min(r[1].submit_s for r in results)
        t_last = max(r[1].done_s for r in results)
        ok = all(r[0].status == 0 and np.array_equal(r[0].pairs, alone[pick[i]].pairs) for i, r in enumerate(results))
        return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "events_per_s": float(sum(int(pool[j][1].shape[0]) for j in pick) / (t_last - t_first)),
                "makespan_s": float(t_last - t_first), "passes": int(passes), "same_as_alone": bool(ok)}

    served = run(256, 2, True)
    say(f"served (open loop): {served}")
    plain = run(1, 1, True)
    say(f"plain (open loop, one request per pass): {plain}")
    served_sat = run(256, 2, False)
    say(f"served (saturated): {served_sat}")
    plain_sat = run(1, 1, False)
    say(f"plain (saturated): {plain_sat}")
    n_events = int(sum(int(pool[j][1].shape[0]) for j in pick))
    out = {
        "value": served_sat["events_per_s"],
        "unit": "events/s",
        "ms_per_step": served_sat["makespan_s"] * 1e3,
        "config": {
            "workload": f"served form: Poisson {args.served_rate:.0f} req/s for {args.served_seconds:.0f} s "
                        f"({n_req} requests, {n_events:,} events), sizes log-uniform [102,400, 8,388,608], "
                        f"{args.served_distinct} distinct traces, 64 GiB arena, seed 5; value = capacity with every "
                        f"request submitted at once",
            "requests": n_req, "events": n_events},
        "served_open_loop": served,
        "plain_open_loop": plain,
        "served_saturated": served_sat,
        "plain_saturated": plain_sat,
        "capacity_served_vs_plain": served_sat["events_per_s"] / plain_sat["events_per_s"],
        "offered_events_per_s": n_events / args.served_seconds,
    }
    same = served["same_as_alone"] and plain["same_as_alone"] and served_sat["same_as_alone"] and plain_sat["same_as_alone"]
    if with_oracle:
        # every distinct trace with a pair (all of them, by the plants) against the oracle; every
        # request's answer equals its trace checked alone, so this covers every request
        need = [j for j in range(len(pool)) if len(alone[j].pairs) > 0]
        with cf.ProcessPoolExecutor(max_workers=workers) as ex:
            res = list(ex.map(_oracle_member, [pool[j] for j in need], chunksize=1))
        ok = all(st == 0 and np.array_equal(p, alone[j].pairs) for j, (st, p, _) in zip(need, res))
        covered = float(np.isin(pick, need).mean()) if n_req else 0.0
        out["parity"] = (f"bit-exact: every request equal to its trace checked alone; the oracle on the "
                         f"{len(need)} distinct traces with a pair ({covered:.0%} of the requests)") if ok and same \
            else "MISMATCH"
    else:
        out["parity"] = "every request equal to its trace checked alone" if same else "MISMATCH"
    return out


# ---------------------------------------------------------------- profiles

def _short(name):
    return name.split("(")[0].replace("void ", "").replace("rd::", "").strip()


def summarize_trace(trace_csv: str, label: str, title: str, command: str) -> None:
    """Writes profiles/<label>_kernel_stats.txt from the kernel trace CSV of a rocprofv3
    --kernel-trace --stats run: per (kernel, grid) launches, average and total duration."""
    import csv
    from collections import defaultdict
    dur = defaultdict(list)
    for r in csv.DictReader(open(trace_csv)):
        g = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        dur[(_short(r["Kernel_Name"]), g)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in dur.values())
    lines = [f"# per-kernel durations from rocprofv3 --kernel-trace --stats, {title}, MI355X",
             f"# command: {command}",
             "# keyed by (kernel, grid); 'worked' = launches above 10% of the kernel's longest (a sort pass",
             "# past the key width exits at once)", "",
             f"{'kernel':34s} {'grid':>9s} {'calls':>6s} {'worked':>6s} {'avg_us':>9s} {'sum_ms':>8s} {'pct':>6s}"]
    for (k, g), v in sorted(dur.items(), key=lambda kv: -sum(kv[1])):
        hi = max(v)
        w = [x for x in v if x > 0.1 * hi]
        lines.append(f"{k[:34]:34s} {g:9d} {len(v):6d} {len(w):6d} {sum(w)/len(w):9.1f} {sum(v)/1e3:8.3f} "
                     f"{100*sum(v)/total:6.2f}")
    lines.append(f"\n# total kernel time {total/1e3:.3f} ms over the profiled run")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    open(os.path.join(ROOT, "profiles", f"{label}_kernel_stats.txt"), "w").write("\n".join(lines) + "\n")


def summarize_counters(label: str, fetch_csv: str, write_csv: str, checks: int, events: int, variant: int,
                       command: str) -> None:
    """HBM bytes from two rocprofv3 --pmc runs of `bench.py --counter-run` (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads for the run's plain
    1 GiB copy: profiles/<label>_hbm_traffic.txt and the workload's entry in profiles/traffic.json
    (bytes per check over the library's kernels, bytes per launch of each kernel)."""
    import csv
    from collections import defaultdict

    def per_kernel(path):
        agg = defaultdict(list)
        for r in csv.DictReader(open(path)):
            agg[_short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
        return agg

    fetch, write = per_kernel(fetch_csv), per_kernel(write_csv)
    copy_f = [v for k, vs in fetch.items() if "copyBuffer" in k for v in vs]
    copy_w = [v for k, vs in write.items() if "copyBuffer" in k for v in vs]
    gib_kib = 1024 * 1024
    sf = gib_kib / max(copy_f) if copy_f else 1.0
    sw = gib_kib / max(copy_w) if copy_w else 1.0
    names = sorted(k for k in set(fetch) | set(write) if k.startswith("k_"))
    per_launch, per_check_total = {}, 0.0
    rows = []
    for k in names:
        f, w = fetch.get(k, []), write.get(k, [])
        rb = sum(f) * sf * 1024 / checks
        wb = sum(w) * sw * 1024 / checks
        per_check_total += rb + wb
        launches = max(len(f), len(w)) / checks
        rows.append((rb + wb, k, launches, rb, wb))
        # a kernel run once per pass (the sort) is reported per pass that did work
        worked = [a + b for a, b in zip(f, w)] if len(f) == len(w) else f
        hi = max(worked) if worked else 0
        ww = [x for x in worked if x > 0.1 * hi] if worked else []
        per_launch[k] = (sum(ww) / len(ww)) * 1024 * (sf + sw) / 2 if ww else 0.0
    # the location sort's passes are one kernel for the bench
    sweeps = [k for k in names if k.startswith("k_sort_sweep<3,")]
    if sweeps:
        per_launch["k_sort_sweep"] = max(per_launch[k] for k in sweeps)
    lines = ["# HBM traffic per check from rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE (KiB per dispatch),",
             "# each scaled by what it reads for a 1 GiB plain copy (__amd_rocclr_copyBuffer) of the same run:",
             f"#   copy FETCH_SIZE = {max(copy_f) if copy_f else 0:.0f} KiB -> read scale {sf:.3f};"
             f" copy WRITE_SIZE = {max(copy_w) if copy_w else 0:.0f} KiB -> write scale {sw:.3f}",
             f"# command: {command}", f"# {checks} checks in the profiled run; figures are per check", "",
             f"{'kernel':34s} {'launches':>8s} {'read_MB':>9s} {'write_MB':>9s}"]
    for tot, k, launches, rb, wb in sorted(rows, reverse=True):
        if tot < 0.5e6:
            continue
        lines.append(f"{k[:34]:34s} {launches:8.1f} {rb / 1e6:9.1f} {wb / 1e6:9.1f}")
    lines.append(f"\n# total {per_check_total / 1e9:.3f} GB per check ({per_check_total / events:.1f} B per event)")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    open(os.path.join(ROOT, "profiles", f"{label}_hbm_traffic.txt"), "w").write("\n".join(lines) + "\n")
    try:
        t = json.load(open(COUNTERS_FILE))
    except (OSError, ValueError):
        t = {}
    if t.get("source_digest") != source_digest():
        t = {"source_digest": source_digest(), "workloads": {}}
    t["workloads"][label] = {"events": events, "sort_variant": variant, "checks": checks, "read_scale": sf,
                             "write_scale": sw, "per_check": per_check_total, "per_launch": per_launch}
    json.dump(t, open(COUNTERS_FILE, "w"), indent=1, sort_keys=True)


def counter_run(args) -> None:
    """For rocprofv3 counter runs: a 1 GiB plain device copy (the counters' scale), then exactly
    --steps checks of the workload's trace with the given sort variant, nothing else on the GPU."""
    import torch
    import paper_2111_12478_amd as rd
    import tracegen
    if args.workload == "stencil":
        _, grid, ev, _ = stencil_inputs(args)
        limits = {"clock_bytes": 16 << 30}
    else:
        grid, ev, _, _ = tracegen.generate(tracegen.large(seed=2, scale=args.scale))
        limits = {"max_pairs": max(1 << 20, len(ev) // 4)}
    rc = rd.RaceChecker(0)
    try:
        src = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        rd.rd_set_tuning(rc.ctx, args.sort_variant or 0)
        tr, ws, keep = rc.prepare(grid, torch.from_numpy(ev.view(np.int32)).cuda(), limits)
        for _ in range(args.steps):
            r = rc.run(tr)
            if r.status != 0:
                raise RuntimeError(f"check failed: {r}")
        torch.cuda.synchronize()
        rd.rd_trace_free(rc.ctx, tr)
        print(json.dumps({"counter_run": args.workload, "events": len(ev), "checks": args.steps,
                          "sort_variant": args.sort_variant or 0, "pairs": int(len(r.pairs))}), flush=True)
    finally:
        rc.close()


# ---------------------------------------------------------------- main

def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=1, help="shrink the workloads (tests only)")
    ap.add_argument("--workload", choices=("all", "stencil", "large", "batched", "served", "analyses"), default="all",
                    help="all (default): every workload, the stencil trace as the headline; or one of them alone")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle (parity and CPU baseline)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default location-sort variant")
    ap.add_argument("--sort-variant", type=int, default=None, help="use this location-sort variant, no autotune")
    ap.add_argument("--profile-all", action="store_true", help="print every kernel's time to stderr")
    ap.add_argument("--batch-traces", type=int, default=512)
    ap.add_argument("--served-seconds", type=float, default=60.0, help="arrival window of the served workload")
    ap.add_argument("--served-rate", type=float, default=200.0, help="requests per second")
    ap.add_argument("--served-distinct", type=int, default=256,
                    help="distinct traces the requests draw from (each generated once)")
    ap.add_argument("--counter-run", action="store_true",
                    help="a 1 GiB copy, then exactly --steps checks of --workload (stencil or large); for rocprofv3")
    ap.add_argument("--summarize-trace", nargs=4, metavar=("TRACE_CSV", "LABEL", "TITLE", "COMMAND"),
                    help="write profiles/LABEL_kernel_stats.txt from a rocprofv3 kernel trace and exit")
    ap.add_argument("--summarize-counters", nargs=7,
                    metavar=("LABEL", "FETCH_CSV", "WRITE_CSV", "CHECKS", "EVENTS", "VARIANT", "COMMAND"),
                    help="write profiles/LABEL_hbm_traffic.txt and profiles/traffic.json from two counter runs")
    return ap.parse_args()


def main():
    args = parse()
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_counters:
        a = args.summarize_counters
        summarize_counters(a[0], a[1], a[2], int(a[3]), int(a[4]), int(a[5]), a[6])
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): this build has no multi-GPU "
              f"path, and the value it reports is one GPU's throughput", file=sys.stderr)
        sys.exit(2)
    if args.counter_run:
        counter_run(args)
        return
    oracle_on = not args.no_cpu_baseline
    head = {"metric": METRIC, "n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u32", "data": "synthetic (seeded generators of the workloads' shapes)"}

    # the stencil trace and its whole-trace oracle first: the oracle runs in a forked process (before
    # this one touches the GPU) while the GPU workloads run
    st_inputs = oracle_wait = cpu_sample = None
    if args.workload in ("all", "stencil"):
        st_inputs = stencil_inputs(args)
        if oracle_on:
            _, grid, ev, _ = st_inputs
            m = min(len(ev), 120_000_000)
            r, secs = oracle_prefix(grid, ev, m)
            cpu_sample = (m, secs, f"the first {m:,} events of the trace (a valid trace), one core")
            say(f"stencil: oracle on the first {m:,} events in {secs:.1f} s")
            oracle_wait = background_oracle(grid, ev)

    import torch  # noqa: F401  (after the fork)
    import paper_2111_12478_amd as rd
    rc = rd.RaceChecker(0)
    try:
        if args.workload == "large":
            out, (grid, ev, want) = run_large(args, rc, oracle_on)
            out["race_kinds"] = race_kinds_figures(rc, grid, ev, want)
            print(json.dumps({**head, **out, "warmup": args.warmup}), flush=True)
            return
        if args.workload == "batched":
            out = run_batched(args, rc, oracle_on)
            print(json.dumps({**head, **out, "warmup": args.warmup}), flush=True)
            return
        if args.workload == "served":
            out = run_served(args, rc, oracle_on)
            print(json.dumps({**head, **out, "steps": 1, "warmup": 0}), flush=True)
            return
        if args.workload == "analyses":
            out = run_analyses(args, rc, oracle_on)
            print(json.dumps({**head, **out, "steps": args.steps, "warmup": 1}), flush=True)
            return
        # headline: the stencil trace (its oracle runs meanwhile; the comparison is made last)
        st, st_pairs = run_stencil(args, rc, st_inputs, cpu_sample)
        configs = {}
        if args.workload == "all":
            lg, (grid, ev, want) = run_large(args, rc, oracle_on)
            lg["race_kinds"] = race_kinds_figures(rc, grid, ev, want)
            configs["large"] = lg
            del grid, ev, want
            configs["batched"] = run_batched(args, rc, oracle_on)
            configs["served"] = run_served(args, rc, oracle_on)
            configs["analyses"] = run_analyses(args, rc, oracle_on)
        if oracle_wait is not None:
            say("stencil: waiting for the oracle over the whole trace")
            st["parity"] = parity_of(st_pairs, oracle_wait())
        line = {**head, **st}
        if configs:
            line["configs"] = configs
        print(json.dumps(line), flush=True)
    finally:
        rc.close()


if __name__ == "__main__":
    main()
