"""Throughput of the scoped happens-before race check on one MI355X.

A step is one whole check of one trace: rd_check (every stage of the pipeline, on the device) and
rd_races (the report: pair sort on the device and the copy of the canonical pairs to the host).
The trace is resident in HBM before the timed region starts.  The default workload is the single
large trace: 1024 blocks x 256 threads, 16,777,216 events, 1M words, Zipf(1.1) reuse (synthetic,
seeded; see tracegen.large).

Prints one JSON line with events checked per second, the roofline of the dominant kernel (its
algorithmic bytes per launch over its average launch time, measured live with HIP events on the
launch stream), and the CPU oracle timed on this host as a baseline.
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


def algorithmic_bytes(name: str, n_events: int, n_acc: int, n_sync: int, packed: bool = False) -> int | None:
    """Bytes a kernel must move per launch by what it computes (not what it happens to move).
    Packed elements (category and phase in the key word) are 12 bytes, else 16."""
    e = 12 if packed else 16
    table = {
        # every record read once
        "k_ingest": 16 * n_events,
        # every record read once, one element written per access
        "k_elements": 16 * n_events + e * n_acc,
        # one pass of the location sort: each element read and written once
        "k_sort_sweep": 2 * e * n_acc,
        # the summaries read each sorted element once, its index aside
        "k_seg_reduce": (e - 4) * n_acc,
        "k_seg_check": (e - 4) * n_acc,
    }
    return table.get(name)


def key_bits(ev: np.ndarray, n_blocks: int) -> int:
    """Bits of the location-key span (global words, then each block's shared words), as the checker
    computes it on the device."""
    kind = ev[:, 2] & 15
    acc = np.isin(kind, (0, 1, 2, 6, 7))
    sh = ((ev[:, 2] >> 6) & 1) == 1
    g = ev[acc & ~sh, 0]
    s = ev[acc & sh, 0]
    gs = int(g.max()) - int(g.min()) + 1 if len(g) else 0
    ss = int(s.max()) - int(s.min()) + 1 if len(s) else 0
    total = gs + n_blocks * ss
    return max(0, int(total - 1).bit_length()) if total > 1 else 0


def packed_elements(ev: np.ndarray, n_blocks: int) -> bool:
    """Whether the checker packs category and phase into the key word: key bits + 2 + bits of the
    largest phase (a thread's barrier count) fit in 32 bits."""
    kind = ev[:, 2] & 15
    bars = ev[kind == 4, 1]
    max_phase = int(np.bincount(bars).max()) if len(bars) else 0
    return key_bits(ev, n_blocks) + 2 + max_phase.bit_length() <= 32


def key_passes(ev: np.ndarray, n_blocks: int, tpb: int, radix_bits: int) -> int:
    """Passes of the location sort: bits of the location-key span (global words, then each block's
    shared words), as the checker computes it on the device."""
    kind = ev[:, 2] & 15
    acc = np.isin(kind, (0, 1, 2, 6, 7))
    sh = ((ev[:, 2] >> 6) & 1) == 1
    g = ev[acc & ~sh, 0]
    s = ev[acc & sh, 0]
    gs = int(g.max()) - int(g.min()) + 1 if len(g) else 0
    ss = int(s.max()) - int(s.min()) + 1 if len(s) else 0
    total = gs + n_blocks * ss
    bits = max(0, int(total - 1).bit_length()) if total > 1 else 0
    return (bits + radix_bits - 1) // radix_bits


def source_digest() -> str:
    """Digest of the sources that define the location sort's sweep (its file and the headers it
    includes): a stored traffic figure is used only for the kernel it measured."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2111_12478_amd", "csrc")
    for f in ("rd_internal.h", "rd_kernels.h", "rd_sort.hip"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def summarize_trace(trace_csv: str, label: str, title: str, command: str) -> None:
    """Writes profiles/<label>_kernel_stats.txt from the kernel trace CSV of a rocprofv3
    --kernel-trace --stats run: per (kernel, grid) launches, average and total duration."""
    import csv
    from collections import defaultdict

    def short(name):
        return name.split("(")[0].replace("void ", "").replace("rd::", "")

    dur = defaultdict(list)
    for r in csv.DictReader(open(trace_csv)):
        g = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        dur[(short(r["Kernel_Name"]), g)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
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


def summarize_profiles(trace_csv: str, fetch_csv: str, write_csv: str, command: str) -> None:
    """Turns rocprofv3 CSV output (the kernel trace of a --kernel-trace --stats run, then FETCH_SIZE
    and WRITE_SIZE counter runs of the same command with a 1 GiB plain copy first) into the
    summaries under profiles/.  Kernels are keyed by (name, grid size); launches that did no work
    (a sort pass past the key width: under 10% of the kernel's longest launch) are left out."""
    import csv
    from collections import defaultdict
    out_dir = os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)

    def short(name):
        return name.split("(")[0].replace("void ", "").replace("rd::", "")

    summarize_trace(trace_csv, "large_trace", "large trace (16,777,216 events)", command)

    def per_kernel(path):
        agg = defaultdict(list)
        for r in csv.DictReader(open(path)):
            agg[(short(r["Kernel_Name"]), int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
        return agg

    fetch, write = per_kernel(fetch_csv), per_kernel(write_csv)
    copy_f = [v for (k, g), vs in fetch.items() if "copyBuffer" in k for v in vs]
    copy_w = [v for (k, g), vs in write.items() if "copyBuffer" in k for v in vs]
    gib_kib = 1024 * 1024
    sf = gib_kib / max(copy_f) if copy_f else 1.0
    sw = gib_kib / max(copy_w) if copy_w else 1.0
    lines = ["# HBM traffic per dispatch from rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE (KiB),",
             "# scaled by a 1 GiB plain copy (__amd_rocclr_copyBuffer) of the same run:",
             f"#   copy FETCH_SIZE = {max(copy_f) if copy_f else 0:.0f} KiB -> read scale {sf:.3f};"
             f" copy WRITE_SIZE = {max(copy_w) if copy_w else 0:.0f} KiB -> write scale {sw:.3f}",
             f"# command: {command}", "# averages over launches that did work (above 10% of the largest)", "",
             f"{'kernel':30s} {'grid':>9s} {'n':>3s} {'read_MB':>9s} {'write_MB':>9s}"]
    result = {}
    for key in sorted(set(fetch) | set(write), key=lambda k: -(sum(fetch.get(k, [0])) + sum(write.get(k, [0])))):
        fv, wv = fetch.get(key, []), write.get(key, [])
        f = [v for v in fv if v > 0.1 * max(fv)] if fv else []
        w = [v for v in wv if v > 0.1 * max(wv)] if wv else []
        rd_mb = (sum(f) / len(f) if f else 0) * sf * 1024 / 1e6
        wr_mb = (sum(w) / len(w) if w else 0) * sw * 1024 / 1e6
        if rd_mb + wr_mb < 0.5:
            continue
        lines.append(f"{key[0][:30]:30s} {key[1]:9d} {max(len(f), len(w)):3d} {rd_mb:9.1f} {wr_mb:9.1f}")
        result[key] = (rd_mb, wr_mb)
    open(os.path.join(out_dir, "large_trace_hbm_traffic.txt"), "w").write("\n".join(lines) + "\n")
    # every element-sort variant (template arguments) ran during the autotune, so each one's
    # traffic is stored and the bench reads the figure of the variant it timed
    sweeps = {k: {"bytes_per_launch": (r + w) * 1e6, "read_bytes": r * 1e6, "write_bytes": w * 1e6}
              for (k, g), (r, w) in result.items() if k.startswith("k_sort_sweep<3,")}
    if sweeps:
        json.dump({"kernel": "k_sort_sweep", "workload_events": 16777216, "source_digest": source_digest(),
                   "read_scale": sf, "write_scale": sw, "variants": sweeps},
                  open(os.path.join(out_dir, "traffic.json"), "w"), indent=1)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=1, help="shrink the workload (tests only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default location-sort variant")
    ap.add_argument("--profile-all", action="store_true", help="print every kernel's time to stderr")
    ap.add_argument("--summarize-profiles", nargs=4, metavar=("TRACE_CSV", "FETCH_CSV", "WRITE_CSV", "COMMAND"),
                    help="write profiles/ summaries from rocprofv3 CSV files and exit")
    ap.add_argument("--summarize-trace", nargs=4, metavar=("TRACE_CSV", "LABEL", "TITLE", "COMMAND"),
                    help="write profiles/LABEL_kernel_stats.txt from a rocprofv3 kernel trace and exit")
    ap.add_argument("--workload", choices=("large", "batched", "served", "stencil"), default="large",
                    help="large: one 16M-event trace (default); batched: 512 traces, one pass vs one per trace; "
                         "served: Poisson arrivals through the request loop")
    ap.add_argument("--batch-traces", type=int, default=512)
    ap.add_argument("--served-seconds", type=float, default=60.0, help="arrival window of the served workload")
    ap.add_argument("--served-rate", type=float, default=200.0, help="requests per second")
    ap.add_argument("--served-distinct", type=int, default=96,
                    help="distinct traces the requests draw from (each generated once)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="run one plain device copy of this many bytes first (calibrates HBM counters)")
    return ap.parse_args()


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


def bench_batched(args):
    """512 independent traces (lengths lognormal around 200K events) checked two ways on the same
    resident events: one rd_check + rd_races per trace, in turn (plain), and one rd_check_many +
    rd_races_many over all of them (batched).  The JSON line reports the batched rate."""
    import concurrent.futures as cf
    import torch
    import tracegen
    import paper_2111_12478_amd as rd

    cfgs = tracegen.batch(seed=4, n_traces=args.batch_traces, scale=args.scale)
    workers = min(16, os.cpu_count() or 1)
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        items = list(ex.map(_gen_member, cfgs, chunksize=4))
    n_total = sum(int(ev.shape[0]) for _, ev in items)
    print(f"batched: {len(items)} traces, {n_total:,} events generated", file=sys.stderr, flush=True)
    rc = rd.RaceChecker(0)
    limits = {"clock_bytes": 16 << 20}
    bound = [rc.prepare(g, torch.from_numpy(ev.view(np.int32)).cuda(), limits) for g, ev in items]
    traces = [b[0] for b in bound]
    bws_bytes = rd.rd_batch_workspace_bytes(rc.ctx, traces, None)
    bws = torch.empty(bws_bytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    print(f"batched: bound, member workspaces {sum(b[1].numel() for b in bound) / 2**30:.1f} GiB, "
          f"batch workspace {bws_bytes / 2**30:.1f} GiB", file=sys.stderr, flush=True)

    def plain_step():
        return [rc.run(t) for t in traces]

    def batched_step():
        st = rd.rd_check_many(rc.ctx, traces, bws.data_ptr(), bws.numel(), None, stream)
        if st != rd.RD_OK:
            raise RuntimeError(f"rd_check_many failed: {st}")
        return rc.report_many(traces)

    def timed(fn, steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, res

    steps = max(1, min(args.steps, 5))
    tune_ms = None
    if not args.no_tune:
        st, best, tune_ms = rd.rd_autotune(rc.ctx, traces, bws.data_ptr(), bws.numel(), stream)
        if st != rd.RD_OK:
            raise RuntimeError(f"rd_autotune failed: {st}")
        print(f"batched: autotuned variant {best} {rd.rd_tuning_get(best)}: {['%.2f' % m for m in tune_ms]} ms",
              file=sys.stderr, flush=True)
    variant = rd.rd_get_tuning(rc.ctx)
    for _ in range(max(1, min(args.warmup, 2))):
        plain_res = plain_step()
        batch_res = batched_step()
    t_plain, plain_res = timed(plain_step, steps)
    print(f"batched: plain {t_plain * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
    t_batch, batch_res = timed(batched_step, steps)
    print(f"batched: batched {t_batch * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
    same = all(a.status == b.status == 0 and np.array_equal(a.pairs, b.pairs) for a, b in zip(plain_res, batch_res))
    n_pairs = sum(len(r.pairs) for r in batch_res)
    out = {
        "metric": "memory events checked/sec (bit-exact race set) and % of HBM peak; batched vs plain",
        "value": n_total / t_batch,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": max(1, min(args.warmup, 2)),
        "ms_per_step": t_batch * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded generator, same shape as the workload)",
        "config": {
            "workload": f"batched form: {len(items)} traces, lengths lognormal(median 204,800, sigma 1) in "
                        f"[10,240, 4,194,304], 2^U{{6..11}} blocks x 128|256 threads, mix of the 16M-event "
                        f"trace, seed 4; one rd_check_many + rd_races_many",
            "events": n_total,
            "race_pairs": int(n_pairs),
            "sort_variant": {"index": variant, "digit_bits": rd.rd_tuning_get(variant)[0],
                             "waves": rd.rd_tuning_get(variant)[1], "items": rd.rd_tuning_get(variant)[2],
                             "autotune_ms": tune_ms},
        },
        "plain": {"value": n_total / t_plain, "unit": "events/s", "ms_per_step": t_plain * 1e3,
                  "form": "one rd_check + rd_races per trace, in turn, same resident events"},
        "batched_vs_plain": t_plain / t_batch,
        "batched_equals_plain": bool(same),
    }
    if not args.no_cpu_baseline:
        # oracle on a bounded sample of the members, in a process pool over the host's cores
        rng = np.random.default_rng(4)
        order = rng.permutation(len(items))
        sample, budget = [], 0
        for j in order:
            if budget + int(items[j][1].shape[0]) > 40_000_000:
                continue
            sample.append(int(j))
            budget += int(items[j][1].shape[0])
        c0 = time.perf_counter()
        with cf.ProcessPoolExecutor(max_workers=workers) as ex:
            res = list(ex.map(_oracle_member, [items[j] for j in sample], chunksize=1))
        c1 = time.perf_counter()
        ok = all(st == 0 and np.array_equal(p, batch_res[j].pairs) for j, (st, p, _) in zip(sample, res))
        out["cpu_baseline"] = {
            "value": budget / (c1 - c0),
            "unit": "events/s",
            "cores": workers,
            "kind": "oracle",
            "sample": f"{len(sample)} of the {len(items)} traces ({budget:,} events), one trace per process",
        }
        out["parity"] = "bit-exact" if ok and same else "MISMATCH"
    for t in traces:
        rd.rd_trace_free(rc.ctx, t)
    print(json.dumps(out), flush=True)


def _served_cfg(i, n):
    import tracegen
    return tracegen.MixConfig(n_blocks=max(1, -(-n // 16384)), tpb=256, n_events=n, n_global=max(16, (n // 16) * 4 // 5),
                              n_shared=max(1, (n // 16 - (n // 16) * 4 // 5) // max(1, -(-n // 16384))),
                              zipf_s=1.1, p_write=0.30, p_atomic_block=0.01, p_atomic_device=0.01, bar_period=64,
                              fence_period=512, plant_rate=1e-4, p_plant_same_block=0.5, plant_victim_cap=256,
                              frac_ro=0.3, frac_da=0.05, frac_priv=0.7, frac_pro=0.25, p_read_ro=0.3, seed=5,
                              trace_index=i)


def bench_served(args):
    """Poisson arrivals (rate, window) of check requests with sizes log-uniform on [102,400,
    8,388,608] events (256 threads per block, one block per 16,384 events, the mix of the 16M-event
    trace, seed 5), answered by the request loop under a 64 GiB arena.  The same arrival list is
    replayed with one request per pass and one pass in flight (plain) for comparison.  Requests
    draw their traces from a pool of distinct generated traces."""
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
    workers = min(16, os.cpu_count() or 1)
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        pool = list(ex.map(_gen_member, cfgs, chunksize=1))
    print(f"served: {n_req} requests over {args.served_seconds:.0f} s from {len(pool)} distinct traces",
          file=sys.stderr, flush=True)
    rc = rd.RaceChecker(0)
    alone = [rc.check(g, ev) for g, ev in pool]  # each distinct trace checked alone (plain)
    budget = 64 << 30

    def run(max_batch, max_inflight):
        srv = rd.Server(rc, budget, max_batch=max_batch, max_inflight=max_inflight)
        tickets = [None] * n_req
        results = [None] * n_req
        t_base = [0.0]

        def submitter():
            t0 = time.perf_counter()
            for i in range(n_req):
                d = arrivals[i] - (time.perf_counter() - t0)
                if d > 0:
                    time.sleep(d)
                tickets[i] = srv.submit(*pool[pick[i]])
                ready[i].set()

        ready = [threading.Event() for _ in range(n_req)]

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

    served = run(256, 2)
    print(f"served: {served}", file=sys.stderr, flush=True)
    plain = run(1, 1)
    print(f"served (plain, one request per pass): {plain}", file=sys.stderr, flush=True)
    n_events = int(sum(int(pool[j][1].shape[0]) for j in pick))
    out = {
        "metric": "memory events checked/sec (bit-exact race set) and % of HBM peak; batched vs plain",
        "value": served["events_per_s"],
        "unit": "events/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": served["makespan_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded generator, same shape as the workload)",
        "config": {
            "workload": f"served form: Poisson {args.served_rate:.0f} req/s for {args.served_seconds:.0f} s "
                        f"({n_req} requests, {n_events:,} events), sizes log-uniform [102,400, 8,388,608], "
                        f"{args.served_distinct} distinct traces, 64 GiB arena, seed 5",
            "requests": n_req,
            "events": n_events,
        },
        "served": served,
        "plain": plain,
    }
    print(json.dumps(out), flush=True)


def _plants_hit(grid, ev, pairs, plants, cfg):
    """Every planted downgrade shows up: a fence pair as a race between the neighbour block (first)
    and the acquiring block (second), a lock pair as a race of the section's block on the
    accumulator or the lock word."""
    tpb = grid[1]
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


def bench_stencil(args):
    """The halo-exchange stencil with a lock-guarded reduction (4096 blocks x 256 threads,
    268,508,160 events), resident in HBM; a step is rd_check + rd_races."""
    import torch
    import tracegen
    import paper_2111_12478_amd as rd

    cfg = tracegen.stencil()
    if args.scale > 1:
        cfg = tracegen.StencilConfig(rb=max(1, cfg.rb // args.scale), cb=cfg.cb, tpb=cfg.tpb, rows=cfg.rows,
                                     sweeps=cfg.sweeps, pitch=cfg.pitch, group=cfg.group,
                                     plant_rate=cfg.plant_rate * args.scale, seed=cfg.seed)
    t0 = time.perf_counter()
    grid, ev, gst, plants = tracegen.generate_stencil(cfg)
    n = int(ev.shape[0])
    print(f"stencil: {n:,} events generated in {time.perf_counter() - t0:.1f} s, {len(plants)} plants",
          file=sys.stderr, flush=True)
    rc = rd.RaceChecker(0)
    dev_ev = torch.from_numpy(ev.view(np.int32)).cuda()
    limits = {"clock_bytes": int(os.environ.get("RD_CLOCK_BYTES", str(16 << 30)))}
    tr, ws, keep = rc.prepare(grid, dev_ev, limits)
    print(f"stencil: workspace {ws.numel() / 2**30:.1f} GiB", file=sys.stderr, flush=True)
    res = rc.run(tr)
    if res.status != 0:
        raise RuntimeError(f"check failed: {res} {res.message} {rd.rd_last_error(rc.ctx)}")
    # the location-sort variant for this trace (untimed), as for the large trace
    if not args.no_tune:
        st, best, tune_ms = rd.rd_autotune(rc.ctx, [tr], None, 0, torch.cuda.current_stream().cuda_stream)
        if st != rd.RD_OK:
            raise RuntimeError(f"rd_autotune failed: {st}")
        print(f"stencil: autotuned variant {best} {rd.rd_tuning_get(best)}: {['%.1f' % m for m in tune_ms]} ms",
              file=sys.stderr, flush=True)
    variant = rd.rd_get_tuning(rc.ctx)
    lib = rd.load_library()
    steps = max(1, min(args.steps, 5))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        res = rc.run(tr)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    per = (t2 - t1) / steps
    if args.profile_all:
        lib.rd_profile_enable.argtypes = [ctypes.c_void_p, ctypes.c_char_p]

        class KT(ctypes.Structure):
            _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_uint32), ("total_ms", ctypes.c_double)]

        lib.rd_profile_read.argtypes = [ctypes.c_void_p, ctypes.POINTER(KT), ctypes.c_uint32,
                                        ctypes.POINTER(ctypes.c_uint32)]
        lib.rd_profile_enable(rc.ctx, b"*")
        rc.run(tr)
        buf = (KT * 96)()
        cnt = ctypes.c_uint32()
        lib.rd_profile_read(rc.ctx, buf, 96, ctypes.byref(cnt))
        lib.rd_profile_enable(rc.ctx, None)
        rows = sorted(((buf[i].total_ms, buf[i].launches, buf[i].name.decode()) for i in range(cnt.value)), reverse=True)
        for ms, c, name in rows:
            print(f"  {name:28s} launches={c:3d} total={ms:8.3f} ms", file=sys.stderr)
    pairs = res.pairs
    missing = _plants_hit(grid, ev, pairs, plants, cfg)
    print(f"stencil: {per * 1e3:.1f} ms/step, {len(pairs)} pairs, plants missing {missing}", file=sys.stderr,
          flush=True)
    out = {
        "metric": "memory events checked/sec (bit-exact race set) and % of HBM peak; batched vs plain",
        "value": n / per,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 1,
        "ms_per_step": per * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded generator, same shape as the workload)",
        "config": {
            "workload": f"stencil and reduction: {grid[0]} blocks x {grid[1]} threads, {n:,} events, "
                        f"{cfg.sweeps} sweeps of a 5-point stencil over two {cfg.rb * cfg.rows} x "
                        f"{cfg.cb * cfg.tpb} buffers (row pitch {cfg.pitch}), halo flags, device lock, "
                        f"{len(plants)} planted scope downgrades, seed {cfg.seed}",
            "events": n,
            "race_pairs": int(len(pairs)),
            "plants_missing": int(missing),
            "sort_variant": {"index": variant, "digit_bits": rd.rd_tuning_get(variant)[0],
                             "waves": rd.rd_tuning_get(variant)[1], "items": rd.rd_tuning_get(variant)[2]},
        },
    }
    if not args.no_cpu_baseline:
        # the oracle on a prefix of the trace (a prefix of a valid trace is valid), against the GPU
        import oracle
        m = min(n, 72_000_000)  # two sweeps: the first plants and the reads that race with them
        sub = np.ascontiguousarray(ev[:m])
        g_sub = rc.check(grid, sub, limits)
        c0 = time.perf_counter()
        want = oracle.check(grid, sub)
        c1 = time.perf_counter()
        out["cpu_baseline"] = {"value": m / (c1 - c0), "unit": "events/s", "cores": 1, "kind": "oracle",
                               "sample": f"the first {m:,} events of the trace (a valid trace), one core"}
        out["parity"] = "bit-exact on the prefix" if (want.status == g_sub.status == 0 and
                                                       np.array_equal(want.pairs, g_sub.pairs)) else "MISMATCH"
    rd.rd_trace_free(rc.ctx, tr)
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.summarize_profiles:
        summarize_profiles(*args.summarize_profiles)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the checker has no "
              f"multi-GPU path in this build", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "served":
        bench_served(args)
        return
    if args.workload == "stencil":
        bench_stencil(args)
        return
    import torch
    import tracegen
    import paper_2111_12478_amd as rd

    cfg = tracegen.large(seed=2, scale=args.scale)
    grid, ev, gstats, _ = tracegen.generate(cfg)
    n = int(ev.shape[0])
    kinds = np.bincount(ev[:, 2] & 15, minlength=8)
    n_acc = int(kinds[0] + kinds[1] + kinds[2] + kinds[6] + kinds[7])
    n_sync = int(n - kinds[0] - kinds[1])

    rc = rd.RaceChecker(0)
    dev_ev = torch.from_numpy(ev.view(np.int32)).cuda()
    limits = {"max_pairs": max(1 << 20, n // 4)}
    tr, ws, keep = rc.prepare(grid, dev_ev, limits)
    lib = rd.load_library()

    class KT(ctypes.Structure):
        _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_uint32), ("total_ms", ctypes.c_double)]

    lib.rd_profile_enable.argtypes = [ctypes.c_void_p, ctypes.c_char_p]
    lib.rd_profile_read.argtypes = [ctypes.c_void_p, ctypes.POINTER(KT), ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]

    def read_profile():
        buf = (KT * 64)()
        cnt = ctypes.c_uint32()
        lib.rd_profile_read(rc.ctx, buf, 64, ctypes.byref(cnt))
        return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms) for i in range(cnt.value)}

    def step():
        res = rc.run(tr)
        if res.status != 0:
            raise RuntimeError(f"check failed: {res}")
        return res

    # pick the location-sort variant for this trace (untimed), as a user of the library would
    tune_ms = None
    if not args.no_tune:
        st, best, tune_ms = rd.rd_autotune(rc.ctx, [tr], None, 0, torch.cuda.current_stream().cuda_stream)
        if st != rd.RD_OK:
            raise RuntimeError(f"rd_autotune failed: {st}")
    variant = rd.rd_get_tuning(rc.ctx)
    if args.copy_bytes:
        src_t = torch.empty(args.copy_bytes // 4, dtype=torch.int32, device="cuda")
        dst_t = torch.empty_like(src_t)
        src_t.fill_(1)
        torch.cuda.synchronize()
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        del src_t, dst_t
    for _ in range(args.warmup):
        res = step()
    # one profiled step to find the dominant kernel
    lib.rd_profile_enable(rc.ctx, b"*")
    res = step()
    prof = read_profile()
    lib.rd_profile_enable(rc.ctx, None)
    if args.profile_all:
        for k, (c, ms) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
            print(f"  {k:28s} launches={c:3d} total={ms:8.3f} ms", file=sys.stderr)
    # the element sort runs one sweep per key digit; its passes count as one kernel
    radix_bits = rd.rd_tuning_get(variant)[0]
    passes = key_passes(ev, grid[0], grid[1], radix_bits)
    pass_names = [f"k_sort_sweep_p{p}" for p in range(passes)]

    def merged(prof):
        out = {}
        for k, (c, ms) in prof.items():
            if k.startswith("k_sort_sweep_p"):
                if k not in pass_names:
                    continue  # a pass the key width makes empty
                k = "k_sort_sweep"
            c0, m0 = out.get(k, (0, 0.0))
            out[k] = (c0 + c, m0 + ms)
        return out

    packed = packed_elements(ev, grid[0])
    candidates = [(ms, k) for k, (c, ms) in merged(prof).items()
                  if algorithmic_bytes(k, n, n_acc, n_sync, packed) is not None]
    dom = max(candidates)[1]

    # timed region: K steps, the dominant kernel bracketed by HIP events on its stream (recorded
    # inside the check's graph, which one untimed step captures with those records)
    filt = b"k_sort_sweep_p*" if dom == "k_sort_sweep" else dom.encode()
    lib.rd_profile_enable(rc.ctx, filt)
    res = step()
    lib.rd_profile_enable(rc.ctx, filt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kp = merged(read_profile())
    lib.rd_profile_enable(rc.ctx, None)
    launches, total_ms = kp.get(dom, (0, 0.0))
    if dom == "k_sort_sweep":
        # the sweeps run back to back and one pair of events brackets them all, the passes past
        # the key width (which exit at once) included: their time counts, only the real passes
        # count as launches (a conservative average)
        launches = passes * args.steps
    avg_s = (total_ms / max(1, launches)) / 1e3
    alg = algorithmic_bytes(dom, n, n_acc, n_sync, packed)
    achieved = alg / avg_s / 1e9 if avg_s > 0 else 0.0
    elapsed = t1 - t0
    ms_per_step = elapsed * 1e3 / args.steps
    value = n * args.steps / elapsed

    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        try:
            t = json.load(open(tfile))
            rb, waves, items = rd.rd_tuning_get(variant)
            rec = t.get("variants", {}).get(f"k_sort_sweep<3, {rb}, {waves}, {items}, false>")
            if (rec and t.get("kernel") == dom and t.get("workload_events") == n
                    and t.get("source_digest") == source_digest()):
                traffic = rec["bytes_per_launch"]
        except Exception:
            traffic = None

    gpu_pairs = res.pairs
    out = {
        "metric": "memory events checked/sec (bit-exact race set) and % of HBM peak; batched vs plain",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded generator, same shape as the workload)",
        "config": {
            "workload": f"single large trace, plain method: {grid[0]} blocks x {grid[1]} threads, {n:,} events, "
                        f"{cfg.n_global + cfg.n_blocks * cfg.n_shared:,} words (Zipf {cfg.zipf_s}), seed {cfg.seed}",
            "events": n,
            "accesses": n_acc,
            "race_pairs": int(len(gpu_pairs)),
            "radix_bits": radix_bits,
            "sort_passes": passes,
            "packed_elements": bool(packed),
            "sort_variant": {"index": variant, "digit_bits": rd.rd_tuning_get(variant)[0],
                             "waves": rd.rd_tuning_get(variant)[1], "items": rd.rd_tuning_get(variant)[2],
                             "autotune_ms": tune_ms},
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": alg,
            "avg_launch_ms": avg_s * 1e3,
            "launches": launches,
        },
    }

    if not args.no_cpu_baseline:
        import oracle
        c0 = time.perf_counter()
        want = oracle.check(grid, ev)
        c1 = time.perf_counter()
        out["cpu_baseline"] = {
            "value": n / (c1 - c0),
            "unit": "events/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"the whole {n:,}-event trace, single-threaded per-event vector-clock detector",
        }
        out["parity"] = "bit-exact" if np.array_equal(want.pairs, gpu_pairs) else \
            f"MISMATCH gpu={len(gpu_pairs)} oracle={len(want.pairs)}"

    # unique race kinds of the report (site-id pairs), built on the device after the timed steps:
    # wall time per call (it waits for the check's state, builds the kinds, copies them back)
    st, kinds = rc.kinds(tr)
    reps = 5
    torch.cuda.synchronize()
    k0 = time.perf_counter()
    for _ in range(reps):
        st, kinds = rc.kinds(tr)
    k1 = time.perf_counter()
    out["race_kinds"] = {"kinds": int(kinds.shape[0]), "pairs": int(len(gpu_pairs)), "status": int(st),
                         "ms_per_call": (k1 - k0) * 1e3 / reps}
    if not args.no_cpu_baseline:
        wk = oracle.race_kinds(ev, want.pairs)
        out["race_kinds"]["parity"] = "bit-exact" if np.array_equal(wk, kinds) else \
            f"MISMATCH gpu={len(kinds)} oracle={len(wk)}"

    rd.rd_trace_free(rc.ctx, tr)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
