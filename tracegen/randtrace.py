"""Seeded random *valid* tiny traces with every event kind (input generator; no race logic).

A trace is built by writing a small program per thread (reads, writes, scoped atomics, scoped
fences, explicit lock acquires/releases, block barriers and warp barriers) and interleaving the
threads with a seeded random scheduler that respects the waiting rules of barriers: a thread that
arrives at a block barrier waits until every active thread of its block has arrived there, and a
lane that arrives at a warp barrier waits until every lane of the barrier's mask has arrived.

The programs keep barriers consistent so the scheduler never deadlocks: every thread of a block
takes the same number of block barriers, and a warp barrier step is taken by exactly the lanes
of its mask.  Nothing here knows which pairs race.
"""
from __future__ import annotations

import numpy as np

from .format import make_meta, KIND, SCOPE

_KINDS_ACCESS = ("R", "W", "A")


def random_trace(seed: int, max_blocks: int = 3, max_tpb: int = 6, max_events: int = 400, wbar: bool = True):
    """Returns (grid, events) with grid = (n_blocks, tpb, warp_size) and events (N, 4) uint32.
    wbar=False: no warp barriers."""
    rng = np.random.default_rng(seed)
    nb = int(rng.integers(1, max_blocks + 1))
    tpb = int(rng.integers(1, max_tpb + 1))
    ws = int(rng.integers(1, min(tpb, 4) + 1))
    n_threads = nb * tpb
    n_glob = int(rng.integers(1, 6))
    n_shared = int(rng.integers(0, 3))
    n_locks = int(rng.integers(1, 3))
    n_phases = int(rng.integers(1, 4))  # block barriers = n_phases - 1
    p_kind = rng.dirichlet(np.ones(8))  # read, write, atomic, fence, acq, rel, fenced-atomic, wbar-step
    budget = max(1, max_events // max(1, n_threads))

    def addr_pick():
        if n_shared and rng.random() < 0.3:
            return int(rng.integers(0, n_shared)), 1
        return 100 + int(rng.integers(0, n_glob)), 0

    def scope_pick():
        return int(rng.choice([0, 0, 1, 1, 2]))

    # programs[t] = list of ops: (kind_name, scope, space, addr, aux) ; "BAR" and "WBAR" included
    programs = [[] for _ in range(n_threads)]
    warp_ids = {}
    inactive = set()
    if n_threads > 1 and rng.random() < 0.15 and n_phases == 1:
        inactive.add(int(rng.integers(0, n_threads)))  # a thread with no events at all
    for b in range(nb):
        for ph in range(n_phases):
            # steps of this phase; a step is either per-thread ops or a warp-barrier step
            n_steps = int(rng.integers(1, 4))
            for _step in range(n_steps):
                if wbar and rng.random() < p_kind[7] * 2 and ws > 1:
                    # warp barrier step: one warp, a mask of its existing lanes.  Every warp
                    # barrier with a given (warp, id) uses one mask, so the lanes' occurrence
                    # counts of that id stay aligned.
                    n_warps = (tpb + ws - 1) // ws
                    w = int(rng.integers(0, n_warps))
                    ids = warp_ids.setdefault((b, w), {})
                    if ids and rng.random() < 0.3:
                        wid = int(rng.choice(sorted(ids)))
                        mask = ids[wid]
                    else:
                        lanes = [l for l in range(ws) if w * ws + l < tpb]
                        lanes = [l for l in lanes if (b * tpb + w * ws + l) not in inactive]
                        if not lanes:
                            continue
                        k = int(rng.integers(1, len(lanes) + 1))
                        chosen = sorted(rng.choice(lanes, size=k, replace=False).tolist())
                        mask = 0
                        for l in chosen:
                            mask |= 1 << l
                        wid = len(ids) + 7 * b
                        ids[wid] = mask
                    for l in range(ws):
                        if (mask >> l) & 1:
                            programs[b * tpb + w * ws + l].append(("WBAR", 0, 0, wid, mask))
                    continue
                for tl in range(tpb):
                    t = b * tpb + tl
                    if t in inactive:
                        continue
                    n_ops = int(rng.integers(0, max(1, budget // (n_phases * n_steps)) + 1))
                    for _ in range(n_ops):
                        c = int(rng.choice(7, p=p_kind[:7] / p_kind[:7].sum()))
                        if c == 0 or c == 1:
                            a, sp = addr_pick()
                            programs[t].append(("R" if c == 0 else "W", 0, sp, a, 0))
                        elif c == 2:
                            a, sp = addr_pick()
                            programs[t].append(("A", scope_pick(), sp, a, 0))
                        elif c == 3:
                            programs[t].append(("F", scope_pick(), 0, 0, 0))
                        elif c == 4 or c == 5:
                            lk = 50 + int(rng.integers(0, n_locks))
                            sp = 1 if (n_shared and rng.random() < 0.2) else 0
                            programs[t].append(("ACQ" if c == 4 else "REL", scope_pick(), sp, lk, 0))
                        else:
                            # fence-atomic-fence shapes: release and/or acquire by inference
                            lk = 50 + int(rng.integers(0, n_locks))
                            sp = 1 if (n_shared and rng.random() < 0.2) else 0
                            if rng.random() < 0.6:
                                programs[t].append(("F", scope_pick(), 0, 0, 0))
                            programs[t].append(("A", scope_pick(), sp, lk, 0))
                            if rng.random() < 0.6:
                                programs[t].append(("F", scope_pick(), 0, 0, 0))
            if ph + 1 < n_phases:
                for tl in range(tpb):
                    t = b * tpb + tl
                    if t not in inactive:
                        programs[t].append(("BAR", 0, 0, 0, 0))
    # make every non-inactive thread active (>= 1 event), so barrier participants are predictable
    for t in range(n_threads):
        if t not in inactive and not programs[t]:
            a, sp = addr_pick()
            programs[t].append(("R", 0, sp, a, 0))

    # scheduler
    pc = [0] * n_threads
    active = [t for t in range(n_threads) if programs[t]]
    n_active_blk = [0] * nb
    for t in active:
        n_active_blk[t // tpb] += 1
    bar_count = [0] * n_threads            # BARs emitted so far
    bar_arrived = {}                        # (block, k) -> arrivals
    wbar_seen = {}                          # (thread, id) -> occurrences emitted
    wbar_arrived = {}                       # (warp0, id, occ) -> set of lanes arrived
    waiting = {}                            # thread -> predicate key
    events = []

    def blocked(t):
        w = waiting.get(t)
        if w is None:
            return False
        if w[0] == "BAR":
            return bar_arrived.get(w[1], 0) < n_active_blk[w[1][0]]
        inst, mask = w[1], w[2]
        got = wbar_arrived.get(inst, 0)
        return got != mask

    while True:
        runnable = [t for t in active if pc[t] < len(programs[t]) and not blocked(t)]
        if not runnable:
            break
        t = int(rng.choice(runnable))
        waiting.pop(t, None)
        op = programs[t][pc[t]]
        pc[t] += 1
        name, sc, sp, a, aux = op
        events.append((a, t, make_meta(KIND[name], sc, sp), aux))
        if name == "BAR":
            key = (t // tpb, bar_count[t])
            bar_count[t] += 1
            bar_arrived[key] = bar_arrived.get(key, 0) + 1
            waiting[t] = ("BAR", key)
        elif name == "WBAR":
            occ = wbar_seen.get((t, a), 0)
            wbar_seen[(t, a)] = occ + 1
            lane = (t % tpb) % ws
            warp0 = t - lane
            inst = (warp0, a, occ)
            wbar_arrived[inst] = wbar_arrived.get(inst, 0) | (1 << lane)
            waiting[t] = ("WBAR", inst, aux)
    assert all(pc[t] == len(programs[t]) for t in range(n_threads)), "scheduler deadlock"
    ev = np.array(events, dtype=np.uint32).reshape(-1, 4)
    return (nb, tpb, ws), ev
