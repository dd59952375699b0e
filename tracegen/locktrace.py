"""Seeded random valid traces built around critical sections (input generator; no race logic).

Each thread runs a small program of reads, writes and atomics on a few data words, and critical
sections on a few lock words: an acquire, a body of accesses (possibly a nested section on a lock of
a higher id, so lock waits cannot cycle) and the matching release with the acquire's scope.  Locks
are explicit ACQ/REL events or, with ``inferred``, the fence idiom of Section 2.1 (an atomic
followed by a fence acquires, a fence followed by an atomic releases).  A seeded scheduler
interleaves the threads and respects mutual exclusion: a thread waits to acquire a lock while
another thread holds it with an overlapping scope (either device scoped, or both in one block).
Optional block barriers (every thread of a block takes the same number; no lock is held across one)
and flag publications (a release of a flag word with no acquire, and acquires of it that are never
released) add happens-before edges that are not critical sections.
"""
from __future__ import annotations

import numpy as np

from .format import KIND, make_meta

R, W, A, F, BAR, ACQ, REL = (KIND[k] for k in ("R", "W", "A", "F", "BAR", "ACQ", "REL"))
BLK, DEV = 0, 1


def lock_trace(seed: int, max_blocks: int = 3, max_tpb: int = 4, max_events: int = 300, barriers: bool = False,
               flags: bool = False, inferred: bool = True, grid=None, locks: int | None = None,
               data_words: int | None = None):
    """Returns (grid, events (N, 4) uint32).  grid, locks (<= 64) and data_words fix what is
    otherwise drawn: the grid, the number of lock words and of global data words (more than 100
    data words start at word 4096)."""
    rng = np.random.default_rng(seed)
    nb = int(rng.integers(1, max_blocks + 1))
    tpb = int(rng.integers(1, max_tpb + 1))
    if grid is not None:
        nb, tpb = int(grid[0]), int(grid[1])
    T = nb * tpb
    n_locks = int(rng.integers(1, 4))
    n_data = int(rng.integers(1, 5))
    if locks is not None:
        n_locks = min(int(locks), 64)
    if data_words is not None:
        n_data = int(data_words)
    data_base = 100 if n_data <= 100 else 4096
    n_shared = int(rng.integers(0, 2))
    n_phases = int(rng.integers(1, 3)) if barriers else 1
    budget = max(4, max_events // max(1, T))

    def data_op(atomics=True):
        if n_shared and rng.random() < 0.25:
            space, addr = 1, int(rng.integers(0, n_shared))
        else:
            space, addr = 0, data_base + int(rng.integers(0, n_data))
        r = rng.random()
        kind = R if r < 0.45 else (W if r < 0.9 or not atomics else A)
        scope = int(rng.choice([0, 1])) if kind == A else 0
        return [("op", addr, make_meta(kind, scope, space))]

    def section(lo_lock, depth):
        lk = int(rng.integers(lo_lock, n_locks))
        scope = BLK if rng.random() < 0.35 else DEV
        word = 200 + lk
        ops = []
        fenced = inferred and rng.random() < 0.4
        if fenced:
            # an atomic on the lock word then a fence acquires; a fence then an atomic releases
            acq = [("acq", word, make_meta(A, scope), lk, scope, "acq"), ("op", 0, make_meta(F, scope))]
            rel = [("op", 0, make_meta(F, scope)), ("rel", word, make_meta(A, scope), lk, scope, "rel")]
        else:
            acq = [("acq", word, make_meta(ACQ, scope), lk, scope)]
            rel = [("rel", word, make_meta(REL, scope), lk, scope)]
        ops += acq
        for _ in range(int(rng.integers(0, 4))):
            if depth == 0 and lk + 1 < n_locks and rng.random() < 0.2:
                ops += section(lk + 1, depth + 1)
            else:
                # no data atomic next to the section's fences (it would be read as a lock operation)
                ops += data_op(atomics=not fenced)
        ops += rel
        return ops

    def flag_op():
        word = 300 + int(rng.integers(0, 2))
        if rng.random() < 0.5:  # publish: fence, atomic (a release with no critical section)
            return [("op", 0, make_meta(F, 1)), ("op", word, make_meta(A, 1), None, None, "rel")]
        return [("op", word, make_meta(A, 1), None, None, "acq"), ("op", 0, make_meta(F, 1))]  # take: atomic, fence

    def separate(prog):
        """A read between an atomic and a fence next to it that is not its own (a nested section's
        boundary next to the outer one's, a data atomic next to a section), so that every
        atomic-fence adjacency is an intended acquire or release."""
        out = []
        for j, op in enumerate(prog):
            is_a = op[0] != "bar" and (op[2] & 15) == A
            role = op[5] if len(op) > 5 else None
            prev_f = bool(out) and out[-1][0] != "bar" and (out[-1][2] & 15) == F
            if is_a and prev_f and role != "rel":
                out.append(("op", 100, make_meta(R)))
            out.append(op)
            nxt = prog[j + 1] if j + 1 < len(prog) else None
            next_f = nxt is not None and nxt[0] != "bar" and (nxt[2] & 15) == F
            if is_a and next_f and role != "acq":
                out.append(("op", 100, make_meta(R)))
        return out

    programs = [[] for _ in range(T)]
    for t in range(T):
        for ph in range(n_phases):
            n_items = int(rng.integers(1, max(2, budget // (3 * n_phases)) + 1))
            for _ in range(n_items):
                r = rng.random()
                if r < 0.45:
                    programs[t] += section(0, 0)
                elif flags and r < 0.55:
                    programs[t] += flag_op()
                else:
                    programs[t] += data_op()
            if ph + 1 < n_phases:
                programs[t].append(("bar",))
        programs[t] = separate(programs[t])
    # drop the programs of some threads (inactive threads take no barrier either)
    if T > 1 and rng.random() < 0.2:
        programs[int(rng.integers(0, T))] = []

    pc = [0] * T
    holder = {}  # lock id -> list of (thread, scope key)
    arrived = {}  # (block, k) -> arrivals
    bars_done = [0] * T
    active = [len(p) > 0 for p in programs]
    n_active = [sum(active[b * tpb:(b + 1) * tpb]) for b in range(nb)]
    out = []

    def key(t, scope):
        return -1 if scope == DEV else t // tpb

    def overlaps(k1, k2):
        return k1 == -1 or k2 == -1 or k1 == k2

    def runnable(t):
        if pc[t] >= len(programs[t]):
            return False
        op = programs[t][pc[t]]
        if op[0] == "acq":
            k = key(t, op[4])
            for (u, ku) in holder.get(op[3], []):
                if u != t and overlaps(k, ku):
                    return False
        if bars_done[t] > 0:
            b = t // tpb
            if arrived.get((b, bars_done[t]), 0) < n_active[b]:
                return False
        return True

    while True:
        cand = [t for t in range(T) if runnable(t)]
        if not cand:
            break
        t = int(rng.choice(cand))
        op = programs[t][pc[t]]
        pc[t] += 1
        if op[0] == "bar":
            b = t // tpb
            bars_done[t] += 1
            arrived[(b, bars_done[t])] = arrived.get((b, bars_done[t]), 0) + 1
            out.append((0, t, make_meta(BAR), 0))
            continue
        if op[0] == "acq":
            holder.setdefault(op[3], []).append((t, key(t, op[4])))
        if op[0] == "rel":
            holder[op[3]] = [(u, k) for (u, k) in holder.get(op[3], []) if u != t]
        out.append((op[1], t, op[2], 0))
    assert all(pc[t] == len(programs[t]) for t in range(T)), "scheduler stalled"
    ws = int(rng.integers(1, min(tpb, 4) + 1))
    return (nb, tpb, ws), np.array(out, dtype=np.uint32).reshape(-1, 4)
