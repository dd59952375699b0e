"""Malformed traces made from valid ones, for the validation tests (input generator; no analysis).

``mutate(grid, events, kind, seed)`` returns a copy of a valid trace with one defect of the given
kind and the indices of the records it changed (``None`` for defects that are not record rules):

  record rules    "kind" (kind 8..15), "scope" (scope 3), "reserved" (a meta bit 7..31 set),
                  "tid" (a thread id past the grid), "space" (a fence or a barrier in shared space);
  barrier rules   "runahead" (a thread's next event moved before the other threads of its block
                  have reached the barrier it just passed), "wbar_mask" (a lane bit of a warp
                  barrier's mask flipped), "swap" (two events exchanged; the result may be valid).
"""
from __future__ import annotations

import numpy as np

RECORD_KINDS = ("kind", "scope", "reserved", "tid", "space")
BARRIER_KINDS = ("runahead", "wbar_mask", "swap")


def mutate(grid, events: np.ndarray, kind: str, seed: int):
    rng = np.random.default_rng(seed)
    ev = np.array(events, dtype=np.uint32, copy=True)
    n = ev.shape[0]
    nb, tpb = int(grid[0]), int(grid[1])
    k = ev[:, 2] & 15
    if n == 0:
        return ev, None
    if kind in ("kind", "scope", "reserved", "tid"):
        i = int(rng.integers(0, n))
        if kind == "kind":
            ev[i, 2] = (ev[i, 2] & ~np.uint32(15)) | np.uint32(8 + rng.integers(0, 8))
        elif kind == "scope":
            ev[i, 2] = (ev[i, 2] & ~np.uint32(0x30)) | np.uint32(0x30)
        elif kind == "reserved":
            ev[i, 2] |= np.uint32(1 << int(rng.integers(7, 32)))
        else:
            ev[i, 1] = np.uint32(nb * tpb + int(rng.integers(0, 1000)))
        return ev, [i]
    if kind == "space":
        cand = np.flatnonzero((k == 3) | (k == 4) | (k == 5))
        if len(cand) == 0:
            return ev, []
        i = int(rng.choice(cand))
        ev[i, 2] |= np.uint32(1 << 6)
        return ev, [i]
    if kind == "runahead":
        bars = np.flatnonzero(k == 4)
        rng.shuffle(bars)
        for i in bars:
            t = int(ev[i, 1])
            later = np.flatnonzero(ev[i + 1:, 1] == t)
            if len(later) == 0:
                continue
            j = int(i + 1 + later[0])
            if j == i + 1:
                continue
            row = ev[j].copy()
            ev[i + 2: j + 1] = ev[i + 1: j]
            ev[i + 1] = row
            return ev, None
        return ev, None
    if kind == "wbar_mask":
        w = np.flatnonzero(k == 5)
        if len(w) == 0:
            return ev, None
        i = int(rng.choice(w))
        ws = int(grid[2]) if len(grid) > 2 and grid[2] else 32
        ev[i, 3] ^= np.uint32(1 << int(rng.integers(0, ws)))
        return ev, None
    if kind == "swap":
        a, b = (int(x) for x in rng.integers(0, n, 2))
        ev[[a, b]] = ev[[b, a]]
        return ev, None
    raise ValueError(kind)
