"""Parser for the hand-built traces under tests/golden (see tests/golden/README.txt)."""
from __future__ import annotations

import glob
import os

import numpy as np

from tracegen.format import KIND, SCOPE, SPACE, make_meta

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


class GoldenCase:
    def __init__(self, name, grid, events, expected, header, by_reading=None):
        self.name = name
        self.grid = grid
        self.events = events
        self.expected = expected  # (M, 2) uint32, sorted
        self.header = header
        # pairs expected under another reading of the paper ("inclusive": the other scope rule
        # for atomics and release -> acquire edges; "gwcp": the predictive GWCP relation), when the
        # file states them
        self.by_reading = by_reading or {}

    def __repr__(self):
        return f"GoldenCase({self.name})"


def parse(path: str) -> GoldenCase:
    grid = None
    events = []
    expected = []
    names = {}
    header = []
    none = False
    other = {}  # reading -> list of pairs (an empty list: "none")
    for raw in open(path):
        line = raw.strip()
        if line.startswith("#"):
            header.append(line[1:].strip())
            continue
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "grid":
            grid = tuple(int(x) for x in tok[1:])
            if len(grid) == 2:
                grid = grid + (32,)
        elif tok[0] == "ev":
            kind, scope, space, tid, addr = tok[1:6]
            aux = int(tok[6]) if len(tok) > 6 else 0
            try:
                a = int(addr)
            except ValueError:
                if addr not in names:
                    names[addr] = 100 + len(names)
                a = names[addr]
            events.append((a, int(tid), make_meta(KIND[kind], SCOPE[scope], SPACE[space]), aux))
        elif tok[0] == "expect":
            expected.append((int(tok[1]), int(tok[2])))
        elif tok[0] == "expect-none":
            none = True
        elif tok[0].startswith("expect-"):
            reading = tok[0][len("expect-"):]
            if reading.endswith("-none"):
                other.setdefault(reading[:-len("-none")], [])
            else:
                other.setdefault(reading, []).append((int(tok[1]), int(tok[2])))
        else:
            raise ValueError(f"{path}: bad directive {tok[0]}")
    assert grid is not None, path
    assert none or expected, f"{path}: no expectation"
    exp = np.array(sorted(expected), dtype=np.uint32).reshape(-1, 2)
    ev = np.array(events, dtype=np.uint32).reshape(-1, 4)
    by_reading = {r: np.array(sorted(v), dtype=np.uint32).reshape(-1, 2) for r, v in other.items()}
    return GoldenCase(os.path.basename(path)[:-4], grid, ev, exp, header, by_reading)


def all_cases():
    return [parse(p) for p in sorted(glob.glob(os.path.join(GOLDEN_DIR, "*.txt"))) if not p.endswith("README.txt")]
