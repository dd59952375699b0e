"""Seeded synthetic GPU event traces (inputs for the checker and for the oracle; no analysis).

``generate(cfg)`` calls the C generator (``tracegen.c``) for the "mix" workloads; the shapes below
stand in for the paper's applications, which are not available: the paper measures on benchmark
programs (Section 6.1), and these synthetic traces reproduce the thread grid, event count, word
footprint, access mix, barrier/fence periods and reuse distribution of each workload.

``random_trace`` (randtrace.py) builds tiny valid traces with every event kind for property tests.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libtracegen.so")
_SRC = os.path.join(_HERE, "tracegen.c")


@dataclasses.dataclass
class MixConfig:
    n_blocks: int
    tpb: int
    n_events: int
    n_global: int
    n_shared: int = 0
    warp_size: int = 32
    zipf_s: float = 0.0
    p_write: float = 0.3
    p_atomic_block: float = 0.01
    p_atomic_device: float = 0.01
    bar_period: int = 0
    fence_period: int = 0
    plant_rate: float = 0.0
    plant_count: int = 0
    plant_ww: int = 0
    p_plant_same_block: float = 0.5
    plant_victim_cap: int = 256
    frac_ro: float = 0.3
    frac_da: float = 0.05
    frac_priv: float = 0.7
    frac_pro: float = 0.25
    p_read_ro: float = 0.3
    addr_base: int = 0
    seed: int = 0
    trace_index: int = 0

    @property
    def grid(self):
        return (self.n_blocks, self.tpb, self.warp_size)


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("n_blocks", ctypes.c_uint32), ("tpb", ctypes.c_uint32), ("warp_size", ctypes.c_uint32),
        ("n_global", ctypes.c_uint32), ("n_shared", ctypes.c_uint32), ("n_events", ctypes.c_uint64),
        ("zipf_s", ctypes.c_double), ("p_write", ctypes.c_double), ("p_atomic_block", ctypes.c_double),
        ("p_atomic_device", ctypes.c_double), ("bar_period", ctypes.c_uint32),
        ("fence_period", ctypes.c_uint32), ("plant_rate", ctypes.c_double),
        ("plant_count", ctypes.c_uint32), ("plant_ww", ctypes.c_uint32),
        ("p_plant_same_block", ctypes.c_double), ("plant_victim_cap", ctypes.c_uint32),
        ("frac_ro", ctypes.c_double), ("frac_da", ctypes.c_double), ("frac_priv", ctypes.c_double),
        ("frac_pro", ctypes.c_double), ("p_read_ro", ctypes.c_double), ("addr_base", ctypes.c_uint32),
        ("seed", ctypes.c_uint64), ("trace_index", ctypes.c_uint64),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("n_planted", "n_degraded", "n_bar", "n_fence", "n_write", "n_read", "n_atomic")]


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.tg_generate.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_void_p, ctypes.POINTER(_Stats),
                                    ctypes.c_void_p, ctypes.c_uint64]
        lib.tg_generate.restype = ctypes.c_int
        _lib = lib
    return _lib


def generate(cfg: MixConfig, max_plants: int = 1 << 20):
    """Returns (grid, events (N,4) uint32, stats dict, plant event indices)."""
    lib = _load()
    c = _Cfg(**{f.name: getattr(cfg, f.name) for f in dataclasses.fields(cfg)})
    out = np.empty((cfg.n_events, 4), dtype=np.uint32)
    st = _Stats()
    plants = np.zeros(max_plants, dtype=np.uint64)
    rc = lib.tg_generate(ctypes.byref(c), out.ctypes.data, ctypes.byref(st), plants.ctypes.data, max_plants)
    if rc != 0:
        raise RuntimeError(f"trace generation failed ({rc}) for {cfg}")
    stats = {n: int(getattr(st, n)) for n, _ in _Stats._fields_}
    return cfg.grid, out, stats, plants[: min(stats["n_planted"], max_plants)].copy()


# ---------------------------------------------------------------- named workloads
# "K" and "M" are binary (2^10, 2^20).

def tiny(seed: int = 1) -> MixConfig:
    """2 blocks x 64 threads, 4,096 events, 256 global words chosen uniformly, 25% writes,
    1% block-scope atomicAdd, a block barrier every 32 events per thread, 3 planted unordered
    write-write races across blocks."""
    return MixConfig(n_blocks=2, tpb=64, n_events=4096, n_global=256, n_shared=0, zipf_s=0.0,
                     p_write=0.25, p_atomic_block=0.01, p_atomic_device=0.0, bar_period=32,
                     fence_period=0, plant_count=3, plant_ww=1, frac_ro=0.1, frac_da=0.0,
                     frac_priv=0.8, frac_pro=0.15, p_read_ro=0.2, plant_victim_cap=0, seed=seed)


def large(seed: int = 2, scale: int = 1) -> MixConfig:
    """1024 blocks x 256 threads, 16M events, 1M words (80% global, 20% per-block shared),
    Zipf(1.1) reuse, 30% writes, 2% atomics (half block, half device scope), device fences every
    512 and barriers every 64 events per thread, plants with probability 1e-4 per event.
    ``scale`` > 1 shrinks blocks, events and words by that factor (for fast tests)."""
    nb = max(1, 1024 // scale)
    return MixConfig(n_blocks=nb, tpb=256, n_events=(16 << 20) // scale,
                     n_global=838_861 // scale, n_shared=205, zipf_s=1.1, p_write=0.30,
                     p_atomic_block=0.01, p_atomic_device=0.01, bar_period=64, fence_period=512,
                     plant_rate=1e-4, p_plant_same_block=0.5, plant_victim_cap=256,
                     frac_ro=0.3, frac_da=0.05, frac_priv=0.7, frac_pro=0.25, p_read_ro=0.3, seed=seed)


from .randtrace import random_trace  # noqa: E402,F401
