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


def batch(seed: int = 4, n_traces: int = 512, scale: int = 1, median: int = 204_800,
          lo: int = 10_240, hi: int = 4_194_304):
    """Many independent traces of uneven length with the event mix of ``large``: lengths
    lognormal(ln median, 1.0) clipped to [lo, hi], 2^U{6..11} blocks of 128 or 256 threads, words
    at the density of ``large`` (one per 16 events, 80% global, 20% spread over the blocks' shared
    spaces).  Trace i draws from (seed, i).  ``scale`` > 1 divides lengths and block counts (tests).
    Returns a list of MixConfig."""
    rng = np.random.default_rng([seed, 0x5eed])
    out = []
    for i in range(n_traces):
        n = int(np.clip(np.exp(rng.normal(np.log(median), 1.0)), lo, hi)) // scale
        nb = max(1, (1 << int(rng.integers(6, 12))) // scale)
        tpb = 128 if rng.random() < 0.5 else 256
        n = max(n, 64)
        words = max(64, n // 16)
        n_global = max(16, (words * 4) // 5)
        n_shared = max(1, (words - n_global) // nb)
        out.append(MixConfig(n_blocks=nb, tpb=tpb, n_events=n, n_global=n_global, n_shared=n_shared,
                             zipf_s=1.1, p_write=0.30, p_atomic_block=0.01, p_atomic_device=0.01,
                             bar_period=64, fence_period=512, plant_rate=1e-4, p_plant_same_block=0.5,
                             plant_victim_cap=256, frac_ro=0.3, frac_da=0.05, frac_priv=0.7, frac_pro=0.25,
                             p_read_ro=0.3, seed=seed, trace_index=i))
    return out


# ---------------------------------------------------------------- halo-exchange stencil

_STENCIL_SRC = os.path.join(_HERE, "stencil.c")
_STENCIL_LIB = os.path.join(_HERE, "libstencil.so")


class _StencilCfg(ctypes.Structure):
    _fields_ = [("rb", ctypes.c_uint32), ("cb", ctypes.c_uint32), ("tpb", ctypes.c_uint32),
                ("warp_size", ctypes.c_uint32), ("rows", ctypes.c_uint32), ("sweeps", ctypes.c_uint32),
                ("pitch", ctypes.c_uint32), ("group", ctypes.c_uint32), ("plant_rate", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class _StencilStats(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_uint64), ("n_fence_plants", ctypes.c_uint64),
                ("n_lock_plants", ctypes.c_uint64), ("buf0", ctypes.c_uint32), ("buf1", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("acc", ctypes.c_uint32), ("lock", ctypes.c_uint32)]


@dataclasses.dataclass
class StencilConfig:
    rb: int
    cb: int
    tpb: int
    rows: int
    sweeps: int
    pitch: int
    group: int = 64
    plant_rate: float = 0.0
    warp_size: int = 32
    seed: int = 3

    @property
    def grid(self):
        return (self.rb * self.cb, self.tpb, self.warp_size)


def build_stencil(force: bool = True) -> str:
    if force or not os.path.exists(_STENCIL_LIB):
        tmp = _STENCIL_LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, _STENCIL_SRC])
        os.replace(tmp, _STENCIL_LIB)
    return _STENCIL_LIB


_slib = None


def _load_stencil():
    global _slib
    if _slib is None:
        if not os.path.exists(_STENCIL_LIB):
            build_stencil(force=False)
        lib = ctypes.CDLL(_STENCIL_LIB)
        lib.tg_stencil.argtypes = [ctypes.POINTER(_StencilCfg), ctypes.c_void_p, ctypes.c_uint64,
                                   ctypes.POINTER(_StencilStats), ctypes.c_void_p, ctypes.c_uint64]
        lib.tg_stencil.restype = ctypes.c_int
        _slib = lib
    return _slib


def generate_stencil(cfg: StencilConfig, max_plants: int = 1 << 16):
    """Returns (grid, events (N,4) uint32, stats dict, plants (k,4) uint32: kind 0 = fence pair
    (block, sweep, direction of the acquire), kind 1 = lock pair (block, section index, 0))."""
    lib = _load_stencil()
    c = _StencilCfg(cfg.rb, cfg.cb, cfg.tpb, cfg.warp_size, cfg.rows, cfg.sweeps, cfg.pitch, cfg.group,
                    cfg.plant_rate, cfg.seed)
    st = _StencilStats()
    if lib.tg_stencil(ctypes.byref(c), None, 0, ctypes.byref(st), None, 0) != 0:
        raise RuntimeError(f"bad stencil configuration {cfg}")
    n = int(st.n_events)
    out = np.empty((n, 4), dtype=np.uint32)
    plants = np.zeros((max_plants, 4), dtype=np.uint32)
    if lib.tg_stencil(ctypes.byref(c), out.ctypes.data, n, ctypes.byref(st), plants.ctypes.data, max_plants) != 0:
        raise RuntimeError("stencil generation failed")
    stats = {f: int(getattr(st, f)) for f, _ in _StencilStats._fields_}
    k = min(max_plants, stats["n_fence_plants"] + stats["n_lock_plants"])
    return cfg.grid, out, stats, plants[:k].copy()


def stencil(seed: int = 3) -> StencilConfig:
    """4096 blocks (64 x 64) x 256 threads, 5 rows per block, 8 Jacobi sweeps of a 5-point stencil
    over two 320 x 16,384 buffers with rows 104,857 words apart (about 64M words of address span),
    halo flags published by fence + atomic and taken by atomic + fence, a device lock around a
    global accumulator, 0.1% of fences and lock operations downgraded to block scope in pairs."""
    return StencilConfig(rb=64, cb=64, tpb=256, rows=5, sweeps=8, pitch=104_857, group=64, plant_rate=1e-3,
                         seed=seed)


def stencil_small(seed: int = 3, rb: int = 4, cb: int = 4, tpb: int = 32, rows: int = 3, sweeps: int = 4,
                  plant_rate: float = 0.05) -> StencilConfig:
    """The same kernel shape at test size."""
    return StencilConfig(rb=rb, cb=cb, tpb=tpb, rows=rows, sweeps=sweeps, pitch=cb * tpb + 7, group=4,
                         plant_rate=plant_rate, seed=seed)
