"""Seeded synthetic DNA inputs (stand-ins for the paper's genome datasets).

This module holds no arithmetic of the compression method. It draws ASCII
bases from seeded Markov sources, plants repeats and N runs, and returns
plain bytes. The oracle tests, the GPU tests and the bench all take their
inputs from here, so both sides see identical data.

The sequential sampling runs in a small C helper (``gen.c``), which is
compiled on first use with gcc. Dirichlet rows come from NumPy's
``default_rng(seed).dirichlet``.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C sampler (gcc -O2 -shared)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.synth_markov.argtypes = [u8p, ctypes.c_uint64, ctypes.c_int, dp, dp, ctypes.c_uint64, ctypes.c_uint64]
        lib.synth_markov.restype = None
        lib.synth_repeats.argtypes = [u8p, ctypes.c_uint64, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.c_double, ctypes.c_uint64]
        lib.synth_repeats.restype = ctypes.c_uint64
        lib.synth_nruns.argtypes = [u8p, ctypes.c_uint64, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64]
        lib.synth_nruns.restype = ctypes.c_uint64
        _lib = lib
    return _lib


@dataclass
class Recipe:
    """One synthetic source. Sizes are in bases (bytes of ASCII)."""
    n: int
    order: int = 3
    seed: int = 1
    rho: float = 0.0            # fraction covered by planted repeats
    rep_len: tuple = (50, 500)
    p_revcomp: float = 0.0      # share of repeats that are reverse-complemented
    gc: tuple | None = None     # (lo, hi): GC content drawn per segment
    gc_seg: int = 1 << 20
    n_rate: float = 0.0         # fraction of bases that are N (expected)
    n_max: int = 100
    meta: dict = field(default_factory=dict)


def generate(r: Recipe) -> np.ndarray:
    """Return a uint8 array of ASCII bases following recipe ``r``."""
    lib = _load()
    rng = np.random.default_rng(r.seed)
    rows = np.ascontiguousarray(rng.dirichlet([0.5] * 4, size=4 ** r.order).astype(np.float64))
    gc = None
    if r.gc is not None:
        nseg = max(1, (r.n + r.gc_seg - 1) // r.gc_seg)
        gc = np.ascontiguousarray(rng.uniform(r.gc[0], r.gc[1], size=nseg).astype(np.float64))
    out = np.empty(r.n, dtype=np.uint8)
    if r.n == 0:
        return out
    u8p = out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    dp = ctypes.POINTER(ctypes.c_double)
    lib.synth_markov(u8p, r.n, r.order, rows.ctypes.data_as(dp),
                     gc.ctypes.data_as(dp) if gc is not None else None, r.gc_seg, r.seed)
    if r.rho > 0:
        lib.synth_repeats(u8p, r.n, r.rho, r.rep_len[0], r.rep_len[1], r.p_revcomp, r.seed)
    if r.n_rate > 0:
        lib.synth_nruns(u8p, r.n, r.n_rate, r.n_max, r.seed)
    return out


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(memoryview(np.ascontiguousarray(a))).hexdigest()


MiB = 1 << 20


def recipe_cfg1(seed: int = 1, n: int = 1 << 18) -> Recipe:
    """256 KiB, order-3 Markov, 5% exact repeats of length 50-500."""
    return Recipe(n=n, order=3, seed=seed, rho=0.05)


def recipe_cfg2(seed: int = 2, n: int = 1 << 26) -> Recipe:
    """64 MiB, order-5, GC 0.35-0.65 per 1 MiB segment, 10% repeats (half
    reverse-complement), rare N runs (0.01% of bases, length 1-100)."""
    return Recipe(n=n, order=5, seed=seed, rho=0.10, p_revcomp=0.5, gc=(0.35, 0.65),
                  gc_seg=MiB, n_rate=1e-4, n_max=100)


def recipe_cfg2_static(seed: int = 102, n: int = 1 << 20) -> Recipe:
    """Separate sequence (same recipe, its own seed) on which the frozen
    static model is pre-trained."""
    return recipe_cfg2(seed=seed, n=n)


def lognormal_blocks(total: int, n_blocks: int, median: int, sigma: float, seed: int) -> list[int]:
    """Block lengths: lognormal(ln median, sigma) draws rescaled to sum to
    ``total`` (largest-remainder rounding)."""
    rng = np.random.default_rng(seed)
    x = rng.lognormal(np.log(median), sigma, size=n_blocks)
    share = x / x.sum() * total
    base = np.floor(share).astype(np.int64)
    rem = int(total - base.sum())
    order = np.argsort(-(share - base), kind="stable")
    base[order[:rem]] += 1
    return [int(v) for v in base]


def archive_files(n_files: int = 64, lo: int = 1 << 10, hi: int = 1 << 29, seed: int = 5000,
                  scale: float = 1.0) -> list[Recipe]:
    """Mixed archive: file sizes log-uniform in [lo, hi] bytes, per-file
    order 2..8, GC 0.3-0.7, repeat density 0-30%, N runs."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(lo), np.log(hi), size=n_files))
    out = []
    for f in range(n_files):
        fr = np.random.default_rng(seed + f + 1)
        n = max(1, int(sizes[f] * scale))
        g = float(fr.uniform(0.3, 0.7))
        out.append(Recipe(n=n, order=int(fr.integers(2, 9)), seed=seed + f, rho=float(fr.uniform(0.0, 0.3)),
                          p_revcomp=0.5, gc=(g, g), gc_seg=max(n, 1), n_rate=1e-4, n_max=100))
    return out
