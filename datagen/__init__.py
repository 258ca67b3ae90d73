"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This module draws column values and row IDs only; it holds none of the
scan/lookup method.  The generator is ``gen.c`` (SplitMix64 used as a
counter-based stream, Zipf by inverse CDF or rejection-inversion), loaded
through ctypes and compiled with gcc on first use when no build is present.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libdatagen.so")
_lib = None

SCATTER = 0
SORTED = 1


def build(force: bool = False) -> str:
    """Compile gen.c into libdatagen.so (gcc, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm", "-lpthread"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.dg_zipf_u32.restype = ctypes.c_int
        lib.dg_zipf_u32.argtypes = [
            ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double,
            ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32,
        ]
        lib.dg_uniform_u32.restype = ctypes.c_int
        lib.dg_uniform_u32.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        lib.dg_perm.restype = ctypes.c_uint64
        lib.dg_perm.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64]
        lib.dg_draw_u64.restype = ctypes.c_uint64
        lib.dg_draw_u64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        _lib = lib
    return _lib


def default_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def zipf_column(n: int, w: int, s: float, seed: int, mapping: int = SCATTER,
                threads: int | None = None) -> np.ndarray:
    """n uint32 values: Zipf(s) ranks over 2^w values mapped into [0, 2^w).

    s == 0 gives the uniform distribution.  ``mapping`` SCATTER places rank k at a
    seeded bijection of k-1; SORTED places it at k-1.
    """
    out = np.empty(int(n), dtype=np.uint32)
    rc = _load().dg_zipf_u32(out.ctypes.data, int(n), int(w), float(s), int(seed) & (2**64 - 1),
                             int(mapping), int(threads or default_threads()))
    if rc != 0:
        raise ValueError("dg_zipf_u32 rejected n=%d w=%d s=%g" % (n, w, s))
    return out


def gaussian_column(n: int, w: int, sigma: float, seed: int) -> np.ndarray:
    """n uint32 values: a normal distribution centred in [0, 2^w) with standard
    deviation sigma, rounded to integers and clipped to the domain (numpy's
    seeded PCG64 generator)."""
    rng = np.random.Generator(np.random.PCG64(int(seed) & (2**64 - 1)))
    hi = float((1 << int(w)) - 1)
    x = rng.normal(loc=float(1 << (int(w) - 1)), scale=float(sigma), size=int(n))
    return np.clip(np.rint(x), 0.0, hi).astype(np.uint32)


def uniform_ids(m: int, bound: int, seed: int) -> np.ndarray:
    """m uint32 integers uniform in [0, bound) (row IDs drawn with replacement)."""
    out = np.empty(int(m), dtype=np.uint32)
    if m:
        rc = _load().dg_uniform_u32(out.ctypes.data, int(m), int(bound), int(seed) & (2**64 - 1))
        if rc != 0:
            raise ValueError("dg_uniform_u32 rejected bound=%d" % bound)
    return out


def perm(w: int, seed: int, x: int) -> int:
    """The SCATTER bijection on [0, 2^w) applied to x."""
    return int(_load().dg_perm(int(w), int(seed) & (2**64 - 1), int(x)))


def draw_u64(seed: int, ctr: int) -> int:
    """Draw ``ctr`` of the counter-based stream ``seed``."""
    return int(_load().dg_draw_u64(int(seed) & (2**64 - 1), int(ctr)))


def random_mask_words(n: int, seed: int, density: float = 0.5) -> np.ndarray:
    """A seeded row mask as LSB-first uint64 words (bit r%64 of word r//64), tail bits 0."""
    nw = (n + 63) // 64
    if n == 0:
        return np.zeros(0, dtype=np.uint64)
    thr = int(density * 4294967296.0)
    u = uniform_ids(n, 1 << 32, seed).astype(np.uint64)
    bits = (u < thr).astype(np.uint8)
    pad = np.zeros(nw * 64, dtype=np.uint8)
    pad[:n] = bits
    return np.packbits(pad, bitorder="little").view(np.uint64).copy()
