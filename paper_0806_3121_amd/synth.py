"""Seeded synthetic inputs.

This module only draws random numbers; it holds none of the checksum
arithmetic.  Both the CPU oracle's tests and the GPU path take their inputs
from here, so that the two sides are compared on identical data.

Generator: splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used counter-based.  Element ``idx`` of
stream ``s`` under seed ``S`` is ``mix64(key + (idx + 1) * GAMMA)`` with
``key = mix64(S * 256 + s)``: the (idx+1)-th output of a sequential
splitmix64 generator started from ``key``.  The uniform maps use integer
operations and one exact scaling, so a GPU implementation of the same
definition produces identical bits.

Streams: 0 = A, 1 = B, 2 = flip positions and bits, 3 = erasure positions,
4 = batched shapes, 5 = residual vector, 6 = outlier mask, 7 = campaign picks.
The workloads are the paper's random dense matrices (Sec. 4.3, the weak-scaling
runs), drawn uniform on [-1, 1).
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
MASK64 = (1 << 64) - 1

BASE_SEED = 20080523  # the paper's date, used as the default base seed

STREAM_A, STREAM_B, STREAM_FLIP, STREAM_ERASE, STREAM_SHAPES, STREAM_X, STREAM_OUTLIER, STREAM_PICK = range(8)


def mix64_int(z: int) -> int:
    """splitmix64 finaliser on a Python int (mod 2**64)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def stream_key(seed: int, stream: int) -> int:
    return mix64_int(((seed & MASK64) * 256 + stream) & MASK64)


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def raw_u64(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """64-bit outputs at counter positions ``idx`` (any integer array)."""
    key = np.uint64(stream_key(seed, stream))
    with np.errstate(over="ignore"):
        z = key + (np.asarray(idx, dtype=np.uint64) + np.uint64(1)) * GAMMA
        return _mix64_np(z)


def u64_to_f64(x: np.ndarray) -> np.ndarray:
    """uniform on [-1, 1): 2 * ((x >> 11) * 2^-53) - 1, exact in binary64."""
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -52) - 1.0


def u64_to_f32(x: np.ndarray) -> np.ndarray:
    """uniform on [-1, 1): 2 * ((x >> 40) * 2^-24) - 1, exact in binary32."""
    return ((x >> np.uint64(40)).astype(np.float64) * (2.0 ** -23) - 1.0).astype(np.float32)


def _chunked(total: int, fn, out: np.ndarray, chunk: int = 1 << 24) -> np.ndarray:
    flat = out.reshape(-1)
    for s in range(0, total, chunk):
        e = min(total, s + chunk)
        flat[s:e] = fn(np.arange(s, e, dtype=np.uint64))
    return out


def uniform(seed: int, stream: int, rows: int, cols: int, dtype=np.float64) -> np.ndarray:
    """rows x cols row-major matrix; element (i, j) uses counter i*cols + j."""
    dtype = np.dtype(dtype)
    out = np.empty((rows, cols), dtype=dtype)
    conv = u64_to_f64 if dtype == np.float64 else u64_to_f32
    if dtype not in (np.dtype(np.float64), np.dtype(np.float32)):
        raise ValueError("uniform: float64 or float32 only")
    return _chunked(rows * cols, lambda ix: conv(raw_u64(seed, stream, ix)), out)


def uniform_rows(seed: int, stream: int, row_ids, cols: int, dtype=np.float64) -> np.ndarray:
    """Selected rows of the matrix ``uniform(seed, stream, ?, cols)``."""
    row_ids = np.asarray(row_ids, dtype=np.uint64)
    idx = row_ids[:, None] * np.uint64(cols) + np.arange(cols, dtype=np.uint64)[None, :]
    conv = u64_to_f64 if np.dtype(dtype) == np.float64 else u64_to_f32
    return conv(raw_u64(seed, stream, idx))


def uniform_ints(seed: int, stream: int, rows: int, cols: int, lo: int, hi: int) -> np.ndarray:
    """Integer-valued float64 matrix with entries in [lo, hi] (for exact-arithmetic cases)."""
    span = hi - lo + 1
    x = raw_u64(seed, stream, np.arange(rows * cols, dtype=np.uint64)).reshape(rows, cols)
    return (x % np.uint64(span)).astype(np.int64).astype(np.float64) + lo


def randint(seed: int, stream: int, idx: int, n: int) -> int:
    """One integer uniform on [0, n) from counter ``idx`` (modulo draw; n << 2^64)."""
    return int(raw_u64(seed, stream, np.array([idx]))[0]) % n


def normal_with_outliers(seed: int, rows: int, cols: int, frac: float = 0.01, scale: float = 1e3) -> np.ndarray:
    """N(0,1) by Box-Muller (float64, then rounded to float32); each entry is
    multiplied by fl32(scale) with probability ``frac`` (Bernoulli on the
    outlier stream).  Host-only: it needs libm."""
    n = rows * cols
    out = np.empty(n, dtype=np.float32)
    chunk = 1 << 23
    s32 = np.float32(scale)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        ix = np.arange(s, e, dtype=np.uint64)
        u1 = ((raw_u64(seed, STREAM_A, ix) >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
        u2 = (raw_u64(seed, STREAM_B, ix) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
        z32 = z.astype(np.float32)
        pick = (raw_u64(seed, STREAM_OUTLIER, ix) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 < frac
        z32[pick] = z32[pick] * s32
        out[s:e] = z32
    return out.reshape(rows, cols)


def flip_site(seed: int, run: int, rows: int, cols: int, bit_lo: int, bit_hi: int,
              avoid=None):
    """(i, j, bit) for run ``run``: i < rows, j < cols, bit in [bit_lo, bit_hi].
    ``avoid`` = (i0, j0, h, w) rectangle the site must lie outside of."""
    t = 0
    while True:
        base = (run * 64 + t) * 3
        i = randint(seed, STREAM_FLIP, base, rows)
        j = randint(seed, STREAM_FLIP, base + 1, cols)
        b = bit_lo + randint(seed, STREAM_FLIP, base + 2, bit_hi - bit_lo + 1)
        t += 1
        if avoid is not None:
            i0, j0, h, w = avoid
            if i0 <= i < i0 + h and j0 <= j < j0 + w:
                continue
        return i, j, b


def erase_block(seed: int, run: int, grid_rows: int, grid_cols: int):
    """Block coordinates (I, J) on a grid_rows x grid_cols block grid."""
    return (randint(seed, STREAM_ERASE, 2 * run, grid_rows),
            randint(seed, STREAM_ERASE, 2 * run + 1, grid_cols))


def batched_shapes(seed: int, count: int, lo: int = 64, hi: int = 2048, step: int = 32):
    """count triples (m, n, k), each uniform on {lo, lo+step, ..., hi}."""
    nvals = (hi - lo) // step + 1
    out = []
    for p in range(count):
        m = lo + step * randint(seed, STREAM_SHAPES, 3 * p, nvals)
        n = lo + step * randint(seed, STREAM_SHAPES, 3 * p + 1, nvals)
        k = lo + step * randint(seed, STREAM_SHAPES, 3 * p + 2, nvals)
        out.append((m, n, k))
    return out


def pick_distinct(seed: int, count: int, n_total: int, stream: int = STREAM_PICK):
    """``count`` distinct indices in [0, n_total), drawn without replacement."""
    chosen = []
    t = 0
    while len(chosen) < count:
        v = randint(seed, stream, t, n_total)
        t += 1
        if v not in chosen:
            chosen.append(v)
    return chosen
