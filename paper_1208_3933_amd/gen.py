"""Seeded synthetic inputs for the flow-shop bounding path.

This module is shared by the oracle tests and by the GPU path; it holds no
arithmetic of the bound or of branch-and-bound, only random numbers.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), in its counter form: output i of stream
``seed`` is ``mix(seed + (i + 1) * 0x9E3779B97F4A7C15)`` with the published
two-multiply finaliser.  Seeds are ``(config << 40) | (instance << 8) | purpose``
with purpose 0 = processing times, 1 = pool, 2 = arrivals, 3 = pool sizes.

The paper's experiments run on Taillard's benchmark instances (Sec. IV); those
are not used here.  Seeded instances of the same shapes with processing times
drawn i.i.d. uniform on [1, 99] stand in for them (Taillard's own generator
draws from the same range).
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

PURPOSE_TIMES = 0
PURPOSE_POOL = 1
PURPOSE_ARRIVALS = 2
PURPOSE_SIZES = 3


def make_seed(config: int, instance: int, purpose: int) -> int:
    """Stream id for (config, instance, purpose)."""
    return ((int(config) << 40) | (int(instance) << 8) | int(purpose)) & 0xFFFFFFFFFFFFFFFF


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+count-1 of the SplitMix64 stream ``seed`` (uint64)."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed) + i * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def processing_times(n: int, m: int, seed: int, lo: int = 1, hi: int = 99) -> np.ndarray:
    """int32 [n, m] matrix p[j, k], i.i.d. lo + (x mod (hi - lo + 1))."""
    x = splitmix64(seed, n * m)
    span = np.uint64(hi - lo + 1)
    return (np.int64(lo) + (x % span).astype(np.int64)).astype(np.int32).reshape(n, m)


def random_pool(n: int, count: int, seed: int, dmin: int = 0, dmax: int | None = None):
    """A pool of ``count`` sub-problems of an n-job instance.

    Each node is a row of a uniformly random permutation of 0..n-1 (ranked
    random keys) and a depth d uniform on dmin..dmax (default 0..n-1); the
    first d entries of the row are the scheduled prefix, the rest is the
    unscheduled set in arbitrary order.  Returns (prefixes int32 [count, n],
    depths int32 [count]).
    """
    if dmax is None:
        dmax = n - 1
    span = dmax - dmin + 1
    xd = splitmix64(seed, count)
    depths = (np.int64(dmin) + (xd % np.uint64(span)).astype(np.int64)).astype(np.int32)
    rows = []
    chunk = max(1, (1 << 22) // max(n, 1))
    for s in range(0, count, chunk):
        c = min(chunk, count - s)
        keys = splitmix64(seed, c * n, start=count + s * n).reshape(c, n)
        rows.append(np.argsort(keys, axis=1, kind="stable").astype(np.int32))
    prefixes = np.concatenate(rows, axis=0) if rows else np.zeros((0, n), np.int32)
    return np.ascontiguousarray(prefixes), depths


def uniform01(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of the stream."""
    x = splitmix64(seed, count, start)
    return (x >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def lognormal_pool_sizes(count: int, seed: int, median: float = 4096.0, sigma: float = 1.5,
                         lo: int = 256, hi: int = 131072) -> np.ndarray:
    """Pool sizes clamp(round(median * exp(sigma * z)), lo, hi) with z ~ N(0,1) (Box-Muller)."""
    u = uniform01(seed, 2 * count)
    u1 = np.maximum(u[0::2], 1e-300)
    u2 = u[1::2]
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return np.clip(np.rint(median * np.exp(sigma * z)), lo, hi).astype(np.int64)
