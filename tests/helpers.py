"""Shared helpers for the tests: seeded workloads, oracle fan-out, device setup."""
from __future__ import annotations

import concurrent.futures as cf
import os

import numpy as np
import pytest

import oracle
from paper_1208_3933_amd import gen

# The pool workloads (n, m, pool size) of the plain bounding configurations.
CONFIG_SHAPES = {0: (20, 5, 4096), 1: (50, 10, 65536), 2: (200, 20, 262144)}


def workload(config: int, n: int, m: int, count: int, instance: int = 0, dmin=0, dmax=None):
    p = gen.processing_times(n, m, gen.make_seed(config, instance, gen.PURPOSE_TIMES))
    pre, dep = gen.random_pool(n, count, gen.make_seed(config, instance, gen.PURPOSE_POOL), dmin, dmax)
    return p, pre, dep


def host_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def oracle_bounds(p, prefixes, depths, threads: int | None = None) -> np.ndarray:
    """Oracle bounds of a pool, fanned out over host threads (each call is the
    plain single-threaded oracle on a slice)."""
    threads = threads or host_threads()
    N = depths.shape[0]
    if N == 0:
        return np.zeros(0, np.int32)
    chunks = np.array_split(np.arange(N), min(threads * 4, N))
    out = np.empty(N, np.int32)
    with cf.ThreadPoolExecutor(threads) as ex:
        futs = {ex.submit(oracle.bound_pool, p, prefixes[c], depths[c]): c for c in chunks if len(c)}
        for f, c in futs.items():
            out[c] = f.result()
    return out


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1208_3933_amd import fspbb
    fspbb.lib()  # raises if the HIP library is missing
    return torch


def to_dev(torch, *arrays):
    return [torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for a in arrays]
